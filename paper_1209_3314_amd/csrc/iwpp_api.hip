// Host side of the C ABI declared in include/iwpp.h: context, argument
// checks, scratch management and launch sequencing.  No exception or C++ type
// crosses the ABI; every entry point returns an iwpp_status code.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/iwpp.h"
#include "iwpp_device.hpp"
#include "iwpp_internal.hpp"

struct iwpp_ctx {
  int device = 0;
  iwpp_options opt{};
  std::string err;
  // fixed area: barrier | counts | lost | ovf | stats
  uint8_t* fixed = nullptr;
  // growable scratch
  uint8_t* scratch = nullptr;
  size_t scratch_bytes = 0;
  hipStream_t last_stream = nullptr;
  int last_op = 0;
  bool have_call = false;
  iwpp::Recorder rec;
};

namespace iwpp {

void Recorder::begin(int kernel, hipStream_t s) {
  open_ = false;
  if (!enabled || count_ >= kCap) return;
  if (count_ >= created_) {
    if (hipEventCreate(&start_[count_]) != hipSuccess) return;
    if (hipEventCreate(&stop_[count_]) != hipSuccess) {
      (void)hipEventDestroy(start_[count_]);
      return;
    }
    created_ = count_ + 1;
  }
  if (hipEventRecord(start_[count_], s) != hipSuccess) return;
  kernel_[count_] = kernel;
  open_ = true;
}

void Recorder::end(hipStream_t s) {
  if (!open_) return;
  open_ = false;
  if (hipEventRecord(stop_[count_], s) == hipSuccess) count_++;
}

int Recorder::read(int* kernels, float* ms, int max) {
  int n = 0;
  for (int i = 0; i < count_ && n < max; ++i) {
    float t = 0.f;
    if (hipEventSynchronize(stop_[i]) != hipSuccess || hipEventElapsedTime(&t, start_[i], stop_[i]) != hipSuccess) {
      (void)hipGetLastError();
      t = -1.f;
    }
    kernels[n] = kernel_[i];
    ms[n] = t;
    n++;
  }
  count_ = 0;
  return n;
}

void Recorder::release() {
  for (int i = 0; i < created_; ++i) {
    (void)hipEventDestroy(start_[i]);
    (void)hipEventDestroy(stop_[i]);
  }
  created_ = 0;
  count_ = 0;
}

}  // namespace iwpp

namespace {

thread_local std::string g_create_err;

constexpr size_t kOffBarrier = 0;
constexpr size_t kOffCounts = kOffBarrier + iwpp::kBarrierBytes;
constexpr size_t kOffLost = kOffCounts + iwpp::kCountsBytes;
constexpr size_t kOffOvf = kOffLost + iwpp::kLostBytes;
constexpr size_t kOffStats = kOffOvf + 256;
constexpr size_t kFixedBytes = kOffStats + iwpp::kStatsBytes;
static_assert(sizeof(iwpp::GridBarrier) <= iwpp::kBarrierBytes, "barrier area too small");
static_assert(kOffStats % 8 == 0, "stats must be 8-byte aligned");

int32_t fail(iwpp_ctx* ctx, int32_t code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

// Makes `dev` current for the duration of a call and restores the caller's device.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) return;
    if (prev != dev && hipSetDevice(dev) != hipSuccess) return;
    ok = true;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb && y < x + na;
}

int32_t ensure_scratch(iwpp_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->scratch_bytes) return IWPP_OK;
  if (ctx->scratch) {
    // The previous call may still be using the old buffer.
    if (hipDeviceSynchronize() != hipSuccess) return fail(ctx, IWPP_EDEVICE, "device error while growing scratch");
    (void)hipFree(ctx->scratch);
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
  }
  size_t want = bytes + bytes / 8;  // headroom against small growth steps
  void* p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, IWPP_ENOMEM, "scratch allocation of " + std::to_string(want) + " bytes failed");
  }
  ctx->scratch = static_cast<uint8_t*>(p);
  ctx->scratch_bytes = want;
  return IWPP_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Clear list fill levels, lost flags and the barrier before a launch group,
// and the statistics too at the start of a call.
int32_t reset_fixed(iwpp_ctx* ctx, hipStream_t stream, bool stats) {
  ctx->rec.begin(IWPP_K_RESET, stream);
  const int r = iwpp::zero_words(reinterpret_cast<uint32_t*>(ctx->fixed), (stats ? kFixedBytes : kOffStats) / 4, stream);
  ctx->rec.end(stream);
  if (r != 0) return fail(ctx, IWPP_EDEVICE, "reset kernel launch failed");
  return IWPP_OK;
}

void bind_fixed_mr(iwpp_ctx* ctx, iwpp::MrArgs& a) {
  a.counts = reinterpret_cast<uint32_t*>(ctx->fixed + kOffCounts);
  a.lost = reinterpret_cast<uint32_t*>(ctx->fixed + kOffLost);
  a.bar = reinterpret_cast<iwpp::GridBarrier*>(ctx->fixed + kOffBarrier);
  a.stats = reinterpret_cast<unsigned long long*>(ctx->fixed + kOffStats);
}

void bind_fixed_edt(iwpp_ctx* ctx, iwpp::EdtArgs& a) {
  a.counts = reinterpret_cast<uint32_t*>(ctx->fixed + kOffCounts);
  a.ovf = reinterpret_cast<uint32_t*>(ctx->fixed + kOffOvf);
  a.bar = reinterpret_cast<iwpp::GridBarrier*>(ctx->fixed + kOffBarrier);
  a.stats = reinterpret_cast<unsigned long long*>(ctx->fixed + kOffStats);
}

// Scratch bytes of one reconstruction launch over `ntiles` tiles / `njobs` images.
size_t mr_scratch_bytes(uint64_t ntiles, uint32_t njobs) {
  return 5 * align256(ntiles * 4) + align256((size_t)njobs * sizeof(iwpp::MrJob));
}

// Scratch bytes of one distance-transform launch over `npix` pixels / `njobs` images.
size_t edt_scratch_bytes(uint64_t npix, uint32_t njobs) {
  return 4 * align256(npix * 8) + align256(npix * 4) + align256((size_t)njobs * sizeof(iwpp::EdtJob));
}

// Launch one reconstruction group (jobs already validated; tile_base filled).
int32_t run_mr(iwpp_ctx* ctx, const std::vector<iwpp::MrJob>& jobs, uint32_t ntiles, int conn, hipStream_t st,
               bool first) {
  iwpp::MrArgs a{};
  const uint32_t nj = (uint32_t)jobs.size();
  a.job0 = jobs[0];
  a.njobs = nj;
  a.ntiles = ntiles;
  const int64_t cap = ctx->opt.mr_list_capacity;
  a.list_cap = (cap > 0 && (uint64_t)cap < ntiles) ? (uint32_t)cap : ntiles;
  a.max_sweeps = ctx->opt.mr_max_sweeps > 0 ? ctx->opt.mr_max_sweeps : 64;
  a.seed_sweeps = a.max_sweeps;
  const size_t tb = align256((size_t)ntiles * 4);
  int32_t rc = ensure_scratch(ctx, mr_scratch_bytes(ntiles, nj));
  if (rc != IWPP_OK) return rc;
  // layout: flags[2][T] | lists[2][T] | tile_job[T] | job table
  a.flags = reinterpret_cast<uint32_t*>(ctx->scratch);
  a.lists = reinterpret_cast<uint32_t*>(ctx->scratch + 2 * tb);
  a.tile_job = nullptr;
  a.jobs = nullptr;
  if (nj > 1) {
    iwpp::MrJob* dj = reinterpret_cast<iwpp::MrJob*>(ctx->scratch + 5 * tb);
    a.tile_job = reinterpret_cast<uint32_t*>(ctx->scratch + 4 * tb);
    a.jobs = dj;
    if (hipMemcpyAsync(dj, jobs.data(), nj * sizeof(iwpp::MrJob), hipMemcpyHostToDevice, st) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, IWPP_EDEVICE, "job table upload failed");
    }
  }
  bind_fixed_mr(ctx, a);
  if ((rc = reset_fixed(ctx, st, first)) != IWPP_OK) return rc;
  const char* e = "";
  if (iwpp::mr_launch(a, conn, ctx->opt.persistent_blocks, st, &ctx->rec, &e) != 0) {
    (void)hipGetLastError();
    return fail(ctx, IWPP_EDEVICE, std::string("morph_recon: ") + e);
  }
  return IWPP_OK;
}

int32_t run_edt(iwpp_ctx* ctx, const std::vector<iwpp::EdtJob>& jobs, uint64_t npix, int conn, hipStream_t st,
                bool first) {
  iwpp::EdtArgs a{};
  const uint32_t nj = (uint32_t)jobs.size();
  a.job0 = jobs[0];
  a.njobs = nj;
  a.npix = (uint32_t)npix;
  const size_t kb = align256((size_t)npix * 8);
  int32_t rc = ensure_scratch(ctx, edt_scratch_bytes(npix, nj));
  if (rc != IWPP_OK) return rc;
  a.key0 = reinterpret_cast<unsigned long long*>(ctx->scratch);
  a.key1 = reinterpret_cast<unsigned long long*>(ctx->scratch + kb);
  a.lists = reinterpret_cast<unsigned long long*>(ctx->scratch + 2 * kb);
  a.stamp = reinterpret_cast<uint32_t*>(ctx->scratch + 4 * kb);
  a.jobs = nullptr;
  if (nj > 1) {
    iwpp::EdtJob* dj = reinterpret_cast<iwpp::EdtJob*>(ctx->scratch + 4 * kb + align256((size_t)npix * 4));
    a.jobs = dj;
    if (hipMemcpyAsync(dj, jobs.data(), nj * sizeof(iwpp::EdtJob), hipMemcpyHostToDevice, st) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, IWPP_EDEVICE, "job table upload failed");
    }
  }
  bind_fixed_edt(ctx, a);
  if ((rc = reset_fixed(ctx, st, first)) != IWPP_OK) return rc;
  const char* e = "";
  if (iwpp::edt_launch(a, conn, ctx->opt.persistent_blocks, st, &ctx->rec, &e) != 0) {
    (void)hipGetLastError();
    return fail(ctx, IWPP_EDEVICE, std::string("edt: ") + e);
  }
  return IWPP_OK;
}

}  // namespace

extern "C" {

int32_t iwpp_version(void) { return (0 << 16) | 1; }

int32_t iwpp_create(int32_t device, const iwpp_options* opt, iwpp_ctx** out) {
  if (!out) {
    g_create_err = "iwpp_create: out is NULL";
    return IWPP_EINVAL;
  }
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    g_create_err = "iwpp_create: no HIP device " + std::to_string(device);
    return IWPP_EINVAL;
  }
  iwpp_ctx* ctx = new (std::nothrow) iwpp_ctx();
  if (!ctx) {
    g_create_err = "iwpp_create: out of host memory";
    return IWPP_ENOMEM;
  }
  ctx->device = device;
  if (opt) ctx->opt = *opt;
  ctx->rec.enabled = ctx->opt.profile != 0;
  DeviceGuard g(device);
  void* p = nullptr;
  if (!g.ok || hipMalloc(&p, kFixedBytes) != hipSuccess) {
    (void)hipGetLastError();
    delete ctx;
    g_create_err = "iwpp_create: device allocation failed";
    return IWPP_EDEVICE;
  }
  ctx->fixed = static_cast<uint8_t*>(p);
  if (hipMemset(ctx->fixed, 0, kFixedBytes) != hipSuccess) {
    (void)hipFree(p);
    delete ctx;
    g_create_err = "iwpp_create: device memset failed";
    return IWPP_EDEVICE;
  }
  *out = ctx;
  return IWPP_OK;
}

void iwpp_destroy(iwpp_ctx* ctx) {
  if (!ctx) return;
  {
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->rec.release();
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->fixed) (void)hipFree(ctx->fixed);
  }
  delete ctx;
}

const char* iwpp_last_error(const iwpp_ctx* ctx) {
  if (!ctx) return g_create_err.c_str();
  return ctx->err.c_str();
}

int32_t iwpp_morph_recon_u8(iwpp_ctx* ctx, const uint8_t* marker, const uint8_t* mask, uint8_t* out, int32_t height,
                            int32_t width, int32_t conn, void* stream) {
  if (!ctx) return IWPP_EINVAL;
  if (!marker || !mask || !out) return fail(ctx, IWPP_EINVAL, "morph_recon: NULL image pointer");
  if (height < 1 || width < 1) return fail(ctx, IWPP_EINVAL, "morph_recon: height and width must be >= 1");
  if (conn != 4 && conn != 8) return fail(ctx, IWPP_EINVAL, "morph_recon: conn must be 4 or 8");
  const uint64_t npix = (uint64_t)height * (uint64_t)width;
  if (npix > 0xFFFFFFFFull) return fail(ctx, IWPP_EINVAL, "morph_recon: image larger than 2^32 - 1 pixels");
  if (overlaps(out, npix, mask, npix)) return fail(ctx, IWPP_EINVAL, "morph_recon: out must not alias mask");
  if (out != marker && overlaps(out, npix, marker, npix))
    return fail(ctx, IWPP_EINVAL, "morph_recon: out may equal marker but must not partially overlap it");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, IWPP_EDEVICE, "morph_recon: cannot select the context's device");
  hipStream_t st = static_cast<hipStream_t>(stream);

  iwpp::MrJob job{};
  job.marker = marker;
  job.mask = mask;
  job.out = out;
  job.h = height;
  job.w = width;
  job.tiles_y = (height + 63) / 64;
  job.tiles_x = (width + 63) / 64;
  job.tile_base = 0;
  const uint32_t ntiles = (uint32_t)job.tiles_y * (uint32_t)job.tiles_x;
  const int32_t rc = run_mr(ctx, std::vector<iwpp::MrJob>{job}, ntiles, conn, st, true);
  if (rc != IWPP_OK) return rc;
  ctx->last_stream = st;
  ctx->last_op = 1;
  ctx->have_call = true;
  return IWPP_OK;
}

int32_t iwpp_edt(iwpp_ctx* ctx, const uint8_t* binary, int32_t* sqdist, int32_t* nearest, int32_t height,
                 int32_t width, int32_t conn, void* stream) {
  if (!ctx) return IWPP_EINVAL;
  if (!binary || !sqdist || !nearest) return fail(ctx, IWPP_EINVAL, "edt: NULL image pointer");
  if (height < 1 || width < 1 || height > 32767 || width > 32767)
    return fail(ctx, IWPP_EINVAL, "edt: height and width must be in [1, 32767]");
  if (conn != 4 && conn != 8) return fail(ctx, IWPP_EINVAL, "edt: conn must be 4 or 8");
  const uint64_t npix = (uint64_t)height * (uint64_t)width;
  if (overlaps(sqdist, npix * 4, nearest, npix * 4) || overlaps(sqdist, npix * 4, binary, npix) ||
      overlaps(nearest, npix * 4, binary, npix))
    return fail(ctx, IWPP_EINVAL, "edt: outputs must not alias each other or the input");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, IWPP_EDEVICE, "edt: cannot select the context's device");
  hipStream_t st = static_cast<hipStream_t>(stream);

  iwpp::EdtJob job{};
  job.bin = binary;
  job.sqdist = sqdist;
  job.nearest = nearest;
  job.h = height;
  job.w = width;
  job.pix_base = 0;
  const int32_t rc = run_edt(ctx, std::vector<iwpp::EdtJob>{job}, npix, conn, st, true);
  if (rc != IWPP_OK) return rc;
  ctx->last_stream = st;
  ctx->last_op = 2;
  ctx->have_call = true;
  return IWPP_OK;
}

int32_t iwpp_run_batch(iwpp_ctx* ctx, const iwpp_job* jobs, int32_t n, void* stream) {
  if (!ctx) return IWPP_EINVAL;
  if (!jobs || n < 1) return fail(ctx, IWPP_EINVAL, "run_batch: need at least one job");
  struct Span {
    const void* p;
    size_t n;
    int job;
    bool out;
  };
  std::vector<Span> spans;
  for (int32_t i = 0; i < n; ++i) {
    const iwpp_job& j = jobs[i];
    const std::string at = "run_batch: job " + std::to_string(i) + ": ";
    if (j.op != IWPP_OP_RECON && j.op != IWPP_OP_EDT) return fail(ctx, IWPP_EINVAL, at + "op must be RECON or EDT");
    if (j.conn != 4 && j.conn != 8) return fail(ctx, IWPP_EINVAL, at + "conn must be 4 or 8");
    if (j.height < 1 || j.width < 1) return fail(ctx, IWPP_EINVAL, at + "height and width must be >= 1");
    const uint64_t np = (uint64_t)j.height * (uint64_t)j.width;
    if (j.op == IWPP_OP_RECON) {
      if (!j.in0 || !j.in1 || !j.out0 || j.out1) return fail(ctx, IWPP_EINVAL, at + "recon needs in0, in1, out0 and no out1");
      if (np > 0xFFFFFFFFull) return fail(ctx, IWPP_EINVAL, at + "image larger than 2^32 - 1 pixels");
      spans.push_back({j.in1, np, i, false});
      if (j.out0 != j.in0) spans.push_back({j.in0, np, i, false});
      spans.push_back({j.out0, np, i, true});
    } else {
      if (!j.in0 || j.in1 || !j.out0 || !j.out1) return fail(ctx, IWPP_EINVAL, at + "EDT needs in0, out0, out1 and no in1");
      if (j.height > 32767 || j.width > 32767) return fail(ctx, IWPP_EINVAL, at + "EDT sides must be <= 32767");
      spans.push_back({j.in0, np, i, false});
      spans.push_back({j.out0, np * 4, i, true});
      spans.push_back({j.out1, np * 4, i, true});
    }
  }
  for (size_t a = 0; a < spans.size(); ++a)
    for (size_t b = a + 1; b < spans.size(); ++b)
      if ((spans[a].out || spans[b].out) && overlaps(spans[a].p, spans[a].n, spans[b].p, spans[b].n))
        return fail(ctx, IWPP_EINVAL, "run_batch: an output of job " + std::to_string(spans[a].out ? spans[a].job : spans[b].job) +
                                          " overlaps a buffer of job " + std::to_string(spans[a].out ? spans[b].job : spans[a].job));
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, IWPP_EDEVICE, "run_batch: cannot select the context's device");
  hipStream_t st = static_cast<hipStream_t>(stream);
  bool first = true;
  for (int op : {IWPP_OP_RECON, IWPP_OP_EDT}) {
    for (int conn : {8, 4}) {
      if (op == IWPP_OP_RECON) {
        std::vector<iwpp::MrJob> group;
        uint64_t tiles = 0;
        for (int32_t i = 0; i < n; ++i) {
          const iwpp_job& j = jobs[i];
          if (j.op != op || j.conn != conn) continue;
          iwpp::MrJob m{};
          m.marker = j.in0;
          m.mask = j.in1;
          m.out = static_cast<uint8_t*>(j.out0);
          m.h = j.height;
          m.w = j.width;
          m.tiles_y = (j.height + 63) / 64;
          m.tiles_x = (j.width + 63) / 64;
          m.tile_base = (uint32_t)tiles;
          tiles += (uint64_t)m.tiles_y * (uint64_t)m.tiles_x;
          group.push_back(m);
        }
        if (group.empty()) continue;
        if (tiles >= 0x7FFFFFFFull) return fail(ctx, IWPP_EINVAL, "run_batch: too many reconstruction tiles");
        const int32_t rc = run_mr(ctx, group, (uint32_t)tiles, conn, st, first);
        if (rc != IWPP_OK) return rc;
      } else {
        std::vector<iwpp::EdtJob> group;
        uint64_t pix = 0;
        for (int32_t i = 0; i < n; ++i) {
          const iwpp_job& j = jobs[i];
          if (j.op != op || j.conn != conn) continue;
          iwpp::EdtJob e{};
          e.bin = j.in0;
          e.sqdist = static_cast<int32_t*>(j.out0);
          e.nearest = static_cast<int32_t*>(j.out1);
          e.h = j.height;
          e.w = j.width;
          e.pix_base = (uint32_t)pix;
          pix += (uint64_t)j.height * (uint64_t)j.width;
          group.push_back(e);
          if (pix > 0xFFFFFFFFull) return fail(ctx, IWPP_EINVAL, "run_batch: EDT group larger than 2^32 - 1 pixels");
        }
        if (group.empty()) continue;
        const int32_t rc = run_edt(ctx, group, pix, conn, st, first);
        if (rc != IWPP_OK) return rc;
      }
      first = false;
    }
  }
  ctx->last_stream = st;
  ctx->last_op = 3;
  ctx->have_call = true;
  return IWPP_OK;
}

int32_t iwpp_profile_read(iwpp_ctx* ctx, iwpp_kernel_time* out, int32_t max, int32_t* n) {
  if (!ctx) return IWPP_EINVAL;
  if (!out || !n || max < 0) return fail(ctx, IWPP_EINVAL, "profile_read: NULL argument");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, IWPP_EDEVICE, "profile_read: cannot select the context's device");
  static thread_local int ks[iwpp::Recorder::kCap];
  static thread_local float ms[iwpp::Recorder::kCap];
  const int m = ctx->rec.read(ks, ms, iwpp::Recorder::kCap);
  int w = 0;
  for (int i = 0; i < m && w < max; ++i, ++w) {
    out[w].kernel = ks[i];
    out[w].ms = ms[i];
  }
  *n = w;
  return IWPP_OK;
}

int32_t iwpp_get_stats(iwpp_ctx* ctx, iwpp_stats* out) {
  if (!ctx || !out) return ctx ? fail(ctx, IWPP_EINVAL, "get_stats: out is NULL") : IWPP_EINVAL;
  std::memset(out, 0, sizeof(*out));
  if (!ctx->have_call) return IWPP_OK;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, IWPP_EDEVICE, "get_stats: cannot select the context's device");
  if (hipStreamSynchronize(ctx->last_stream) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, IWPP_EDEVICE, "get_stats: the last call's stream reported an error");
  }
  unsigned long long h[iwpp::kStatShards * iwpp::kStatFields];
  if (hipMemcpy(h, ctx->fixed + kOffStats, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, IWPP_EDEVICE, "get_stats: copy failed");
  }
  unsigned long long f[iwpp::kStatFields] = {};
  for (int s = 0; s < iwpp::kStatShards; ++s)
    for (int k = 0; k < iwpp::kStatFields; ++k) f[k] += h[s * iwpp::kStatFields + k];
  out->op = ctx->last_op;
  out->seeds = (int64_t)f[iwpp::kStatSeeds];
  out->items = (int64_t)f[iwpp::kStatItems];
  out->sweeps = (int64_t)f[iwpp::kStatSweeps];
  out->rounds = (int64_t)f[iwpp::kStatRounds];
  out->updates = (int64_t)f[iwpp::kStatUpdates];
  out->overflow_restarts = (int64_t)f[iwpp::kStatRestarts];
  out->status = f[iwpp::kStatError] ? IWPP_EDEVICE : IWPP_OK;
  if (out->status != IWPP_OK) ctx->err = "a kernel hit its safety limit (grid barrier timeout)";
  return IWPP_OK;
}

}  // extern "C"
