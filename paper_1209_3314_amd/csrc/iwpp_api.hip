// Host side of the C ABI declared in include/iwpp.h: context, argument
// checks, launch plans, scratch management and graph capture.  No exception
// or C++ type crosses the ABI; every entry point returns an iwpp_status code.
//
// A call is turned into a plan: its images grouped by (operation,
// connectivity), each group with the job table its kernels read.  A group is
// launched on a scratch area (work lists, flags, EDT feature buffers) and a
// small fixed area (grid barrier, list counts, statistics).  Eager calls use
// the context's areas, growing the scratch on demand; a batch graph owns its
// areas so that its captured launches stay valid.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/iwpp.h"
#include "iwpp_device.hpp"
#include "iwpp_internal.hpp"
#include "iwpp_runtime.hpp"

static_assert(sizeof(iwpp::GridBarrier) <= iwpp::kBarrierBytes, "barrier area too small");

struct iwpp_graph {
  iwpp_ctx* ctx = nullptr;
  uint8_t* fixed = nullptr;
  uint8_t* scratch = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t last_stream = nullptr;
  bool launched = false;
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

namespace iwpp::rt {

thread_local std::string g_create_err;

int32_t fail(iwpp_ctx* ctx, int32_t code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

DeviceGuard::DeviceGuard(int dev) {
  if (hipGetDevice(&prev) != hipSuccess) return;
  if (prev != dev && hipSetDevice(dev) != hipSuccess) return;
  ok = true;
}

DeviceGuard::~DeviceGuard() {
  int cur = -1;
  if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
}

size_t job_scratch_bytes(int op, int32_t h, int32_t w) {
  if (op == IWPP_OP_RECON_ERODE) op = IWPP_OP_RECON;  // the same kernels
  const int ts = op == IWPP_OP_RECON ? iwpp::kMrTile : iwpp::kEdtTile;
  const uint64_t t = (uint64_t)((h + ts - 1) / ts) * (uint64_t)((w + ts - 1) / ts);
  const uint64_t np = (uint64_t)h * (uint64_t)w;
  // 20 tile words, and per tile 256 bytes of recon border columns or 264 bytes
  // of EDT visit stamps and change masks (+ alignment slack of the per-group
  // arrays is added by the caller)
  return (size_t)(80 * t + 20 * 256 + (op == IWPP_OP_EDT ? 8 * np + 2 * iwpp::kEdtStatePad + 264 * t : 256 * t) +
                  (op == IWPP_OP_RECON ? sizeof(iwpp::MrJob) : sizeof(iwpp::EdtJob)));
}

bool edt_dims_ok(int32_t h, int32_t w) {
  if (h < 1 || w < 1 || h > 46340 || w > 46340) return false;
  const int64_t a = h - 1, b = w - 1;
  return a * a + b * b <= 0x7FFFFFFFll;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb && y < x + na;
}

// ---- plans ---------------------------------------------------------------------

void mr_place(iwpp::MrJob& m, uint64_t& tiles) {
  m.tiles_y = (m.h + iwpp::kMrTile - 1) / iwpp::kMrTile;
  m.tiles_x = (m.w + iwpp::kMrTile - 1) / iwpp::kMrTile;
  m.tile_base = (uint32_t)tiles;
  tiles += (uint64_t)m.tiles_y * (uint64_t)m.tiles_x;
}

void edt_place(iwpp::EdtJob& e, uint64_t& pix, uint64_t& tiles) {
  e.tiles_y = (e.h + iwpp::kEdtTile - 1) / iwpp::kEdtTile;
  e.tiles_x = (e.w + iwpp::kEdtTile - 1) / iwpp::kEdtTile;
  e.tile_base = (uint32_t)tiles;
  e.pix_base = pix;
  tiles += (uint64_t)e.tiles_y * (uint64_t)e.tiles_x;
  pix += (uint64_t)e.h * (uint64_t)e.w;
}

// Validate the jobs and group them by (op, conn).  `who` prefixes messages.
int32_t build_plan(iwpp_ctx* ctx, const iwpp_job* jobs, int32_t n, const char* who, Plan& plan) {
  if (!jobs || n < 1) return fail(ctx, IWPP_EINVAL, std::string(who) + ": need at least one job");
  struct Span {
    const void* p;
    size_t n;
    int job;
    bool out;
  };
  std::vector<Span> spans;
  for (int32_t i = 0; i < n; ++i) {
    const iwpp_job& j = jobs[i];
    const std::string at = std::string(who) + ": job " + std::to_string(i) + ": ";
    if (j.op != IWPP_OP_RECON && j.op != IWPP_OP_RECON_ERODE && j.op != IWPP_OP_EDT)
      return fail(ctx, IWPP_EINVAL, at + "op must be RECON, RECON_ERODE or EDT");
    if (j.conn != 4 && j.conn != 8) return fail(ctx, IWPP_EINVAL, at + "conn must be 4 or 8");
    if (j.height < 1 || j.width < 1) return fail(ctx, IWPP_EINVAL, at + "height and width must be >= 1");
    const uint64_t np = (uint64_t)j.height * (uint64_t)j.width;
    if (j.op != IWPP_OP_EDT) {
      if (!j.in0 || !j.in1 || !j.out0 || j.out1)
        return fail(ctx, IWPP_EINVAL, at + "reconstruction needs in0 (marker), in1 (mask), out0 and no out1");
      // A tile's 66-row band of the image is addressed with 32-bit offsets.
      if (j.width > (1 << 25)) return fail(ctx, IWPP_EINVAL, at + "reconstruction width must be <= 2^25");
      if (overlaps(j.out0, np, j.in1, np)) return fail(ctx, IWPP_EINVAL, at + "out must not alias mask");
      if (j.out0 != j.in0 && overlaps(j.out0, np, j.in0, np))
        return fail(ctx, IWPP_EINVAL, at + "out may equal marker but must not partially overlap it");
      spans.push_back({j.in1, np, i, false});
      if (j.out0 != j.in0) spans.push_back({j.in0, np, i, false});
      spans.push_back({j.out0, np, i, true});
    } else {
      if (!j.in0 || j.in1 || !j.out0 || !j.out1)
        return fail(ctx, IWPP_EINVAL, at + "EDT needs in0 (binary), out0 (sqdist), out1 (nearest) and no in1");
      if (!edt_dims_ok(j.height, j.width))
        return fail(ctx, IWPP_EINVAL, at + "EDT sides must be <= 46340 with (h-1)^2 + (w-1)^2 < 2^31");
      if (overlaps(j.out0, np * 4, j.out1, np * 4) || overlaps(j.out0, np * 4, j.in0, np) ||
          overlaps(j.out1, np * 4, j.in0, np))
        return fail(ctx, IWPP_EINVAL, at + "outputs must not alias each other or the input");
      spans.push_back({j.in0, np, i, false});
      spans.push_back({j.out0, np * 4, i, true});
      spans.push_back({j.out1, np * 4, i, true});
    }
  }
  for (size_t a = 0; a < spans.size(); ++a)
    for (size_t b = a + 1; b < spans.size(); ++b)
      if (spans[a].job != spans[b].job && (spans[a].out || spans[b].out) &&
          overlaps(spans[a].p, spans[a].n, spans[b].p, spans[b].n))
        return fail(ctx, IWPP_EINVAL, std::string(who) + ": an output of job " +
                                          std::to_string(spans[a].out ? spans[a].job : spans[b].job) +
                                          " overlaps a buffer of job " +
                                          std::to_string(spans[a].out ? spans[b].job : spans[a].job));
  for (int op : {IWPP_OP_RECON, IWPP_OP_EDT}) {
    for (int conn : {8, 4}) {
      Group g;
      g.op = op;
      g.conn = conn;
      for (int32_t i = 0; i < n; ++i) {
        const iwpp_job& j = jobs[i];
        // reconstruction by erosion runs in the dilation group on complemented bytes
        const int jop = j.op == IWPP_OP_RECON_ERODE ? IWPP_OP_RECON : j.op;
        if (jop != op || j.conn != conn) continue;
        if (op == IWPP_OP_RECON) {
          iwpp::MrJob m{};
          m.marker = j.in0;
          m.mask = j.in1;
          m.out = static_cast<uint8_t*>(j.out0);
          m.h = j.height;
          m.w = j.width;
          m.inv = j.op == IWPP_OP_RECON_ERODE ? 0xFFFFFFFFu : 0u;
          mr_place(m, g.ntiles);
          g.mr.push_back(m);
        } else {
          iwpp::EdtJob e{};
          e.bin = j.in0;
          e.sqdist = static_cast<int32_t*>(j.out0);
          e.nearest = static_cast<int32_t*>(j.out1);
          e.h = j.height;
          e.w = j.width;
          edt_place(e, g.npix, g.ntiles);
          g.edt.push_back(e);
        }
      }
      if (g.njobs() == 0) continue;
      // recon addresses its 256-byte border-column blocks with 32-bit offsets
      if (g.ntiles >= (op == IWPP_OP_RECON ? (1ull << 24) : 0x7FFFFFFFull))
        return fail(ctx, IWPP_EINVAL, std::string(who) + ": too many tiles in one group");
      g.table_off = plan.table_bytes;
      plan.table_bytes += g.table_bytes();
      if (g.scratch_bytes() > plan.scratch_bytes) plan.scratch_bytes = g.scratch_bytes();
      plan.groups.push_back(std::move(g));
    }
  }
  return IWPP_OK;
}

int32_t upload_tables(iwpp_ctx* ctx, const Plan& plan, uint8_t* tables, hipStream_t st, bool sync) {
  for (const Group& g : plan.groups) {
    if (g.njobs() <= 1) continue;
    const void* src = g.op == IWPP_OP_RECON ? (const void*)g.mr.data() : (const void*)g.edt.data();
    const size_t bytes = g.op == IWPP_OP_RECON ? g.mr.size() * sizeof(iwpp::MrJob) : g.edt.size() * sizeof(iwpp::EdtJob);
    const hipError_t e = sync ? hipMemcpy(tables + g.table_off, src, bytes, hipMemcpyHostToDevice)
                              : hipMemcpyAsync(tables + g.table_off, src, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, IWPP_EDEVICE, "job table upload failed");
    }
  }
  return IWPP_OK;
}

void pack_tables(const Plan& plan, uint8_t* host) {
  for (const Group& g : plan.groups) {
    if (g.njobs() <= 1) continue;
    const void* src = g.op == IWPP_OP_RECON ? (const void*)g.mr.data() : (const void*)g.edt.data();
    const size_t bytes = g.op == IWPP_OP_RECON ? g.mr.size() * sizeof(iwpp::MrJob) : g.edt.size() * sizeof(iwpp::EdtJob);
    std::memcpy(host + g.table_off, src, bytes);
  }
}

// Launch the kernels of one group on `st`, using `scratch`/`fixed`/`tables`.
// `first` also clears the statistics.
int32_t launch_group(iwpp_ctx* ctx, const Group& g, uint8_t* scratch, uint8_t* fixed, uint8_t* tables, hipStream_t st,
                     bool first, iwpp::Recorder* rec, bool seed_only) {
  rec->begin(IWPP_K_RESET, st);
  const int zr = iwpp::zero_words(reinterpret_cast<uint32_t*>(fixed), (first ? kFixedBytes : kOffStats) / 4, st);
  rec->end(st);
  if (zr != 0) return fail(ctx, IWPP_EDEVICE, "reset kernel launch failed");
  const size_t tb = align256(g.ntiles * 4);
  const uint32_t nj = g.njobs();
  const char* e = "";
  int lr = 0;
  if (g.op == IWPP_OP_RECON) {
    iwpp::MrArgs a{};
    a.job0 = g.mr[0];
    a.njobs = nj;
    a.ntiles = (uint32_t)g.ntiles;
    const int64_t cap = ctx->opt.mr_list_capacity;
    a.list_cap = (cap > 0 && (uint64_t)cap < g.ntiles) ? (uint32_t)cap : (uint32_t)g.ntiles;
    // Defaults from measurement on the 16384^2 workloads: a visit that stops
    // after two sweep iterations and is listed again is cheaper overall than
    // one swept to stability, since neighbours keep changing its halo; the
    // seed pass does one iteration with 8-connectivity, two with 4 (whose
    // paths inside a tile are longer).
    a.max_sweeps = ctx->opt.mr_max_sweeps > 0 ? ctx->opt.mr_max_sweeps : 2;
    a.seed_sweeps = ctx->opt.mr_seed_sweeps > 0 ? ctx->opt.mr_seed_sweeps : (g.conn == 8 ? 1 : 2);
    a.seed_only = seed_only ? 1u : 0u;
    a.seed_strip = (uint32_t)ctx->opt.mr_seed_strip;
    a.stage_depth = (uint32_t)ctx->opt.stage_depth;
    a.wg_waves = ctx->opt.wg_waves == 8 ? 8u : 4u;
    a.flags = reinterpret_cast<uint32_t*>(scratch);
    a.lists = reinterpret_cast<uint32_t*>(scratch + 2 * tb);
    a.unsettled = reinterpret_cast<uint32_t*>(scratch + 18 * tb);
    a.tile_job = nj > 1 ? reinterpret_cast<uint32_t*>(scratch + 19 * tb) : nullptr;
    a.cols = scratch + 20 * tb;
    a.jobs = nj > 1 ? reinterpret_cast<const iwpp::MrJob*>(tables + g.table_off) : nullptr;
    a.counts = reinterpret_cast<uint32_t*>(fixed + kOffCounts);
    a.lost = reinterpret_cast<uint32_t*>(fixed + kOffLost);
    a.bar = reinterpret_cast<iwpp::GridBarrier*>(fixed + kOffBarrier);
    a.stats = reinterpret_cast<unsigned long long*>(fixed + kOffStats);
    a.clock = reinterpret_cast<unsigned long long*>(fixed + kOffClock);
    lr = iwpp::mr_launch(a, g.conn, ctx->opt.persistent_blocks, st, rec, &e);
  } else {
    iwpp::EdtArgs a{};
    const size_t fb = align256(g.npix * 4) + iwpp::kEdtStatePad;
    a.job0 = g.edt[0];
    a.njobs = nj;
    a.npix = g.npix;
    a.wide = 0;
    for (const iwpp::EdtJob& e : g.edt)
      if (e.h > 32767 || e.w > 32767) a.wide = 1;
    a.ntiles = (uint32_t)g.ntiles;
    a.feat0 = reinterpret_cast<uint32_t*>(scratch);
    a.feat1 = reinterpret_cast<uint32_t*>(scratch + fb);
    a.flags = reinterpret_cast<uint32_t*>(scratch + 2 * fb);
    a.lists = reinterpret_cast<uint32_t*>(scratch + 2 * fb + 2 * tb);
    a.tile_job = nj > 1 ? reinterpret_cast<uint32_t*>(scratch + 2 * fb + 18 * tb) : nullptr;
    a.stamps = reinterpret_cast<uint32_t*>(scratch + 2 * fb + 19 * tb);
    a.marks = reinterpret_cast<uint32_t*>(scratch + 2 * fb + 21 * tb);
    a.jobs = nj > 1 ? reinterpret_cast<const iwpp::EdtJob*>(tables + g.table_off) : nullptr;
    a.counts = reinterpret_cast<uint32_t*>(fixed + kOffCounts);
    a.ovf = reinterpret_cast<uint32_t*>(fixed + kOffOvf);
    a.stage_depth = (uint32_t)ctx->opt.stage_depth;
    a.wg_waves = ctx->opt.wg_waves == 8 ? 8u : 4u;
    a.bar = reinterpret_cast<iwpp::GridBarrier*>(fixed + kOffBarrier);
    a.stats = reinterpret_cast<unsigned long long*>(fixed + kOffStats);
    a.clock = reinterpret_cast<unsigned long long*>(fixed + kOffClock);
    lr = iwpp::edt_launch(a, g.conn, ctx->opt.persistent_blocks, st, rec, &e);
  }
  if (lr != 0) {
    (void)hipGetLastError();
    return fail(ctx, IWPP_EDEVICE, std::string(g.op == IWPP_OP_RECON ? "morph_recon: " : "edt: ") + e);
  }
  return IWPP_OK;
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

// Run a plan eagerly on the context's areas.
int32_t run_plan(iwpp_ctx* ctx, const Plan& plan, hipStream_t st, int op_code) {
  const size_t sb = align256(plan.scratch_bytes);
  int32_t rc = ensure_scratch(ctx, sb + plan.table_bytes);
  if (rc != IWPP_OK) return rc;
  uint8_t* tables = ctx->scratch + sb;
  if ((rc = upload_tables(ctx, plan, tables, st, false)) != IWPP_OK) return rc;
  bool first = true;
  for (const Group& g : plan.groups) {
    if ((rc = launch_group(ctx, g, ctx->scratch, ctx->fixed, tables, st, first, &ctx->rec)) != IWPP_OK) return rc;
    first = false;
  }
  ctx->last_stream = st;
  ctx->last_fixed = ctx->fixed;
  ctx->last_op = op_code;
  ctx->have_call = true;
  return IWPP_OK;
}

int32_t read_stats(iwpp_ctx* ctx, const uint8_t* fixed, hipStream_t st, int op, iwpp_stats* out) {
  std::memset(out, 0, sizeof(*out));
  if (hipStreamSynchronize(st) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, IWPP_EDEVICE, "get_stats: the last call's stream reported an error");
  }
  unsigned long long h[iwpp::kStatShards * iwpp::kStatFields];
  if (hipMemcpy(h, fixed + kOffStats, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, IWPP_EDEVICE, "get_stats: copy failed");
  }
  fold_stats(h, op, out);
  if (out->status != IWPP_OK) ctx->err = "a kernel hit its safety limit (grid barrier timeout or round cap)";
  return IWPP_OK;
}

void fold_stats(const unsigned long long* h, int op, iwpp_stats* out) {
  std::memset(out, 0, sizeof(*out));
  unsigned long long f[iwpp::kStatFields] = {};
  for (int s = 0; s < iwpp::kStatShards; ++s)
    for (int k = 0; k < iwpp::kStatFields; ++k) f[k] += h[s * iwpp::kStatFields + k];
  out->op = op;
  out->seeds = (int64_t)f[iwpp::kStatSeeds];
  out->items = (int64_t)f[iwpp::kStatItems];
  out->sweeps = (int64_t)f[iwpp::kStatSweeps];
  out->rounds = (int64_t)f[iwpp::kStatRounds];
  out->updates = (int64_t)f[iwpp::kStatUpdates];
  out->overflow_restarts = (int64_t)f[iwpp::kStatRestarts];
  out->status = f[iwpp::kStatError] ? IWPP_EDEVICE : IWPP_OK;
}

// Round timeline words of a fixed area (see iwpp_round_times), after the
// stream that last used it has finished.
int32_t read_clock(iwpp_ctx* ctx, const uint8_t* fixed, hipStream_t st, double* us, int64_t* work, int32_t max,
                   int32_t* n) {
  if (hipStreamSynchronize(st) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, IWPP_EDEVICE, "round_times: the last call's stream reported an error");
  }
  unsigned long long h[iwpp::kClockWords];
  int khz = 0;
  if (hipMemcpy(h, fixed + kOffClock, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess || khz <= 0) {
    (void)hipGetLastError();
    return fail(ctx, IWPP_EDEVICE, "round_times: read failed");
  }
  const unsigned long long cnt = h[0] < (unsigned long long)iwpp::kClockStamps ? h[0] : iwpp::kClockStamps - 1;
  int32_t w = 0;
  for (unsigned long long i = 1; i < cnt && w < max; ++i, ++w) {
    us[w] = (double)(h[i + 1] - h[i]) * 1000.0 / khz;
    if (work) work[w] = (int64_t)h[iwpp::kClockStamps + w];
  }
  *n = w;
  return IWPP_OK;
}

bool options_valid(const iwpp_options& o) {
  return o.mr_list_capacity >= 0 && o.mr_max_sweeps >= 0 && o.persistent_blocks >= 0 && o.profile >= 0 &&
         o.mr_seed_sweeps >= 0 && (o.wg_waves == 0 || o.wg_waves == 4 || o.wg_waves == 8) && o.stage_depth >= 0 &&
         o.stage_depth <= 64 && o.mr_seed_strip >= 0;
}

}  // namespace iwpp::rt

using namespace iwpp::rt;

extern "C" {

int32_t iwpp_version(void) { return (0 << 16) | 3; }

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
  if (opt && !options_valid(*opt)) {
    delete ctx;
    g_create_err = "iwpp_create: option out of range (negative, wg_waves not 0/4/8 or stage_depth above 64)";
    return IWPP_EINVAL;
  }
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
  // Set-up of the allocation-free entry point; if it fails that entry point
  // reports IWPP_EDEVICE and everything else works.
  (void)noalloc_setup(ctx);
  *out = ctx;
  return IWPP_OK;
}

void iwpp_destroy(iwpp_ctx* ctx) {
  if (!ctx) return;
  if (ctx->server) (void)iwpp_server_stop(ctx->server);
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
  if (ctx->server) return fail(ctx, IWPP_EBUSY, "morph_recon: the context is serving");
  if (!marker || !mask || !out) return fail(ctx, IWPP_EINVAL, "morph_recon: NULL image pointer");
  iwpp_job j{IWPP_OP_RECON, conn, height, width, marker, mask, out, nullptr};
  Plan plan;
  int32_t rc = build_plan(ctx, &j, 1, "morph_recon", plan);
  if (rc != IWPP_OK) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, IWPP_EDEVICE, "morph_recon: cannot select the context's device");
  return run_plan(ctx, plan, static_cast<hipStream_t>(stream), 1);
}

int32_t iwpp_morph_recon_erode_u8(iwpp_ctx* ctx, const uint8_t* marker, const uint8_t* mask, uint8_t* out,
                                  int32_t height, int32_t width, int32_t conn, void* stream) {
  if (!ctx) return IWPP_EINVAL;
  if (ctx->server) return fail(ctx, IWPP_EBUSY, "morph_recon_erode: the context is serving");
  if (!marker || !mask || !out) return fail(ctx, IWPP_EINVAL, "morph_recon_erode: NULL image pointer");
  iwpp_job j{IWPP_OP_RECON_ERODE, conn, height, width, marker, mask, out, nullptr};
  Plan plan;
  int32_t rc = build_plan(ctx, &j, 1, "morph_recon_erode", plan);
  if (rc != IWPP_OK) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, IWPP_EDEVICE, "morph_recon_erode: cannot select the context's device");
  return run_plan(ctx, plan, static_cast<hipStream_t>(stream), 1);
}

int32_t iwpp_edt(iwpp_ctx* ctx, const uint8_t* binary, int32_t* sqdist, int32_t* nearest, int32_t height,
                 int32_t width, int32_t conn, void* stream) {
  if (!ctx) return IWPP_EINVAL;
  if (ctx->server) return fail(ctx, IWPP_EBUSY, "edt: the context is serving");
  if (!binary || !sqdist || !nearest) return fail(ctx, IWPP_EINVAL, "edt: NULL image pointer");
  iwpp_job j{IWPP_OP_EDT, conn, height, width, binary, nullptr, sqdist, nearest};
  Plan plan;
  int32_t rc = build_plan(ctx, &j, 1, "edt", plan);
  if (rc != IWPP_OK) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, IWPP_EDEVICE, "edt: cannot select the context's device");
  return run_plan(ctx, plan, static_cast<hipStream_t>(stream), 2);
}

int32_t iwpp_run_batch(iwpp_ctx* ctx, const iwpp_job* jobs, int32_t n, void* stream) {
  if (!ctx) return IWPP_EINVAL;
  if (ctx->server) return fail(ctx, IWPP_EBUSY, "run_batch: the context is serving");
  Plan plan;
  int32_t rc = build_plan(ctx, jobs, n, "run_batch", plan);
  if (rc != IWPP_OK) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, IWPP_EDEVICE, "run_batch: cannot select the context's device");
  return run_plan(ctx, plan, static_cast<hipStream_t>(stream), 3);
}

int32_t iwpp_set_options(iwpp_ctx* ctx, const iwpp_options* opt) {
  if (!ctx) return IWPP_EINVAL;
  if (ctx->server) return fail(ctx, IWPP_EBUSY, "set_options: the context is serving");
  if (!opt) return fail(ctx, IWPP_EINVAL, "set_options: NULL options");
  if (!options_valid(*opt))
    return fail(ctx, IWPP_EINVAL, "set_options: option out of range (negative, wg_waves not 0/4/8 or stage_depth above 64)");
  ctx->opt = *opt;
  ctx->rec.enabled = ctx->opt.profile != 0;
  return IWPP_OK;
}

int32_t iwpp_batch_graph_create(iwpp_ctx* ctx, const iwpp_job* jobs, int32_t n, iwpp_graph** out) {
  if (!ctx) return IWPP_EINVAL;
  if (ctx->server) return fail(ctx, IWPP_EBUSY, "batch_graph_create: the context is serving");
  if (!out) return fail(ctx, IWPP_EINVAL, "batch_graph_create: out is NULL");
  *out = nullptr;
  Plan plan;
  int32_t rc = build_plan(ctx, jobs, n, "batch_graph_create", plan);
  if (rc != IWPP_OK) return rc;
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(ctx, IWPP_EDEVICE, "batch_graph_create: cannot select the context's device");
  iwpp_graph* g = new (std::nothrow) iwpp_graph();
  if (!g) return fail(ctx, IWPP_ENOMEM, "batch_graph_create: out of host memory");
  g->ctx = ctx;
  const size_t sb = align256(plan.scratch_bytes);
  void* p = nullptr;
  void* f = nullptr;
  if (hipMalloc(&p, sb + plan.table_bytes + 256) != hipSuccess || hipMalloc(&f, kFixedBytes) != hipSuccess) {
    (void)hipGetLastError();
    if (p) (void)hipFree(p);
    delete g;
    return fail(ctx, IWPP_ENOMEM, "batch_graph_create: device allocation failed");
  }
  g->scratch = static_cast<uint8_t*>(p);
  g->fixed = static_cast<uint8_t*>(f);
  hipStream_t cs = nullptr;
  iwpp::Recorder off;  // no event records inside a graph
  ctx->err.clear();
  rc = upload_tables(ctx, plan, g->scratch + sb, nullptr, true);
  if (rc == IWPP_OK && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
    rc = fail(ctx, IWPP_EDEVICE, "batch_graph_create: stream creation failed");
  if (rc == IWPP_OK && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
    rc = fail(ctx, IWPP_EDEVICE, "batch_graph_create: capture could not start");
  if (rc == IWPP_OK) {
    bool first = true;
    for (const Group& grp : plan.groups) {
      rc = launch_group(ctx, grp, g->scratch, g->fixed, g->scratch + sb, cs, first, &off);
      if (rc != IWPP_OK) break;
      first = false;
    }
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (rc == IWPP_OK && (ec != hipSuccess || !graph)) rc = fail(ctx, IWPP_EDEVICE, "batch_graph_create: capture failed");
    g->graph = graph;
  }
  if (rc == IWPP_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
    rc = fail(ctx, IWPP_EDEVICE, "batch_graph_create: instantiation failed");
  if (cs) (void)hipStreamDestroy(cs);
  if (rc != IWPP_OK) {
    (void)hipGetLastError();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    (void)hipFree(g->scratch);
    (void)hipFree(g->fixed);
    delete g;
    if (ctx->err.empty()) ctx->err = "batch_graph_create: device error";
    return rc == IWPP_EINVAL ? rc : IWPP_EDEVICE;
  }
  *out = g;
  return IWPP_OK;
}

int32_t iwpp_batch_graph_launch(iwpp_graph* g, void* stream) {
  if (!g) return IWPP_EINVAL;
  DeviceGuard dg(g->ctx->device);
  if (!dg.ok) return fail(g->ctx, IWPP_EDEVICE, "batch_graph_launch: cannot select the context's device");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipGraphLaunch(g->exec, st) != hipSuccess) {
    (void)hipGetLastError();
    return fail(g->ctx, IWPP_EDEVICE, "batch_graph_launch: launch failed");
  }
  g->last_stream = st;
  g->launched = true;
  return IWPP_OK;
}

int32_t iwpp_batch_graph_stats(iwpp_graph* g, iwpp_stats* out) {
  if (!g || !out) return g ? fail(g->ctx, IWPP_EINVAL, "batch_graph_stats: out is NULL") : IWPP_EINVAL;
  std::memset(out, 0, sizeof(*out));
  if (!g->launched) return IWPP_OK;
  DeviceGuard dg(g->ctx->device);
  if (!dg.ok) return fail(g->ctx, IWPP_EDEVICE, "batch_graph_stats: cannot select the context's device");
  return read_stats(g->ctx, g->fixed, g->last_stream, 3, out);
}

void iwpp_batch_graph_destroy(iwpp_graph* g) {
  if (!g) return;
  {
    DeviceGuard dg(g->ctx->device);
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->scratch) (void)hipFree(g->scratch);
    if (g->fixed) (void)hipFree(g->fixed);
  }
  delete g;
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

int32_t iwpp_round_times(iwpp_ctx* ctx, double* us, int32_t max, int32_t* n) {
  if (!ctx) return IWPP_EINVAL;
  if (!us || !n || max < 0) return fail(ctx, IWPP_EINVAL, "round_times: NULL argument");
  *n = 0;
  if (!ctx->have_call) return IWPP_OK;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, IWPP_EDEVICE, "round_times: cannot select the context's device");
  return read_clock(ctx, ctx->last_fixed, ctx->last_stream, us, nullptr, max, n);
}

int32_t iwpp_round_work(iwpp_ctx* ctx, double* us, int64_t* tiles, int32_t max, int32_t* n) {
  if (!ctx) return IWPP_EINVAL;
  if (!us || !tiles || !n || max < 0) return fail(ctx, IWPP_EINVAL, "round_work: NULL argument");
  *n = 0;
  if (!ctx->have_call) return IWPP_OK;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, IWPP_EDEVICE, "round_work: cannot select the context's device");
  return read_clock(ctx, ctx->last_fixed, ctx->last_stream, us, tiles, max, n);
}

int32_t iwpp_batch_graph_round_times(iwpp_graph* gr, double* us, int32_t max, int32_t* n) {
  if (!gr) return IWPP_EINVAL;
  if (!us || !n || max < 0) return fail(gr->ctx, IWPP_EINVAL, "batch_graph_round_times: NULL argument");
  *n = 0;
  if (!gr->launched) return IWPP_OK;
  DeviceGuard g(gr->ctx->device);
  if (!g.ok) return fail(gr->ctx, IWPP_EDEVICE, "batch_graph_round_times: cannot select the context's device");
  return read_clock(gr->ctx, gr->fixed, gr->last_stream, us, nullptr, max, n);
}

int32_t iwpp_get_stats(iwpp_ctx* ctx, iwpp_stats* out) {
  if (!ctx || !out) return ctx ? fail(ctx, IWPP_EINVAL, "get_stats: out is NULL") : IWPP_EINVAL;
  std::memset(out, 0, sizeof(*out));
  if (!ctx->have_call) return IWPP_OK;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, IWPP_EDEVICE, "get_stats: cannot select the context's device");
  return read_stats(ctx, ctx->last_fixed, ctx->last_stream, ctx->last_op, out);
}

}  // extern "C"
