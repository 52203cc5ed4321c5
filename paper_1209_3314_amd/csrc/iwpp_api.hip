// Host side of the C ABI declared in include/iwpp.h: context, argument
// checks, scratch management and launch sequencing.  No exception or C++ type
// crosses the ABI; every entry point returns an iwpp_status code.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <new>
#include <string>

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

// Clear counters, list fill levels, flags and the barrier for a new call.
int32_t reset_fixed(iwpp_ctx* ctx, hipStream_t stream) {
  ctx->rec.begin(IWPP_K_RESET, stream);
  const int r = iwpp::zero_words(reinterpret_cast<uint32_t*>(ctx->fixed), kFixedBytes / 4, stream);
  ctx->rec.end(stream);
  if (r != 0) return fail(ctx, IWPP_EDEVICE, "reset kernel launch failed");
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

  iwpp::MrArgs a{};
  a.marker = marker;
  a.mask = mask;
  a.out = out;
  a.h = height;
  a.w = width;
  a.tiles_y = (height + 63) / 64;
  a.tiles_x = (width + 63) / 64;
  a.ntiles = (uint32_t)a.tiles_y * (uint32_t)a.tiles_x;
  const int64_t cap = ctx->opt.mr_list_capacity;
  a.list_cap = (cap > 0 && (uint64_t)cap < a.ntiles) ? (uint32_t)cap : a.ntiles;
  a.max_sweeps = ctx->opt.mr_max_sweeps > 0 ? ctx->opt.mr_max_sweeps : 64;
  a.seed_sweeps = a.max_sweeps;
  const size_t flag_bytes = align256((size_t)a.ntiles * 2 * 4);
  const size_t list_bytes = align256((size_t)a.ntiles * 2 * 4);
  int32_t rc = ensure_scratch(ctx, flag_bytes + list_bytes);
  if (rc != IWPP_OK) return rc;
  a.flags = reinterpret_cast<uint32_t*>(ctx->scratch);
  a.lists = reinterpret_cast<uint32_t*>(ctx->scratch + flag_bytes);
  a.counts = reinterpret_cast<uint32_t*>(ctx->fixed + kOffCounts);
  a.lost = reinterpret_cast<uint32_t*>(ctx->fixed + kOffLost);
  a.bar = reinterpret_cast<iwpp::GridBarrier*>(ctx->fixed + kOffBarrier);
  a.stats = reinterpret_cast<unsigned long long*>(ctx->fixed + kOffStats);
  if ((rc = reset_fixed(ctx, st)) != IWPP_OK) return rc;
  const char* e = "";
  if (iwpp::mr_launch(a, conn, ctx->opt.persistent_blocks, st, &ctx->rec, &e) != 0) {
    (void)hipGetLastError();
    return fail(ctx, IWPP_EDEVICE, std::string("morph_recon: ") + e);
  }
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

  iwpp::EdtArgs a{};
  a.bin = binary;
  a.sqdist = sqdist;
  a.nearest = nearest;
  a.h = height;
  a.w = width;
  a.npix = (uint32_t)npix;
  const size_t key_bytes = align256((size_t)npix * 8);
  const size_t stamp_bytes = align256((size_t)npix * 4);
  const size_t list_bytes = align256((size_t)npix * 2 * 4);
  int32_t rc = ensure_scratch(ctx, 2 * key_bytes + stamp_bytes + list_bytes);
  if (rc != IWPP_OK) return rc;
  a.key0 = reinterpret_cast<unsigned long long*>(ctx->scratch);
  a.key1 = reinterpret_cast<unsigned long long*>(ctx->scratch + key_bytes);
  a.stamp = reinterpret_cast<uint32_t*>(ctx->scratch + 2 * key_bytes);
  a.lists = reinterpret_cast<uint32_t*>(ctx->scratch + 2 * key_bytes + stamp_bytes);
  a.counts = reinterpret_cast<uint32_t*>(ctx->fixed + kOffCounts);
  a.ovf = reinterpret_cast<uint32_t*>(ctx->fixed + kOffOvf);
  a.bar = reinterpret_cast<iwpp::GridBarrier*>(ctx->fixed + kOffBarrier);
  a.stats = reinterpret_cast<unsigned long long*>(ctx->fixed + kOffStats);
  if ((rc = reset_fixed(ctx, st)) != IWPP_OK) return rc;
  const char* e = "";
  if (iwpp::edt_launch(a, conn, ctx->opt.persistent_blocks, st, &ctx->rec, &e) != 0) {
    (void)hipGetLastError();
    return fail(ctx, IWPP_EDEVICE, std::string("edt: ") + e);
  }
  ctx->last_stream = st;
  ctx->last_op = 2;
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
