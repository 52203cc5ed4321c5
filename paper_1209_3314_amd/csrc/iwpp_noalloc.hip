// Reconstruction entry point that allocates nothing (iwpp_morph_recon_u8_noalloc).
//
// Its work lists, tile flags, border-column blocks, list counts, grid barrier
// and statistics live in one static device array of fixed size instead of the
// context's growable scratch, for callers that cannot allocate device memory
// during a call (code under stream capture, tight serving loops).  The array
// exists once per device, for the life of the process; every call on a device
// uses the same array, so such calls must not overlap on one device.
//
// Host code never uses the array's name as an address: the name is only a
// host-side stand-in for the device symbol.  The device address is looked up
// once per device, with that device current, at context creation
// (noalloc_setup) and kept per device.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "../../include/iwpp.h"
#include "iwpp_internal.hpp"
#include "iwpp_runtime.hpp"

// The static work area: the fixed area (barrier, counts, statistics,
// timeline) first, then the group scratch.
static __device__ __align__(256) uint8_t scratch[IWPP_NOALLOC_SCRATCH_BYTES];

namespace iwpp::rt {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint8_t* g_base[kMaxDevices] = {};  // device address of `scratch` per device (null: not set up)
constexpr size_t kNoallocFixed = 4096 * ((kFixedBytes + 4095) / 4096);
static_assert(kNoallocFixed + 256 <= IWPP_NOALLOC_SCRATCH_BYTES, "static area too small");
}  // namespace

// Look up the array's device address on ctx's device (current when this is
// called) once per device, and give it to the context.
int32_t noalloc_setup(iwpp_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices) return IWPP_OK;  // the entry point then reports EDEVICE
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_base[ctx->device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return IWPP_EDEVICE;
    }
    g_base[ctx->device] = static_cast<uint8_t*>(p);
  }
  ctx->noalloc = g_base[ctx->device];
  return IWPP_OK;
}

size_t noalloc_group_limit() { return IWPP_NOALLOC_SCRATCH_BYTES - kNoallocFixed; }

}  // namespace iwpp::rt

using namespace iwpp::rt;

extern "C" int32_t iwpp_morph_recon_u8_noalloc(iwpp_ctx* ctx, const uint8_t* marker, const uint8_t* mask, uint8_t* out,
                                               int32_t height, int32_t width, int32_t conn, void* stream) {
  if (!ctx) return IWPP_EINVAL;
  if (ctx->server) return fail(ctx, IWPP_EBUSY, "morph_recon_noalloc: the context is serving");
  if (!marker || !mask || !out) return fail(ctx, IWPP_EINVAL, "morph_recon_noalloc: NULL image pointer");
  iwpp_job j{IWPP_OP_RECON, conn, height, width, marker, mask, out, nullptr};
  Plan plan;
  int32_t rc = build_plan(ctx, &j, 1, "morph_recon_noalloc", plan);
  if (rc != IWPP_OK) return rc;
  const Group& g = plan.groups[0];
  const size_t need = align256(g.scratch_bytes());
  if (need > noalloc_group_limit())
    return fail(ctx, IWPP_EINVAL,
                "morph_recon_noalloc: the image needs " + std::to_string(need) + " bytes of scratch (" +
                    std::to_string(g.ntiles) + " tiles of 64x64); the static area holds " +
                    std::to_string(noalloc_group_limit()) + " (use iwpp_morph_recon_u8)");
  if (!ctx->noalloc) return fail(ctx, IWPP_EDEVICE, "morph_recon_noalloc: the static area was not set up");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(ctx, IWPP_EDEVICE, "morph_recon_noalloc: cannot select the context's device");
  static iwpp::Recorder off;  // never enabled: recording would create events
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint8_t* fixed = ctx->noalloc;
  // first = true: the fixed area (counts, statistics) is cleared by a fill kernel
  if ((rc = launch_group(ctx, g, ctx->noalloc + kNoallocFixed, fixed, nullptr, st, true, &off)) != IWPP_OK) return rc;
  ctx->last_stream = st;
  ctx->last_fixed = fixed;
  ctx->last_op = 1;
  ctx->have_call = true;
  return IWPP_OK;
}
