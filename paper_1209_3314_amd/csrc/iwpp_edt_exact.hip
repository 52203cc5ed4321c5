// Exact Euclidean distance transform (iwpp_edt_exact).
//
// The propagation EDT of Sec. 2.2 is an approximation; the paper notes that
// exact distances need extra work beyond the 8-neighbour propagation.  This
// is the exact transform by the separable method of Meijster, Roerdink and
// Hesselink (2000), restated for the GPU:
//   1. columns: for every pixel, the nearest feature in its own column (the
//      column is cut into segments scanned in parallel; a segment's nearest
//      feature above and below comes from the summaries of the segments
//      before and after it);
//   2. rows: for every row, the lower envelope of the parabolas
//      x -> (x - x')^2 + (y - r(x'))^2 over the columns x' (r(x') is the row
//      of column x's nearest feature), built left to right with a stack and
//      read right to left; every pixel takes the parabola of the envelope
//      above it.  One lane runs one row; the stacks live in scratch memory.
// All arithmetic is integer; the squared distance is exact and the nearest
// feature is one at exactly that distance (ties: the smaller column, then the
// upper row).
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/iwpp.h"
#include "iwpp_device.hpp"
#include "iwpp_internal.hpp"
#include "iwpp_runtime.hpp"

namespace iwpp {
namespace xedt {

constexpr int kSeg = 128;              // rows per column segment
constexpr int32_t kNone = -1;          // no feature (row index)
constexpr int32_t kBelowNone = 0x7FFFFFFF;

struct XArgs {
  const uint8_t* bin;  // 0 = feature
  int32_t* sqdist;
  int32_t* nearest;
  int32_t* frow;       // [h*w] row of the nearest feature in the pixel's column, or -1
  int32_t* first;      // [nseg][w] first feature row in the segment, or kBelowNone
  int32_t* last;       // [nseg][w] last feature row in the segment, or -1
  int32_t* stk_col;    // [h][w] envelope stacks: parabola columns
  int32_t* stk_from;   // [h][w] the first x each parabola covers
  int32_t* stk_r;      // [h][w] the parabola's feature row
  int32_t h, w, nseg;
};

// Summary of each (segment, column): its first and last feature row.
__global__ __launch_bounds__(64) void k_col_summary(XArgs a) {
  const int x = blockIdx.x * 64 + (int)threadIdx.x, s = blockIdx.y;
  if (x >= a.w) return;
  const int y0 = s * kSeg, y1 = y0 + kSeg < a.h ? y0 + kSeg : a.h;
  int32_t f = kBelowNone, l = kNone;
  for (int y = y0; y < y1; ++y) {
    if (a.bin[(size_t)y * (uint32_t)a.w + (uint32_t)x] == 0) {
      if (f == kBelowNone) f = y;
      l = y;
    }
  }
  a.first[(size_t)s * (uint32_t)a.w + (uint32_t)x] = f;
  a.last[(size_t)s * (uint32_t)a.w + (uint32_t)x] = l;
}

// The nearest feature row in the column for every pixel of a segment: the
// last feature at or above (carried from the segments above), the first at or
// below (carried from the segments below); the closer wins, the upper on a tie.
__global__ __launch_bounds__(64) void k_col(XArgs a) {
  const int x = blockIdx.x * 64 + (int)threadIdx.x, s = blockIdx.y;
  if (x >= a.w) return;
  const int y0 = s * kSeg, y1 = y0 + kSeg < a.h ? y0 + kSeg : a.h;
  int32_t above = kNone, below = kBelowNone;
  for (int t = s - 1; t >= 0 && above == kNone; --t) above = a.last[(size_t)t * (uint32_t)a.w + (uint32_t)x];
  for (int t = s + 1; t < a.nseg && below == kBelowNone; ++t) below = a.first[(size_t)t * (uint32_t)a.w + (uint32_t)x];
  for (int y = y0; y < y1; ++y) {  // downward: the last feature at or above y
    const size_t p = (size_t)y * (uint32_t)a.w + (uint32_t)x;
    if (a.bin[p] == 0) above = y;
    a.frow[p] = above;
  }
  for (int y = y1 - 1; y >= y0; --y) {  // upward: the first at or below y, then the choice
    const size_t p = (size_t)y * (uint32_t)a.w + (uint32_t)x;
    if (a.bin[p] == 0) below = y;
    const int32_t up = a.frow[p];
    const int64_t du = up == kNone ? INT64_MAX : (int64_t)(y - up);
    const int64_t dd = below == kBelowNone ? INT64_MAX : (int64_t)(below - y);
    a.frow[p] = du == INT64_MAX && dd == INT64_MAX ? kNone : (du <= dd ? up : below);
  }
}

// Rows: one lane per row.  f(x') = (y - r(x'))^2, "infinite" for a column
// without features; F(x, x') = (x - x')^2 + f(x').  The envelope is a stack
// of parabolas (column x', its feature row r, the first x it covers); the top
// entry stays in registers, the rest in scratch memory.
__global__ __launch_bounds__(64) void k_row(XArgs a) {
  const int y = blockIdx.x * 64 + (int)threadIdx.x;
  if (y >= a.h) return;
  const int W = a.w;
  const size_t row = (size_t)y * (uint32_t)W;
  const int64_t inf = 4 * ((int64_t)W + a.h) * ((int64_t)W + a.h);
  auto fr = [&](int32_t r) -> int64_t { return r == kNone ? inf : (int64_t)(y - r) * (int64_t)(y - r); };
  int32_t* s_col = a.stk_col + row;
  int32_t* s_from = a.stk_from + row;
  int32_t* s_r = a.stk_r + row;
  // stack entries 0..q-1 in memory, entry q (the top) in registers
  int q = 0;
  int32_t t_col = 0, t_from = 0, t_r = a.frow[row];
  for (int u = 1; u < W; ++u) {
    const int32_t ur = a.frow[row + (uint32_t)u];
    const int64_t fu = fr(ur);
    // pop the parabolas that u beats at the start of their range
    for (;;) {
      const int64_t dt = (int64_t)(t_from - t_col), du = (int64_t)(t_from - u);
      if (dt * dt + fr(t_r) <= du * du + fu) break;
      if (q == 0) {
        q = -1;
        break;
      }
      --q;
      t_col = s_col[q];
      t_from = s_from[q];
      t_r = s_r[q];
    }
    if (q < 0) {  // u beats everything: the envelope restarts with u alone
      q = 0;
      t_col = u;
      t_from = 0;
      t_r = ur;
      continue;
    }
    // the last x at which the top parabola is no worse than u's (floor division)
    const int64_t num = (int64_t)u * u - (int64_t)t_col * t_col + fu - fr(t_r);
    const int64_t den = 2 * (int64_t)(u - t_col);
    const int64_t sep = num >= 0 ? num / den : -((-num + den - 1) / den);
    if (1 + sep < W) {
      s_col[q] = t_col;
      s_from[q] = t_from;
      s_r[q] = t_r;
      ++q;
      t_col = u;
      t_from = (int32_t)(1 + sep);
      t_r = ur;
    }
  }
  for (int u = W - 1; u >= 0; --u) {
    if (t_r == kNone) {
      a.sqdist[row + (uint32_t)u] = -1;
      a.nearest[row + (uint32_t)u] = -1;
    } else {
      const int64_t dx = (int64_t)(u - t_col);
      a.sqdist[row + (uint32_t)u] = (int32_t)(dx * dx + fr(t_r));
      a.nearest[row + (uint32_t)u] = t_r * W + t_col;
    }
    if (u == t_from && q > 0) {
      --q;
      t_col = s_col[q];
      t_from = s_from[q];
      t_r = s_r[q];
    }
  }
}

}  // namespace xedt
}  // namespace iwpp

using namespace iwpp::rt;

extern "C" int32_t iwpp_edt_exact(iwpp_ctx* ctx, const uint8_t* binary, int32_t* sqdist, int32_t* nearest,
                                  int32_t height, int32_t width, void* stream) {
  using namespace iwpp;
  if (!ctx) return IWPP_EINVAL;
  if (ctx->server) return fail(ctx, IWPP_EBUSY, "edt_exact: the context is serving");
  if (!binary || !sqdist || !nearest) return fail(ctx, IWPP_EINVAL, "edt_exact: NULL image pointer");
  // the same argument rules as iwpp_edt (conn is irrelevant here)
  iwpp_job j{IWPP_OP_EDT, 8, height, width, binary, nullptr, sqdist, nearest};
  Plan plan;
  int32_t rc = build_plan(ctx, &j, 1, "edt_exact", plan);
  if (rc != IWPP_OK) return rc;
  const size_t np = (size_t)height * (size_t)width;
  const int nseg = (height + xedt::kSeg - 1) / xedt::kSeg;
  const size_t fb = align256(4 * np), sb = align256(4 * (size_t)nseg * (size_t)width);
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, IWPP_EDEVICE, "edt_exact: cannot select the context's device");
  if ((rc = ensure_scratch(ctx, 4 * fb + 2 * sb)) != IWPP_OK) return rc;
  xedt::XArgs a{};
  a.bin = binary;
  a.sqdist = sqdist;
  a.nearest = nearest;
  a.frow = reinterpret_cast<int32_t*>(ctx->scratch);
  a.stk_col = reinterpret_cast<int32_t*>(ctx->scratch + fb);
  a.stk_from = reinterpret_cast<int32_t*>(ctx->scratch + 2 * fb);
  a.stk_r = reinterpret_cast<int32_t*>(ctx->scratch + 3 * fb);
  a.first = reinterpret_cast<int32_t*>(ctx->scratch + 4 * fb);
  a.last = reinterpret_cast<int32_t*>(ctx->scratch + 4 * fb + sb);
  a.h = height;
  a.w = width;
  a.nseg = nseg;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 cg((unsigned)((width + 63) / 64), (unsigned)nseg);
  ctx->rec.begin(IWPP_K_XEDT, st);
  hipLaunchKernelGGL(xedt::k_col_summary, cg, dim3(64), 0, st, a);
  hipLaunchKernelGGL(xedt::k_col, cg, dim3(64), 0, st, a);
  hipLaunchKernelGGL(xedt::k_row, dim3((unsigned)((height + 63) / 64)), dim3(64), 0, st, a);
  ctx->rec.end(st);
  if (hipGetLastError() != hipSuccess) return fail(ctx, IWPP_EDEVICE, "edt_exact: launch failed");
  ctx->last_stream = st;
  ctx->last_fixed = ctx->fixed;
  ctx->last_op = 2;
  ctx->have_call = false;  // no counters: iwpp_get_stats reports zeros
  return IWPP_OK;
}
