// Grayscale morphological reconstruction by dilation on gfx950.
//
// What is computed (Sec. 2.1): rho_I(J), the limit of the elementary geodesic
// dilation J(p) <- max{J(q) : q in N_G(p) U {p}} ^ I(p).  The result is unique,
// so any schedule of valid updates that reaches stability gives identical
// bytes (the paper's exactness argument for Algorithm 5, which does hold here).
//
// How (the steps of Algorithm 5, re-planned for CDNA4):
//   1. seed pass   -- raster / anti-raster scans, split into row-wise and
//                     column-wise sweeps as Algorithm 5 does, run per 64x64
//                     tile in LDS and repeated until the tile is locally
//                     stable (one wave per tile, lane = row or column);
//   2. seed detect -- dense test of the full-neighbourhood seed condition of
//                     Algorithm 5 on every pixel; a tile holding a pixel that a
//                     neighbour can still raise goes on the first work list;
//   3. propagation -- one persistent, cooperative kernel works off the list in
//                     rounds (the queue swap of Algorithm 4): a wave loads a
//                     listed tile with its one-pixel halo, sweeps it to local
//                     stability, writes it back, and lists each neighbouring
//                     tile whose border pixels it can still raise.  Work lists
//                     are staged per wave in LDS and flushed with one atomic.
//   4. overflow    -- a work list has a capacity (the paper's fixed-size
//                     global queue, Sec. 3.2); an append past it is dropped and
//                     flagged, and the next round rebuilds its list by a dense
//                     seed detection over the current image, which is a valid
//                     restart point because every intermediate image is
//                     (Sec. 3.2: re-running from a partial output gives the same
//                     answer).
//
// The value updates are max-then-min of bytes; the per-tile state is owned by
// exactly one wave at a time (a tile is on a round's list at most once), so no
// atomics touch pixels.  Halo reads may see a neighbour mid-update; any value
// they see is a valid lower bound, and a border change always re-lists the
// neighbour for the next round, which then reads it after a grid barrier.
#include "iwpp_device.hpp"
#include "iwpp_internal.hpp"

namespace iwpp {
namespace mr {

constexpr int T = 64;          // tile side: lanes map to the 64 columns (or rows)
constexpr int kRows = T + 2;   // region rows with the halo
constexpr int P = 76;          // LDS row pitch: 19 dwords, so column walks hit distinct banks
constexpr int kOff = 4;        // LDS byte offset of tile column 0 (4-byte aligned chunks)
constexpr int kRegion = kRows * P;
constexpr int kWavesPerBlock = 4;
constexpr int kStageCap = 128;
constexpr uint32_t kMaxRounds = 1u << 20;

__device__ __forceinline__ int lidx(int y, int x) { return (y + 1) * P + x + kOff; }  // y, x in [-1, 64]

struct WaveLds {
  uint8_t J[kRegion];
  uint8_t I[kRegion];
};

typedef unsigned v4u __attribute__((ext_vector_type(4)));
typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t min_u8x4(uint32_t a, uint32_t b) {
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    uint32_t x = (a >> (8 * k)) & 0xffu, y = (b >> (8 * k)) & 0xffu;
    r |= (x < y ? x : y) << (8 * k);
  }
  return r;
}

__device__ __forceinline__ uint32_t umax(uint32_t a, uint32_t b) { return a > b ? a : b; }
__device__ __forceinline__ uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }

// Load the (T+2) x (T+2) region of tile (ty, tx) -- the tile and its one-pixel
// halo -- into LDS.  Pixels outside the image read as J = I = 0, which can
// neither raise nor be raised, i.e. they are not neighbours.  In the seed pass
// J is the marker clamped to the mask.
template <bool kSeed>
__device__ void load_region(const MrArgs& a, WaveLds& L, int ty, int tx) {
  const int y0 = ty * T, x0 = tx * T;
  const uint32_t total = (uint32_t)a.h * (uint32_t)a.w;
  const __amdgpu_buffer_rsrc_t rj = make_rsrc(kSeed ? a.marker : a.out, total);
  const __amdgpu_buffer_rsrc_t ri = make_rsrc(a.mask, total);
  for (int idx = lane(); idx < kRows * 5; idx += kWave) {
    const int ry = idx / 5, item = idx - ry * 5;
    const int y = y0 - 1 + ry;
    const bool row_ok = y >= 0 && y < a.h;
    if (item < 4) {
      const int xs = x0 + item * 16;
      v4u vj = {0u, 0u, 0u, 0u}, vi = {0u, 0u, 0u, 0u};
      if (row_ok && xs < a.w) {
        const uint32_t off = (uint32_t)y * (uint32_t)a.w + (uint32_t)xs;
        if (xs + 16 <= a.w) {
          vj = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(rj, off, 0, kSc1));
          vi = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(ri, off, 0, kSc1));
        } else {
          const int nb = a.w - xs;
#pragma unroll
          for (int b = 0; b < 16; ++b) {
            if (b < nb) {
              uint32_t jb = __builtin_amdgcn_raw_buffer_load_b8(rj, off + b, 0, kSc1);
              uint32_t ib = __builtin_amdgcn_raw_buffer_load_b8(ri, off + b, 0, kSc1);
              vj[b >> 2] |= jb << (8 * (b & 3));
              vi[b >> 2] |= ib << (8 * (b & 3));
            }
          }
        }
      }
      uint32_t* dj = reinterpret_cast<uint32_t*>(&L.J[lidx(ry - 1, item * 16)]);
      uint32_t* di = reinterpret_cast<uint32_t*>(&L.I[lidx(ry - 1, item * 16)]);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        dj[k] = kSeed ? min_u8x4(vj[k], vi[k]) : vj[k];
        di[k] = vi[k];
      }
    } else {
      uint32_t jl = 0, il = 0, jr = 0, ir = 0;
      if (row_ok && x0 > 0) {
        const uint32_t off = (uint32_t)y * (uint32_t)a.w + (uint32_t)(x0 - 1);
        jl = __builtin_amdgcn_raw_buffer_load_b8(rj, off, 0, kSc1);
        il = __builtin_amdgcn_raw_buffer_load_b8(ri, off, 0, kSc1);
      }
      if (row_ok && x0 + T < a.w) {
        const uint32_t off = (uint32_t)y * (uint32_t)a.w + (uint32_t)(x0 + T);
        jr = __builtin_amdgcn_raw_buffer_load_b8(rj, off, 0, kSc1);
        ir = __builtin_amdgcn_raw_buffer_load_b8(ri, off, 0, kSc1);
      }
      if (kSeed) {
        jl = umin(jl, il);
        jr = umin(jr, ir);
      }
      L.J[lidx(ry - 1, -1)] = (uint8_t)jl;
      L.I[lidx(ry - 1, -1)] = (uint8_t)il;
      L.J[lidx(ry - 1, T)] = (uint8_t)jr;
      L.I[lidx(ry - 1, T)] = (uint8_t)ir;
    }
  }
  wave_sync();
}

// Write the tile interior back to the image (device-coherent stores).
__device__ void store_tile(const MrArgs& a, const WaveLds& L, int ty, int tx) {
  const int y0 = ty * T, x0 = tx * T;
  const uint32_t total = (uint32_t)a.h * (uint32_t)a.w;
  const __amdgpu_buffer_rsrc_t ro = make_rsrc(a.out, total);
  for (int idx = lane(); idx < T * 4; idx += kWave) {
    const int ry = idx >> 2, c = idx & 3;
    const int y = y0 + ry, xs = x0 + c * 16;
    if (y >= a.h || xs >= a.w) continue;
    const uint32_t* s = reinterpret_cast<const uint32_t*>(&L.J[lidx(ry, c * 16)]);
    v4u v = {s[0], s[1], s[2], s[3]};
    const uint32_t off = (uint32_t)y * (uint32_t)a.w + (uint32_t)xs;
    if (xs + 16 <= a.w) {
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i, v), ro, off, 0, kSc1);
    } else {
      const int nb = a.w - xs;
#pragma unroll
      for (int b = 0; b < 16; ++b)
        if (b < nb)
          __builtin_amdgcn_raw_buffer_store_b8((unsigned char)(v[b >> 2] >> (8 * (b & 3))), ro, off + b, 0, kSc1);
    }
  }
}

// Sweep the tile in LDS until a full raster + anti-raster iteration changes
// nothing, or `max_it` iterations.  One iteration is the four axis scans of
// Algorithm 5 in its order: row-wise forward (N^{+,0}), column-wise forward
// (N^{0,+}), row-wise backward (N^{-,0}), column-wise backward (N^{0,-}).
// Every step is one elementary update J(p) <- max(J(p), J(q in the scan's
// neighbour set)) ^ I(p), so the tile never leaves [J ^ I, rho_I(J)].  Halo
// pixels are sources only.  Returns true if the tile is locally stable.
template <int CONN>
__device__ bool sweep_tile(WaveLds& L, int max_it, uint32_t& iters) {
  const int l = lane();
  const uint32_t hl = L.J[lidx(l, -1)], hr = L.J[lidx(l, T)];
  const uint32_t ctl = L.J[lidx(-1, -1)], ctr = L.J[lidx(-1, T)];
  const uint32_t cbl = L.J[lidx(T, -1)], cbr = L.J[lidx(T, T)];
  for (int it = 0; it < max_it; ++it) {
    bool ch = false;
    {  // row-wise, left to right: lane = row
      uint32_t prev = hl;
#pragma unroll
      for (int x = 0; x < T; ++x) {
        const uint32_t v = L.J[lidx(l, x)], i = L.I[lidx(l, x)];
        const uint32_t nv = umin(umax(v, prev), i);
        if (nv != v) {
          L.J[lidx(l, x)] = (uint8_t)nv;
          ch = true;
        }
        prev = nv;
      }
    }
    wave_sync();
    {  // column-wise, top to bottom: lane = column
      uint32_t prev = L.J[lidx(-1, l)];
#pragma unroll
      for (int y = 0; y < T; ++y) {
        const uint32_t v = L.J[lidx(y, l)], i = L.I[lidx(y, l)];
        uint32_t m = umax(v, prev);
        if (CONN == 8) {
          const uint32_t fl = y == 0 ? ctl : readlane(hl, y - 1);
          const uint32_t fr = y == 0 ? ctr : readlane(hr, y - 1);
          m = umax(m, umax(from_left(prev, fl), from_right(prev, fr)));
        }
        const uint32_t nv = umin(m, i);
        if (nv != v) {
          L.J[lidx(y, l)] = (uint8_t)nv;
          ch = true;
        }
        prev = nv;
      }
    }
    wave_sync();
    {  // row-wise, right to left
      uint32_t prev = hr;
#pragma unroll
      for (int x = T - 1; x >= 0; --x) {
        const uint32_t v = L.J[lidx(l, x)], i = L.I[lidx(l, x)];
        const uint32_t nv = umin(umax(v, prev), i);
        if (nv != v) {
          L.J[lidx(l, x)] = (uint8_t)nv;
          ch = true;
        }
        prev = nv;
      }
    }
    wave_sync();
    {  // column-wise, bottom to top
      uint32_t prev = L.J[lidx(T, l)];
#pragma unroll
      for (int y = T - 1; y >= 0; --y) {
        const uint32_t v = L.J[lidx(y, l)], i = L.I[lidx(y, l)];
        uint32_t m = umax(v, prev);
        if (CONN == 8) {
          const uint32_t fl = y == T - 1 ? cbl : readlane(hl, y + 1);
          const uint32_t fr = y == T - 1 ? cbr : readlane(hr, y + 1);
          m = umax(m, umax(from_left(prev, fl), from_right(prev, fr)));
        }
        const uint32_t nv = umin(m, i);
        if (nv != v) {
          L.J[lidx(y, l)] = (uint8_t)nv;
          ch = true;
        }
        prev = nv;
      }
    }
    wave_sync();
    iters++;
    if (ballot(ch) == 0) return true;
  }
  return false;
}

// Can the (possibly stale) halo pixel (qy, qx) be raised by interior value v?
// J(q) < min(v, I(q)) is the propagation condition of Algorithm 5; the halo J
// may only be lower than the truth, so "no" is always safe.
__device__ __forceinline__ bool halo_raisable(const WaveLds& L, int qy, int qx, uint32_t v) {
  const uint32_t jq = L.J[lidx(qy, qx)], iq = L.I[lidx(qy, qx)];
  return jq < umin(v, iq);
}

// Neighbouring tiles that a change of this visit can raise, as a bit mask:
// bit 0 top, 1 bottom, 2 left, 3 right, 4 top-left, 5 top-right,
// 6 bottom-left, 7 bottom-right.  o* are the border values before the visit.
template <int CONN>
__device__ uint32_t border_marks(const WaveLds& L, uint32_t ot, uint32_t ob, uint32_t ol, uint32_t orr) {
  const int l = lane();
  const uint32_t nt = L.J[lidx(0, l)], nb = L.J[lidx(T - 1, l)];
  const uint32_t nl = L.J[lidx(l, 0)], nr = L.J[lidx(l, T - 1)];
  bool t = false, b = false, lf = false, rt = false;
#pragma unroll
  for (int d = -1; d <= 1; ++d) {
    if (CONN == 4 && d != 0) continue;
    const int c = l + d;
    if (c < 0 || c >= T) continue;
    t |= nt > ot && halo_raisable(L, -1, c, nt);
    b |= nb > ob && halo_raisable(L, T, c, nb);
    lf |= nl > ol && halo_raisable(L, c, -1, nl);
    rt |= nr > orr && halo_raisable(L, c, T, nr);
  }
  uint32_t m = 0;
  if (ballot(t)) m |= 1u;
  if (ballot(b)) m |= 2u;
  if (ballot(lf)) m |= 4u;
  if (ballot(rt)) m |= 8u;
  if (CONN == 8) {
    const uint32_t c00 = L.J[lidx(0, 0)], c0e = L.J[lidx(0, T - 1)];
    const uint32_t ce0 = L.J[lidx(T - 1, 0)], cee = L.J[lidx(T - 1, T - 1)];
    const uint32_t o00 = readlane(ot, 0), o0e = readlane(ot, T - 1);
    const uint32_t oe0 = readlane(ob, 0), oee = readlane(ob, T - 1);
    if (c00 > o00 && halo_raisable(L, -1, -1, c00)) m |= 16u;
    if (c0e > o0e && halo_raisable(L, -1, T, c0e)) m |= 32u;
    if (ce0 > oe0 && halo_raisable(L, T, -1, ce0)) m |= 64u;
    if (cee > oee && halo_raisable(L, T, T, cee)) m |= 128u;
  }
  return m;
}

// ---- seed pass --------------------------------------------------------------------
// One wave per tile.  Also clears the work-list bookkeeping for this call.
template <int CONN>
__global__ __launch_bounds__(256) void k_seed(MrArgs a) {
  __shared__ WaveLds lds[kWavesPerBlock];
  const int w = threadIdx.x / kWave;
  const uint32_t t = blockIdx.x * kWavesPerBlock + w;
  if (blockIdx.x == 0 && threadIdx.x < 3 * 64) a.counts[threadIdx.x] = 0u;
  if (blockIdx.x == 0 && threadIdx.x < 2 * 64) a.lost[threadIdx.x] = 0u;
  if (blockIdx.x == 0) {
    uint32_t* bar = reinterpret_cast<uint32_t*>(a.bar);
    for (uint32_t i = threadIdx.x; i < sizeof(GridBarrier) / 4; i += blockDim.x) bar[i] = 0u;
  }
  if (t >= a.ntiles) return;
  if (lane() == 0) {
    a.flags[t] = 0u;
    a.flags[a.ntiles + t] = 0u;
  }
  const int ty = (int)(t / (uint32_t)a.tiles_x), tx = (int)(t % (uint32_t)a.tiles_x);
  WaveLds& L = lds[w];
  load_region<true>(a, L, ty, tx);
  uint32_t iters = 0;
  sweep_tile<CONN>(L, a.seed_sweeps, iters);
  store_tile(a, L, ty, tx);
  if (lane() == 0) stat_add(a.stats, kStatSweeps, iters);
}

// ---- seed detection -----------------------------------------------------------------
// Dense test of every pixel of tile (ty, tx).  Returns (wave-uniform) whether
// some pixel q of the tile can still be raised by a neighbour p, i.e.
// J(q) < J(p) and J(q) < I(q) -- the condition of Algorithm 5, read from the
// receiving side -- and adds to `seeds` the number of pixels p that meet
// Algorithm 5's seed condition (some neighbour q with J(q) < J(p) and
// J(q) < I(q)).  Loads are device-coherent: this also runs inside the
// persistent kernel.
struct RowVals {
  uint32_t j, i, jl, il, jr, ir;
};

__device__ __forceinline__ RowVals load_row(const MrArgs& a, __amdgpu_buffer_rsrc_t rj, __amdgpu_buffer_rsrc_t ri,
                                            int y, int x0) {
  RowVals r = {0u, 0u, 0u, 0u, 0u, 0u};
  if (y < 0 || y >= a.h) return r;
  const uint32_t rowoff = (uint32_t)y * (uint32_t)a.w;
  const int x = x0 + lane();
  if (x < a.w) {
    r.j = __builtin_amdgcn_raw_buffer_load_b8(rj, rowoff + x, 0, kSc1);
    r.i = __builtin_amdgcn_raw_buffer_load_b8(ri, rowoff + x, 0, kSc1);
  }
  if (x0 > 0) {
    r.jl = __builtin_amdgcn_raw_buffer_load_b8(rj, rowoff + x0 - 1, 0, kSc1);
    r.il = __builtin_amdgcn_raw_buffer_load_b8(ri, rowoff + x0 - 1, 0, kSc1);
  }
  if (x0 + T < a.w) {
    r.jr = __builtin_amdgcn_raw_buffer_load_b8(rj, rowoff + x0 + T, 0, kSc1);
    r.ir = __builtin_amdgcn_raw_buffer_load_b8(ri, rowoff + x0 + T, 0, kSc1);
  }
  return r;
}

// g(q) = J(q) if q can still rise (J(q) < I(q)), else 256 (never below J(p)).
__device__ __forceinline__ uint32_t gval(uint32_t j, uint32_t i) { return j < i ? j : 256u; }

template <int CONN>
__device__ bool detect_tile(const MrArgs& a, int ty, int tx, uint32_t& seeds) {
  const int y0 = ty * T, x0 = tx * T;
  const uint32_t total = (uint32_t)a.h * (uint32_t)a.w;
  const __amdgpu_buffer_rsrc_t rj = make_rsrc(a.out, total);
  const __amdgpu_buffer_rsrc_t ri = make_rsrc(a.mask, total);
  const bool col_ok = x0 + lane() < a.w;
  RowVals up = load_row(a, rj, ri, y0 - 1, x0);
  RowVals cur = load_row(a, rj, ri, y0, x0);
  bool any = false;
  const int rows = a.h - y0 < T ? a.h - y0 : T;
  for (int y = 0; y < rows; ++y) {
    RowVals dn = load_row(a, rj, ri, y0 + y + 1, x0);
    // receiving side: largest neighbour value
    uint32_t m = umax(umax(up.j, dn.j), umax(from_left(cur.j, cur.jl), from_right(cur.j, cur.jr)));
    // sending side: smallest raisable neighbour value
    uint32_t g = umin(umin(gval(up.j, up.i), gval(dn.j, dn.i)),
                      umin(from_left(gval(cur.j, cur.i), gval(cur.jl, cur.il)),
                           from_right(gval(cur.j, cur.i), gval(cur.jr, cur.ir))));
    if (CONN == 8) {
      m = umax(m, umax(umax(from_left(up.j, up.jl), from_right(up.j, up.jr)),
                       umax(from_left(dn.j, dn.jl), from_right(dn.j, dn.jr))));
      g = umin(g, umin(umin(from_left(gval(up.j, up.i), gval(up.jl, up.il)),
                            from_right(gval(up.j, up.i), gval(up.jr, up.ir))),
                       umin(from_left(gval(dn.j, dn.i), gval(dn.jl, dn.il)),
                            from_right(gval(dn.j, dn.i), gval(dn.jr, dn.ir)))));
    }
    const bool raisable = col_ok && cur.j < umin(m, cur.i);
    const bool seed = col_ok && cur.j > g;
    any |= raisable;
    seeds += (uint32_t)__popcll(ballot(seed));
    up = cur;
    cur = dn;
  }
  return ballot(any) != 0;
}

// Stage-flush variant for tile work lists: a dropped tile has its flag cleared
// (so a later mark can list it again) and the list's `lost` flag is raised,
// which makes a later round rebuild its list by dense detection.
__device__ void tile_flush(WaveStage& s, uint32_t* list, uint32_t* count, uint32_t cap, uint32_t* flags,
                           uint32_t* lost) {
  const uint32_t n = s.n;
  if (n == 0) return;
  wave_sync();
  uint32_t base = 0;
  if (lane() == 0) base = atomic_add(count, n);
  base = readlane(base, 0);
  bool dropped = false;
  for (uint32_t i = lane(); i < n; i += kWave) {
    const uint32_t slot = base + i, item = s.items[i];
    if (slot < cap) {
      cstore(list + slot, item);
    } else {
      cstore(flags + item, 0u);
      dropped = true;
    }
  }
  if (ballot(dropped) && lane() == 0) cstore(lost, 1u);
  wave_sync();
  s.n = 0;
}

// Put tile `t` (one per lane with pred) on the list of parity `par`, once.
__device__ __forceinline__ void mark_tiles(const MrArgs& a, WaveStage& s, bool pred, uint32_t t, int par,
                                           uint32_t* count) {
  bool fresh = false;
  if (pred) fresh = atomic_or(a.flags + (size_t)par * a.ntiles + t, 1u) == 0u;
  const uint64_t m = ballot(fresh);
  if (m == 0) return;
  const uint32_t k = (uint32_t)__popcll(m);
  if (s.n + k > s.cap) tile_flush(s, a.lists + (size_t)par * a.ntiles, count, a.list_cap, a.flags + (size_t)par * a.ntiles,
                                   a.lost + par * 64);
  if (fresh) s.items[s.n + mbcnt(m)] = t;
  s.n += k;
}

template <int CONN>
__global__ __launch_bounds__(256) void k_detect(MrArgs a) {
  __shared__ uint32_t stage_mem[kWavesPerBlock][kStageCap];
  const int w = threadIdx.x / kWave;
  WaveStage s = {stage_mem[w], (uint32_t)kStageCap, 0u};
  const uint32_t gw = blockIdx.x * kWavesPerBlock + w, nw = gridDim.x * kWavesPerBlock;
  uint32_t seeds = 0;
  for (uint32_t t = gw; t < a.ntiles; t += nw) {
    const int ty = (int)(t / (uint32_t)a.tiles_x), tx = (int)(t % (uint32_t)a.tiles_x);
    const bool any = detect_tile<CONN>(a, ty, tx, seeds);
    mark_tiles(a, s, any && lane() == 0, t, 0, a.counts);
  }
  tile_flush(s, a.lists, a.counts, a.list_cap, a.flags, a.lost);
  if (lane() == 0) stat_add(a.stats, kStatSeeds, seeds);
}

// ---- persistent propagation -----------------------------------------------------------
template <int CONN>
__global__ __launch_bounds__(256) void k_propagate(MrArgs a) {
  __shared__ WaveLds lds[kWavesPerBlock];
  __shared__ uint32_t stage_mem[kWavesPerBlock][kStageCap];
  __shared__ uint32_t decision[2];
  const int w = threadIdx.x / kWave;
  WaveLds& L = lds[w];
  WaveStage s = {stage_mem[w], (uint32_t)kStageCap, 0u};
  const uint32_t gw = blockIdx.x * kWavesPerBlock + w, nw = gridDim.x * kWavesPerBlock;
  uint32_t gen = 0;
  uint32_t visits = 0, iters = 0, rounds = 0, restarts = 0;
  for (uint32_t r = 0;; ++r) {
    const int par = (int)(r & 1u);
    uint32_t* count = a.counts + (r % 3u) * 64u;
    // Decide (identically in every workgroup) whether this round's list must be
    // rebuilt: a drop was recorded for it, or it is empty while a drop is still
    // pending for the other parity.  Nothing writes these words between the
    // last barrier and this read unless the decision is "rebuild".
    if (threadIdx.x == 0) {
      const uint32_t n = cload(count);
      const uint32_t lost_here = cload(a.lost + par * 64), lost_other = cload(a.lost + (1 - par) * 64);
      decision[0] = n;
      decision[1] = (lost_here != 0u) || (n == 0u && lost_other != 0u);
    }
    __syncthreads();
    uint32_t n = decision[0];
    if (decision[1]) {
      if (!grid_barrier(a.bar, gen, a.stats)) break;
      for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < 2u * a.ntiles; i += gridDim.x * blockDim.x)
        cstore(a.flags + i, 0u);
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        cstore(count, 0u);
        cstore(a.lost, 0u);
        cstore(a.lost + 64, 0u);
        restarts++;
      }
      if (!grid_barrier(a.bar, gen, a.stats)) break;
      uint32_t seeds = 0;
      for (uint32_t t = gw; t < a.ntiles; t += nw) {
        const int ty = (int)(t / (uint32_t)a.tiles_x), tx = (int)(t % (uint32_t)a.tiles_x);
        const bool any = detect_tile<CONN>(a, ty, tx, seeds);
        mark_tiles(a, s, any && lane() == 0, t, par, count);
      }
      tile_flush(s, a.lists + (size_t)par * a.ntiles, count, a.list_cap, a.flags + (size_t)par * a.ntiles,
                 a.lost + par * 64);
      if (!grid_barrier(a.bar, gen, a.stats)) break;
      if (threadIdx.x == 0) decision[0] = cload(count);
      __syncthreads();
      n = decision[0];
    }
    if (n == 0u) break;
    if (r >= kMaxRounds) {  // safety limit: report instead of spinning on a logic error
      if (blockIdx.x == 0 && threadIdx.x == 0) stat_add(a.stats, kStatError, 1ull);
      break;
    }
    if (n > a.list_cap) n = a.list_cap;
    // The count of round r+2 is reused: clear it now (it was last read in round
    // r-1, and is next appended to in round r+1, after this round's barrier).
    if (blockIdx.x == 0 && threadIdx.x == 0) cstore(a.counts + ((r + 2u) % 3u) * 64u, 0u);
    const int npar = 1 - par;
    uint32_t* ncount = a.counts + ((r + 1u) % 3u) * 64u;
    const uint32_t* list = a.lists + (size_t)par * a.ntiles;
    for (uint32_t i = gw; i < n; i += nw) {
      const uint32_t t = cload(list + i);
      if (lane() == 0) cstore(a.flags + (size_t)par * a.ntiles + t, 0u);
      const int ty = (int)(t / (uint32_t)a.tiles_x), tx = (int)(t % (uint32_t)a.tiles_x);
      load_region<false>(a, L, ty, tx);
      const int l = lane();
      const uint32_t ot = L.J[lidx(0, l)], ob = L.J[lidx(T - 1, l)];
      const uint32_t ol = L.J[lidx(l, 0)], orr = L.J[lidx(l, T - 1)];
      uint32_t it = 0;
      const bool stable = sweep_tile<CONN>(L, a.max_sweeps, it);
      iters += it;
      visits++;
      const bool changed = it > 1 || !stable;  // the first iteration changed something
      if (changed) store_tile(a, L, ty, tx);
      uint32_t m = changed ? border_marks<CONN>(L, ot, ob, ol, orr) : 0u;
      // Candidate tiles in lanes 0..8 (8 = this tile when not yet stable).
      int dy = 0, dx = 0;
      bool want = false;
      if (l < 8) {
        // bit order of border_marks: top, bottom, left, right, tl, tr, bl, br
        want = (m >> l) & 1u;
        dy = l < 2 ? (l == 0 ? -1 : 1) : (l < 4 ? 0 : (l < 6 ? -1 : 1));
        dx = l < 2 ? 0 : (l < 4 ? (l == 2 ? -1 : 1) : ((l & 1) ? 1 : -1));
      } else if (l == 8) {
        want = !stable;
      }
      const int ny = ty + dy, nx = tx + dx;
      want = want && ny >= 0 && ny < a.tiles_y && nx >= 0 && nx < a.tiles_x;
      mark_tiles(a, s, want, (uint32_t)(ny * a.tiles_x + nx), npar, ncount);
    }
    tile_flush(s, a.lists + (size_t)npar * a.ntiles, ncount, a.list_cap, a.flags + (size_t)npar * a.ntiles,
               a.lost + npar * 64);
    rounds++;
    if (!grid_barrier(a.bar, gen, a.stats)) break;
  }
  if (lane() == 0) {
    stat_add(a.stats, kStatItems, visits);
    stat_add(a.stats, kStatSweeps, iters);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    stat_add(a.stats, kStatRounds, rounds);
    stat_add(a.stats, kStatRestarts, restarts);
  }
}

}  // namespace mr

// ---- host-side launch -----------------------------------------------------------------
int mr_launch(const MrArgs& a, int conn, int persistent_blocks, hipStream_t stream, Recorder* rec, const char** err) {
  using namespace mr;
  const uint32_t seed_blocks = (a.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
  rec->begin(1, stream);
  if (conn == 8)
    hipLaunchKernelGGL(k_seed<8>, dim3(seed_blocks), dim3(256), 0, stream, a);
  else
    hipLaunchKernelGGL(k_seed<4>, dim3(seed_blocks), dim3(256), 0, stream, a);
  rec->end(stream);
  if (hipGetLastError() != hipSuccess) {
    *err = "seed-pass launch failed";
    return -1;
  }
  uint32_t det_blocks = seed_blocks < 2048u ? seed_blocks : 2048u;
  rec->begin(2, stream);
  if (conn == 8)
    hipLaunchKernelGGL(k_detect<8>, dim3(det_blocks), dim3(256), 0, stream, a);
  else
    hipLaunchKernelGGL(k_detect<4>, dim3(det_blocks), dim3(256), 0, stream, a);
  rec->end(stream);
  if (hipGetLastError() != hipSuccess) {
    *err = "seed-detect launch failed";
    return -1;
  }
  void* fn = conn == 8 ? reinterpret_cast<void*>(&k_propagate<8>) : reinterpret_cast<void*>(&k_propagate<4>);
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0) != hipSuccess || per_cu < 1) {
    *err = "occupancy query failed";
    return -1;
  }
  uint32_t blocks = persistent_grid(fn, per_cu, cus);
  if (persistent_blocks > 0 && (uint32_t)persistent_blocks < blocks) blocks = (uint32_t)persistent_blocks;
  MrArgs args = a;
  void* kargs[] = {&args};
  rec->begin(3, stream);
  const hipError_t le = hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(256), kargs, 0, stream);
  rec->end(stream);
  if (le != hipSuccess) {
    *err = "propagation launch failed";
    return -1;
  }
  return 0;
}

}  // namespace iwpp
