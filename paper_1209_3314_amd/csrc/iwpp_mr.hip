// Grayscale morphological reconstruction by dilation on gfx950.
//
// What is computed (Sec. 2.1): rho_I(J), the limit of the elementary geodesic
// dilation J(p) <- max{J(q) : q in N_G(p) U {p}} ^ I(p).  The result is unique,
// so any schedule of valid updates that reaches stability gives identical
// bytes (the paper's exactness argument for Algorithm 5, which does hold here).
//
// How (the steps of Algorithm 5, re-planned for CDNA4).  One persistent,
// cooperative kernel runs in rounds (the queue swap of Algorithm 4); a round
// visits tiles, one wave per 64x64 tile held in LDS with a one-pixel halo:
//   round 0  -- the seed pass: every tile is loaded from the marker (clamped
//               to the mask) and swept with Algorithm 5's raster and
//               anti-raster scans, split into row-wise and column-wise
//               sweeps, until it is locally stable (lane = row or column);
//   round r  -- each tile flagged in round r-1 is loaded from the current
//               image, swept to local stability and written back.
// After a visit the wave flags each neighbouring tile that a border change
// can still raise (Algorithm 5's propagation condition, J(q) < J(p) and
// J(q) < I(q), tested against the halo as loaded), and the tile itself if the
// sweep cap stopped it.  This replaces Algorithm 5's dense seed detection: in
// round 0 a halo pixel holds the neighbour's initial value, and a border pixel
// that did not rise was seen with that same value by the neighbour's own
// sweep, so only risen border pixels can leave a seed across a tile edge.
//
// The tile frontier of a round is a work list split into eight sub-lists, one
// per group of workgroups (one per XCD): a wave stages its appends in LDS and
// flushes them with one atomic on its group's counter, a per-tile flag keeps a
// tile on a round's list once, and the next round splits the concatenated
// sub-lists evenly over all waves, so a round's visits are balanced.  With a
// capacity (the paper's fixed-size global queue, Sec. 3.2) the list is one
// sub-list of that size: an append past it is dropped and flagged, and the
// next round becomes a full round that visits every tile holding a raisable
// pixel of the current image, which is a valid restart point because every
// intermediate image is (Sec. 3.2: re-running from a partial output gives the
// same answer).
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

constexpr int T = kMrTile;     // tile side: lanes map to the 64 columns (or rows)
static_assert(T == 64, "lanes map to tile rows and columns");
constexpr int kRows = T + 2;   // region rows with the halo
constexpr int P = 68;          // LDS row pitch: 17 dwords, so column walks hit distinct banks
constexpr int kOff = 4;        // LDS byte offset of tile column 0 (4-byte aligned chunks)
constexpr int kRegion = kRows * P + 4;  // the last row's column 64 spills into the pad
constexpr int kStageCap = 64;  // LDS work-list stage per wave (iwpp_options.stage_depth caps it)
constexpr uint32_t kMaxRounds = 1u << 20;

__device__ __forceinline__ int lidx(int y, int x) { return (y + 1) * P + x + kOff; }  // y, x in [-1, 64]
// Column 65 of rows -1..64 is never written by a tile load: it is cleared once
// per kernel and read as zeros (it shares bytes with no other column).
constexpr int kZeroCol = T + 1;

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

// A global tile id resolved to its image and tile coordinates (wave-uniform).
struct TileRef {
  MrJob j;
  int ty, tx;
};

__device__ __forceinline__ TileRef tile_ref(const MrArgs& a, uint32_t t) {
  TileRef r;
  r.j = uniform(a.njobs == 1u ? a.job0 : a.jobs[a.tile_job[t]]);
  const uint32_t lt = t - r.j.tile_base;
  r.ty = (int)(lt / (uint32_t)r.j.tiles_x);
  r.tx = (int)(lt - (uint32_t)r.ty * (uint32_t)r.j.tiles_x);
  return r;
}

// Offset that makes a raw buffer access fall outside every buffer (reads 0).
constexpr uint32_t kOutside = 0xFFFFFFF0u;

// Load the (T+2) x (T+2) region of tile (ty, tx) -- the tile and its one-pixel
// halo -- into LDS.  Pixels outside the image read as J = I = 0, which can
// neither raise nor be raised, i.e. they are not neighbours.  In the seed pass
// J is the marker clamped to the mask.  The 66 rows are 264 chunks of 16
// bytes (five per lane) plus 132 halo bytes, each read as the 4-byte word
// that ends at it (three per lane); every load is issued, with no branch in
// between, before the first LDS write, so a visit waits for memory once.
// Loads that would leave the image are pointed outside the buffer (they read
// 0; a raw buffer load that crosses the buffer's end reads 0 as a whole, so
// no load may reach past the image).  A chunk cut by the right edge of the
// image -- one chunk column of the tiles at that edge -- is read byte by byte
// in a second pass.
//
// Seed pass only: with `fresh_top` the halo row above the tile (its 64 bytes,
// not the corners) is read from the output, where the tile above has already
// been written by this wave; a value there is a valid lower bound of the
// result like any other, so it only lets the flood cross the edge earlier.
//
// Propagation rounds (not the seed pass) read the halo columns and corners
// from the neighbouring tiles' border-column blocks (`cols`, `cols_bytes`
// long, rewritten whenever a tile is written): one byte per lane from four
// 64-byte runs instead of 132 words from 66 image rows.
template <bool kSeed>
__device__ void load_region(const TileRef& tr, WaveLds& L, bool fresh_top = false, const uint8_t* cols = nullptr,
                            uint32_t cols_bytes = 0, uint32_t t = 0) {
  const MrJob& a = tr.j;
  const int y0 = tr.ty * T, x0 = tr.tx * T;
  // Buffer resources over the image rows the region touches, [yb, ye): offsets
  // stay 32-bit whatever the image size (a 66-row band of a row of up to 2^31
  // pixels), so images beyond 2^32 pixels are addressed like small ones.
  const int yb = y0 > 0 ? y0 - 1 : 0, ye = y0 + T + 1 < a.h ? y0 + T + 1 : a.h;
  const uint32_t band = (uint32_t)(ye - yb) * (uint32_t)a.w;
  const size_t base = (size_t)yb * (size_t)(uint32_t)a.w;
  const __amdgpu_buffer_rsrc_t rj = make_rsrc((kSeed ? a.marker : a.out) + base, band);
  const __amdgpu_buffer_rsrc_t ri = make_rsrc(a.mask + base, band);
  const __amdgpu_buffer_rsrc_t ro = make_rsrc(a.out + base, band);
  const int rem = a.w - x0;  // image columns from this tile's first column on
  const int cp = (rem < T && (rem & 15) != 0) ? rem >> 4 : -1;  // the cut chunk column, if any
  constexpr int kMain = kRows * 4, kHalo = kRows * 2;
  constexpr int kPerMain = (kMain + kWave - 1) / kWave, kPerHalo = (kHalo + kWave - 1) / kWave;
  v4u vj[kPerMain], vi[kPerMain];
  uint32_t hj[kPerHalo], hi[kPerHalo];
  uint32_t xm[kPerMain], xh[kPerHalo];  // complement of what was read inside the image (erosion), else 0
#pragma unroll
  for (int k = 0; k < kPerMain; ++k) {
    const int idx = lane() + k * kWave;
    const int c = idx & 3;
    const int y = y0 - 1 + (idx >> 2), xs = x0 + 16 * c;
    const bool ok = idx < kMain && y >= 0 && y < a.h && xs + 16 <= a.w;
    xm[k] = ok ? a.inv : 0u;
    const uint32_t off = ok ? (uint32_t)(y - yb) * (uint32_t)a.w + (uint32_t)xs : kOutside;
    vj[k] = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(rj, off, 0, kSc1));
    vi[k] = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(ri, off, 0, kSc1));
  }
  v4u vtop = {0u, 0u, 0u, 0u};
  if (kSeed && fresh_top) {  // wave-uniform; lanes 0..3 hold the row above
    const int y = y0 - 1, xs = x0 + 16 * (lane() & 3);
    const bool ok = lane() < 4 && y >= 0 && xs + 16 <= a.w;
    const uint32_t off = ok ? (uint32_t)(y - yb) * (uint32_t)a.w + (uint32_t)xs : kOutside;
    vtop = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(ro, off, 0, kSc1));
    // lanes 0..3 load the same chunks as vj[0] (row y0 - 1), so xm[0] applies
    if (lane() < 4) vj[0] = vtop;
  }
  if (kSeed) {
#pragma unroll
    for (int k = 0; k < kPerHalo; ++k) {
      const int idx = lane() + k * kWave;
      const int y = y0 - 1 + (idx >> 1);
      const int x = (idx & 1) ? x0 + T : x0 - 1;
      const bool ok = idx < kHalo && y >= 0 && y < a.h && x >= 3 && x < a.w;
      xh[k] = ok ? a.inv : 0u;
      const uint32_t off = ok ? (uint32_t)(y - yb) * (uint32_t)a.w + (uint32_t)(x - 3) : kOutside;
      hj[k] = __builtin_amdgcn_raw_buffer_load_b32(rj, off, 0, kSc1);
      hi[k] = __builtin_amdgcn_raw_buffer_load_b32(ri, off, 0, kSc1);
    }
  } else {
    // Lane l: row l of the left neighbour's right column and of the right
    // neighbour's left column (J and I); lanes 0..3 also one corner each:
    // top-left, top-right, bottom-left, bottom-right.
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(cols, cols_bytes);
    const int l = lane();
    const int tx_n = tr.j.tiles_x, ty_n = tr.j.tiles_y;
    const bool has_l = tr.tx > 0, has_r = tr.tx + 1 < tx_n;
    const uint32_t bl = (t - 1u) * 256u, br = (t + 1u) * 256u;
    const uint32_t ol = has_l ? bl + 64u + (uint32_t)l : kOutside, or_ = has_r ? br + (uint32_t)l : kOutside;
    hj[0] = __builtin_amdgcn_raw_buffer_load_b8(rc, ol, 0, kSc1);
    hi[0] = __builtin_amdgcn_raw_buffer_load_b8(rc, ol == kOutside ? kOutside : ol + 128u, 0, kSc1);
    hj[1] = __builtin_amdgcn_raw_buffer_load_b8(rc, or_, 0, kSc1);
    hi[1] = __builtin_amdgcn_raw_buffer_load_b8(rc, or_ == kOutside ? kOutside : or_ + 128u, 0, kSc1);
    const int cdy = (l & 2) ? 1 : -1, cdx = (l & 1) ? 1 : -1;
    const bool has_c = l < 4 && tr.ty + cdy >= 0 && tr.ty + cdy < ty_n && tr.tx + cdx >= 0 && tr.tx + cdx < tx_n;
    // the corner pixel is the diagonal tile's (right column if it lies left) row 63 (if above) or 0
    const uint32_t tc = (uint32_t)((int)t + cdy * tx_n + cdx);
    const uint32_t oc = has_c ? tc * 256u + (cdx < 0 ? 64u : 0u) + (cdy < 0 ? 63u : 0u) : kOutside;
    hj[2] = __builtin_amdgcn_raw_buffer_load_b8(rc, oc, 0, kSc1);
    hi[2] = __builtin_amdgcn_raw_buffer_load_b8(rc, oc == kOutside ? kOutside : oc + 128u, 0, kSc1);
  }
#pragma unroll
  for (int k = 0; k < kPerMain; ++k) {
    const int idx = lane() + k * kWave;
    if (idx >= kMain) continue;
    const int ry = idx >> 2, c = idx & 3;
    uint32_t* dj = reinterpret_cast<uint32_t*>(&L.J[lidx(ry - 1, c * 16)]);
    uint32_t* di = reinterpret_cast<uint32_t*>(&L.I[lidx(ry - 1, c * 16)]);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      dj[d] = kSeed ? min_u8x4(vj[k][d] ^ xm[k], vi[k][d] ^ xm[k]) : vj[k][d] ^ xm[k];
      di[d] = vi[k][d] ^ xm[k];
    }
  }
  if (kSeed) {
#pragma unroll
    for (int k = 0; k < kPerHalo; ++k) {
      const int idx = lane() + k * kWave;
      if (idx >= kHalo) continue;
      const int ry = idx >> 1;
      const uint32_t jb = (hj[k] ^ xh[k]) >> 24, ib = (hi[k] ^ xh[k]) >> 24;
      const int at = lidx(ry - 1, (idx & 1) ? T : -1);
      L.J[at] = (uint8_t)umin(jb, ib);
      L.I[at] = (uint8_t)ib;
    }
  } else {
    const int l = lane();
    L.J[lidx(l, -1)] = (uint8_t)hj[0];
    L.I[lidx(l, -1)] = (uint8_t)hi[0];
    L.J[lidx(l, T)] = (uint8_t)hj[1];
    L.I[lidx(l, T)] = (uint8_t)hi[1];
    if (l < 4) {
      const int at = lidx((l & 2) ? T : -1, (l & 1) ? T : -1);
      L.J[at] = (uint8_t)hj[2];
      L.I[at] = (uint8_t)hi[2];
    }
  }
  if (cp >= 0) {  // wave-uniform: only tiles cut by the right edge of the image
    const int nb = rem - 16 * cp, xs = x0 + 16 * cp;
#pragma unroll
    for (int k = 0; k < (kRows + kWave - 1) / kWave; ++k) {
      const int ry = lane() + k * kWave;
      const int y = y0 - 1 + ry;
      const bool row_ok = ry < kRows && y >= 0 && y < a.h;
      uint32_t bj[15], bi[15];
      const uint32_t xb = row_ok ? a.inv & 0xffu : 0u;
#pragma unroll
      for (int b = 0; b < 15; ++b) {
        const uint32_t off = (row_ok && b < nb) ? (uint32_t)(y - yb) * (uint32_t)a.w + (uint32_t)(xs + b) : kOutside;
        bj[b] = __builtin_amdgcn_raw_buffer_load_b8(rj, off, 0, kSc1) ^ xb;
        bi[b] = __builtin_amdgcn_raw_buffer_load_b8(ri, off, 0, kSc1) ^ xb;
      }
      if (ry < kRows) {
#pragma unroll
        for (int b = 0; b < 15; ++b) {
          if (b >= nb) break;
          const int at = lidx(ry - 1, 16 * cp + b);
          L.J[at] = (uint8_t)(kSeed ? umin(bj[b], bi[b]) : bj[b]);
          L.I[at] = (uint8_t)bi[b];
        }
      }
    }
  }
  wave_sync();
}

// Propagation visits load a tile in two parts, so that a listed tile that
// turns out to need no work costs a small fraction of a full load.
//
// The frame: everything the skip test (`border_raisable`) and the border
// marks read -- rows -1, 0, 63 and 64 of the region (J and I, one byte per
// lane and row from the image), the tile's own border columns 0 and 63 and
// the halo columns -1 and 64 (J and I, from the border-column blocks of the
// tile and of its left and right neighbours), and the four halo corners
// (from the diagonal neighbours' blocks).  Rows and columns outside the image
// read as 0.
__device__ void load_frame(const TileRef& tr, WaveLds& L, const uint8_t* cols, uint32_t cols_bytes, uint32_t t) {
  const MrJob& a = tr.j;
  const int y0 = tr.ty * T, x0 = tr.tx * T, l = lane();
  const int yb = y0 > 0 ? y0 - 1 : 0, ye = y0 + T + 1 < a.h ? y0 + T + 1 : a.h;
  const uint32_t band = (uint32_t)(ye - yb) * (uint32_t)a.w;
  const size_t base = (size_t)yb * (size_t)(uint32_t)a.w;
  const __amdgpu_buffer_rsrc_t ro = make_rsrc(a.out + base, band);
  const __amdgpu_buffer_rsrc_t ri = make_rsrc(a.mask + base, band);
  const __amdgpu_buffer_rsrc_t rc = make_rsrc(cols, cols_bytes);
  constexpr int kFrameRows[4] = {-1, 0, T - 1, T};
  uint32_t fj[4], fi[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int y = y0 + kFrameRows[k], x = x0 + l;
    const bool ok = y >= 0 && y < a.h && x < a.w;
    const uint32_t off = ok ? (uint32_t)(y - yb) * (uint32_t)a.w + (uint32_t)x : kOutside;
    const uint32_t xb = ok ? a.inv & 0xffu : 0u;
    fj[k] = __builtin_amdgcn_raw_buffer_load_b8(ro, off, 0, kSc1) ^ xb;
    fi[k] = __builtin_amdgcn_raw_buffer_load_b8(ri, off, 0, kSc1) ^ xb;
  }
  // Columns: own block [J left | J right | I left | I right], the left
  // neighbour's right column, the right neighbour's left column (lane = row).
  const uint32_t bo = t * 256u;
  const uint32_t oj0 = __builtin_amdgcn_raw_buffer_load_b8(rc, bo + (uint32_t)l, 0, kSc1);
  const uint32_t oj1 = __builtin_amdgcn_raw_buffer_load_b8(rc, bo + 64u + (uint32_t)l, 0, kSc1);
  const uint32_t oi0 = __builtin_amdgcn_raw_buffer_load_b8(rc, bo + 128u + (uint32_t)l, 0, kSc1);
  const uint32_t oi1 = __builtin_amdgcn_raw_buffer_load_b8(rc, bo + 192u + (uint32_t)l, 0, kSc1);
  const int tx_n = tr.j.tiles_x, ty_n = tr.j.tiles_y;
  const bool has_l = tr.tx > 0, has_r = tr.tx + 1 < tx_n;
  const uint32_t ol = has_l ? (t - 1u) * 256u + 64u + (uint32_t)l : kOutside;
  const uint32_t or_ = has_r ? (t + 1u) * 256u + (uint32_t)l : kOutside;
  const uint32_t hjl = __builtin_amdgcn_raw_buffer_load_b8(rc, ol, 0, kSc1);
  const uint32_t hil = __builtin_amdgcn_raw_buffer_load_b8(rc, ol == kOutside ? kOutside : ol + 128u, 0, kSc1);
  const uint32_t hjr = __builtin_amdgcn_raw_buffer_load_b8(rc, or_, 0, kSc1);
  const uint32_t hir = __builtin_amdgcn_raw_buffer_load_b8(rc, or_ == kOutside ? kOutside : or_ + 128u, 0, kSc1);
  // Corners, lanes 0..3: top-left, top-right, bottom-left, bottom-right.
  const int cdy = (l & 2) ? 1 : -1, cdx = (l & 1) ? 1 : -1;
  const bool has_c = l < 4 && tr.ty + cdy >= 0 && tr.ty + cdy < ty_n && tr.tx + cdx >= 0 && tr.tx + cdx < tx_n;
  const uint32_t tc = (uint32_t)((int)t + cdy * tx_n + cdx);
  const uint32_t oc = has_c ? tc * 256u + (cdx < 0 ? 64u : 0u) + (cdy < 0 ? 63u : 0u) : kOutside;
  const uint32_t cj = __builtin_amdgcn_raw_buffer_load_b8(rc, oc, 0, kSc1);
  const uint32_t ci = __builtin_amdgcn_raw_buffer_load_b8(rc, oc == kOutside ? kOutside : oc + 128u, 0, kSc1);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    L.J[lidx(kFrameRows[k], l)] = (uint8_t)fj[k];
    L.I[lidx(kFrameRows[k], l)] = (uint8_t)fi[k];
  }
  L.J[lidx(l, 0)] = (uint8_t)oj0;
  L.J[lidx(l, T - 1)] = (uint8_t)oj1;
  L.I[lidx(l, 0)] = (uint8_t)oi0;
  L.I[lidx(l, T - 1)] = (uint8_t)oi1;
  L.J[lidx(l, -1)] = (uint8_t)hjl;
  L.I[lidx(l, -1)] = (uint8_t)hil;
  L.J[lidx(l, T)] = (uint8_t)hjr;
  L.I[lidx(l, T)] = (uint8_t)hir;
  if (l < 4) {
    const int at = lidx((l & 2) ? T : -1, (l & 1) ? T : -1);
    L.J[at] = (uint8_t)cj;
    L.I[at] = (uint8_t)ci;
  }
  wave_sync();
}

// The rest of a propagation visit's region: rows 1..62 of the tile (J and I),
// as 16-byte chunks (four per row), and byte by byte where a chunk is cut by
// the image's right edge (see load_region).
__device__ void load_interior(const TileRef& tr, WaveLds& L) {
  const MrJob& a = tr.j;
  const int y0 = tr.ty * T, x0 = tr.tx * T;
  const int yb = y0 > 0 ? y0 - 1 : 0, ye = y0 + T + 1 < a.h ? y0 + T + 1 : a.h;
  const uint32_t band = (uint32_t)(ye - yb) * (uint32_t)a.w;
  const size_t base = (size_t)yb * (size_t)(uint32_t)a.w;
  const __amdgpu_buffer_rsrc_t rj = make_rsrc(a.out + base, band);
  const __amdgpu_buffer_rsrc_t ri = make_rsrc(a.mask + base, band);
  const int rem = a.w - x0;
  const int cp = (rem < T && (rem & 15) != 0) ? rem >> 4 : -1;
  constexpr int kChunks = (T - 2) * 4;
  constexpr int kPer = (kChunks + kWave - 1) / kWave;
  v4u vj[kPer], vi[kPer];
  uint32_t xm[kPer];  // complement of what was read inside the image (erosion), else 0
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int idx = lane() + k * kWave;
    const int c = idx & 3;
    const int y = y0 + 1 + (idx >> 2), xs = x0 + 16 * c;
    const bool ok = idx < kChunks && y < a.h && xs + 16 <= a.w;
    xm[k] = ok ? a.inv : 0u;
    const uint32_t off = ok ? (uint32_t)(y - yb) * (uint32_t)a.w + (uint32_t)xs : kOutside;
    vj[k] = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(rj, off, 0, kSc1));
    vi[k] = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(ri, off, 0, kSc1));
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int idx = lane() + k * kWave;
    if (idx >= kChunks) continue;
    const int ry = 1 + (idx >> 2), c = idx & 3;
    uint32_t* dj = reinterpret_cast<uint32_t*>(&L.J[lidx(ry, c * 16)]);
    uint32_t* di = reinterpret_cast<uint32_t*>(&L.I[lidx(ry, c * 16)]);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      dj[d] = vj[k][d] ^ xm[k];
      di[d] = vi[k][d] ^ xm[k];
    }
  }
  if (cp >= 0) {  // wave-uniform: only tiles cut by the right edge of the image
    const int nb = rem - 16 * cp, xs = x0 + 16 * cp;
    const int ry = 1 + lane();
    const int y = y0 + ry;
    const bool row_ok = ry < T - 1 && y < a.h;
    uint32_t bj[15], bi[15];
    const uint32_t xb = row_ok ? a.inv & 0xffu : 0u;
#pragma unroll
    for (int b = 0; b < 15; ++b) {
      const uint32_t off = (row_ok && b < nb) ? (uint32_t)(y - yb) * (uint32_t)a.w + (uint32_t)(xs + b) : kOutside;
      bj[b] = __builtin_amdgcn_raw_buffer_load_b8(rj, off, 0, kSc1) ^ xb;
      bi[b] = __builtin_amdgcn_raw_buffer_load_b8(ri, off, 0, kSc1) ^ xb;
    }
    if (ry < T - 1) {
#pragma unroll
      for (int b = 0; b < 15; ++b) {
        if (b >= nb) break;
        const int at = lidx(ry, 16 * cp + b);
        L.J[at] = (uint8_t)bj[b];
        L.I[at] = (uint8_t)bi[b];
      }
    }
  }
  wave_sync();
}

// Write the tile interior back to the image (device-coherent stores).
__device__ void store_tile(const TileRef& tr, const WaveLds& L) {
  const MrJob& a = tr.j;
  const int y0 = tr.ty * T, x0 = tr.tx * T;
  const int ye = y0 + T < a.h ? y0 + T : a.h;  // the tile's rows, as a band of their own (see load_region)
  const __amdgpu_buffer_rsrc_t ro =
      make_rsrc(a.out + (size_t)y0 * (size_t)(uint32_t)a.w, (uint32_t)(ye - y0) * (uint32_t)a.w);
  for (int idx = lane(); idx < T * 4; idx += kWave) {
    const int ry = idx >> 2, c = idx & 3;
    const int y = y0 + ry, xs = x0 + c * 16;
    if (y >= a.h || xs >= a.w) continue;
    const uint32_t* s = reinterpret_cast<const uint32_t*>(&L.J[lidx(ry, c * 16)]);
    v4u v = {s[0] ^ a.inv, s[1] ^ a.inv, s[2] ^ a.inv, s[3] ^ a.inv};
    const uint32_t off = (uint32_t)ry * (uint32_t)a.w + (uint32_t)xs;
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

// Write the tile's border columns (J, and with `mask` also I) into its block
// of `cols`: [J left | J right | I left | I right], 64 bytes each.
__device__ void store_cols(const MrArgs& a, uint32_t t, const WaveLds& L, bool mask) {
  const __amdgpu_buffer_rsrc_t rc = make_rsrc(a.cols + (size_t)t * 256u, 256u);
  const int l = lane();
  __builtin_amdgcn_raw_buffer_store_b8(L.J[lidx(l, 0)], rc, (uint32_t)l, 0, kSc1);
  __builtin_amdgcn_raw_buffer_store_b8(L.J[lidx(l, T - 1)], rc, 64u + (uint32_t)l, 0, kSc1);
  if (mask) {
    __builtin_amdgcn_raw_buffer_store_b8(L.I[lidx(l, 0)], rc, 128u + (uint32_t)l, 0, kSc1);
    __builtin_amdgcn_raw_buffer_store_b8(L.I[lidx(l, T - 1)], rc, 192u + (uint32_t)l, 0, kSc1);
  }
}

// Rows and columns of the tile that changed since each axis scan last ran
// (bit = row or column index, wave-uniform).  After a scan in direction D
// every pixel dominates the offers of its D-predecessors (the pixel before it
// along D: left for rows forward, right for rows backward, the row above --
// three pixels with 8-connectivity -- for columns forward, the row below for
// columns backward), and it keeps dominating them until one of those
// predecessors rises.  So a scan only needs the 16-wide chunks whose
// predecessors changed since it last ran, plus any chunk after one that it
// has just changed; and the tile is locally stable exactly when all four sets
// are empty (the four scans' predecessors are all eight neighbours, or all
// four).  Changes made by a row scan are known per row (lane = row) and per
// chunk of columns; those of a column scan per column and per chunk of rows.
struct Dirty {
  uint64_t r_cf, r_cb;  // rows changed since the last column scan forward / backward
  uint64_t c_rf, c_rb;  // columns changed since the last row scan forward / backward
  __device__ bool empty() const { return (r_cf | r_cb | c_rf | c_rb) == 0ull; }
};

// Apply every halo pixel's offer to the border pixels it touches, once:
// J(p) <- max(J(p), min(J(h), I(p))) for border pixel p and halo neighbour h.
// Halo pixels do not change during a visit and J only rises, so afterwards no
// halo offer can raise anything again and the scans can ignore the halo (it
// acts as zeros there).  Rows first, then columns, so a corner pixel takes
// both.  Sets the rows and the columns that hold a border pixel that rose.
template <int CONN>
__device__ void fold_halo(WaveLds& L, uint64_t& rows, uint64_t& cols) {
  const int l = lane();
  auto offer = [&](int hy0, int hx0, int hy1, int hx1, int hy2, int hx2) {  // max of the halo neighbours
    uint32_t h = L.J[lidx(hy1, hx1)];
    if (CONN == 8) h = umax(h, umax((uint32_t)L.J[lidx(hy0, hx0)], (uint32_t)L.J[lidx(hy2, hx2)]));
    return h;
  };
  const uint32_t ht = offer(-1, l - 1, -1, l, -1, l + 1), hb = offer(T, l - 1, T, l, T, l + 1);
  const uint32_t jt = L.J[lidx(0, l)], it = L.I[lidx(0, l)], jb = L.J[lidx(T - 1, l)], ib = L.I[lidx(T - 1, l)];
  const uint32_t nt = umax(jt, umin(ht, it)), nb = umax(jb, umin(hb, ib));
  L.J[lidx(0, l)] = (uint8_t)nt;
  L.J[lidx(T - 1, l)] = (uint8_t)nb;
  const uint64_t top = ballot(nt != jt), bot = ballot(nb != jb);  // lane = column
  // The column phase reads corners that other lanes wrote in the row phase
  // (lane 63 wrote (0, 63), lane 0 wrote (63, 0)): order the two phases.
  wave_sync();
  const uint32_t hl = offer(l - 1, -1, l, -1, l + 1, -1), hr = offer(l - 1, T, l, T, l + 1, T);
  const uint32_t jl = L.J[lidx(l, 0)], il = L.I[lidx(l, 0)], jr = L.J[lidx(l, T - 1)], ir = L.I[lidx(l, T - 1)];
  const uint32_t nl = umax(jl, umin(hl, il)), nr = umax(jr, umin(hr, ir));
  L.J[lidx(l, 0)] = (uint8_t)nl;
  L.J[lidx(l, T - 1)] = (uint8_t)nr;
  const uint64_t left = ballot(nl != jl), right = ballot(nr != jr);  // lane = row
  wave_sync();
  rows = left | right | (top ? 1ull : 0ull) | (bot ? 1ull << (T - 1) : 0ull);
  cols = top | bot | (left ? 1ull : 0ull) | (right ? 1ull << (T - 1) : 0ull);
}

// One axis scan of the tile in LDS, after `fold_halo`: the halo is ignored.
// Vertical scans walk the rows with lane = column, using the previous row's
// values of the three (8-conn) or one (4-conn) upper/lower neighbours;
// horizontal scans walk the columns with lane = row, using the previous
// column.  Steps are loaded from LDS in chunks of kChunk so the wave pays one
// LDS latency per chunk rather than per step; a chunk's results are written
// back if any of them changed, and increases accumulate in `ch`.  A chunk
// whose predecessors did not change since this scan last ran (`Dirty`), and
// that follows no chunk this scan changed, is skipped; the chunk after a
// skipped one reads its carried-in neighbour values from LDS.
constexpr int kChunk = 16;
static_assert(T == 4 * kChunk, "four chunks per scan");

// Predecessor lines of chunk [x0, x0 + 16) in the scan's direction.
__device__ __forceinline__ uint64_t chunk_preds(int x0, bool forward) {
  const uint64_t w = 0xFFFFull << x0;
  return forward ? w >> 1 : w << 1;
}

// Row scans (lane = row) on packed words: one step is a byte-selecting max of
// the old pixel and the previous result, then a byte-selecting min with the
// mask written into the pixel's byte in place (SDWA with the other bytes
// preserved), two instructions per pixel with no unpacking or repacking.
// MR_HSTEP: pixel byte K of word W, previous result in byte PK of word PW.
#define MR_HSTEP(W, PW, I, K, PK)                                                                       \
  do {                                                                                                  \
    uint32_t m_;                                                                                        \
    asm("v_max_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_" #K              \
        " src1_sel:BYTE_" #PK                                                                           \
        : "=v"(m_)                                                                                      \
        : "v"(W), "v"(PW));                                                                             \
    asm("v_min_u32_sdwa %0, %1, %2 dst_sel:BYTE_" #K " dst_unused:UNUSED_PRESERVE src0_sel:DWORD"      \
        " src1_sel:BYTE_" #K                                                                            \
        : "+v"(W)                                                                                       \
        : "v"(m_), "v"(I));                                                                             \
  } while (0)

template <bool kForward, bool kDirty>
__device__ __forceinline__ void row_scan(WaveLds& L, uint32_t& ch, Dirty& dm) {
  const int l = lane();
  uint64_t& mine = kForward ? dm.c_rf : dm.c_rb;
  uint64_t& other = kForward ? dm.c_rb : dm.c_rf;
  uint32_t pw = 0;  // word holding the previous result: byte 3 (forward) or byte 0 (backward)
  bool carried = true;  // pw holds the previous chunk's result (the halo's zero before the first)
  bool carry = false;   // the previous chunk changed
  uint32_t acc = 0;
#pragma unroll 1
  for (int c = 0; c < T / kChunk; ++c) {
    const int x0 = (kForward ? c : T / kChunk - 1 - c) * kChunk;
    if (kDirty && !carry && (mine & chunk_preds(x0, kForward)) == 0ull) {
      carried = false;
      continue;
    }
    uint32_t* jp = reinterpret_cast<uint32_t*>(&L.J[lidx(l, x0)]);
    const uint32_t* ip = reinterpret_cast<const uint32_t*>(&L.I[lidx(l, x0)]);
    if (!carried) pw = kForward ? jp[-1] : jp[4];
    uint32_t w0 = jp[0], w1 = jp[1], w2 = jp[2], w3 = jp[3];
    const uint32_t o0 = w0, o1 = w1, o2 = w2, o3 = w3;
    const uint32_t i0 = ip[0], i1 = ip[1], i2 = ip[2], i3 = ip[3];
    if (kForward) {
      MR_HSTEP(w0, pw, i0, 0, 3); MR_HSTEP(w0, w0, i0, 1, 0); MR_HSTEP(w0, w0, i0, 2, 1); MR_HSTEP(w0, w0, i0, 3, 2);
      MR_HSTEP(w1, w0, i1, 0, 3); MR_HSTEP(w1, w1, i1, 1, 0); MR_HSTEP(w1, w1, i1, 2, 1); MR_HSTEP(w1, w1, i1, 3, 2);
      MR_HSTEP(w2, w1, i2, 0, 3); MR_HSTEP(w2, w2, i2, 1, 0); MR_HSTEP(w2, w2, i2, 2, 1); MR_HSTEP(w2, w2, i2, 3, 2);
      MR_HSTEP(w3, w2, i3, 0, 3); MR_HSTEP(w3, w3, i3, 1, 0); MR_HSTEP(w3, w3, i3, 2, 1); MR_HSTEP(w3, w3, i3, 3, 2);
      pw = w3;
    } else {
      MR_HSTEP(w3, pw, i3, 3, 0); MR_HSTEP(w3, w3, i3, 2, 3); MR_HSTEP(w3, w3, i3, 1, 2); MR_HSTEP(w3, w3, i3, 0, 1);
      MR_HSTEP(w2, w3, i2, 3, 0); MR_HSTEP(w2, w2, i2, 2, 3); MR_HSTEP(w2, w2, i2, 1, 2); MR_HSTEP(w2, w2, i2, 0, 1);
      MR_HSTEP(w1, w2, i1, 3, 0); MR_HSTEP(w1, w1, i1, 2, 3); MR_HSTEP(w1, w1, i1, 1, 2); MR_HSTEP(w1, w1, i1, 0, 1);
      MR_HSTEP(w0, w1, i0, 3, 0); MR_HSTEP(w0, w0, i0, 2, 3); MR_HSTEP(w0, w0, i0, 1, 2); MR_HSTEP(w0, w0, i0, 0, 1);
      pw = w0;
    }
    carried = true;
    const uint32_t d = (o0 ^ w0) | (o1 ^ w1) | (o2 ^ w2) | (o3 ^ w3);
    const uint64_t rows = ballot(d != 0u);
    carry = rows != 0ull;
    if (carry) {  // a chunk that changed nothing is not written back
      jp[0] = w0;
      jp[1] = w1;
      jp[2] = w2;
      jp[3] = w3;
      if (kDirty) {
        dm.r_cf |= rows;
        dm.r_cb |= rows;
        other |= 0xFFFFull << x0;
      }
    }
    acc |= d;
  }
  mine = 0ull;
  ch |= acc;
  wave_sync();
}
#undef MR_HSTEP

// min(v, byte B of w) for a byte-sized v (SDWA selects the mask byte).
template <int B>
__device__ __forceinline__ uint32_t min_byte(uint32_t v, uint32_t w) {
  uint32_t r;
  if (B == 0)
    asm("v_min_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0" : "=v"(r) : "v"(v), "v"(w));
  else if (B == 1)
    asm("v_min_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1" : "=v"(r) : "v"(v), "v"(w));
  else if (B == 2)
    asm("v_min_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2" : "=v"(r) : "v"(v), "v"(w));
  else
    asm("v_min_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_3" : "=v"(r) : "v"(v), "v"(w));
  return r;
}

// The tile's mask column of this lane, four rows per word (row 4w + b in byte
// b of ic[w]): the mask does not change during a visit, so the column scans
// take it from registers and read only J from LDS.
__device__ __forceinline__ void load_mask_column(const WaveLds& L, uint32_t (&ic)[T / 4]) {
  const int l = lane();
#pragma unroll
  for (int w = 0; w < T / 4; ++w) {
    const uint32_t b0 = L.I[lidx(4 * w, l)], b1 = L.I[lidx(4 * w + 1, l)], b2 = L.I[lidx(4 * w + 2, l)],
                   b3 = L.I[lidx(4 * w + 3, l)];
    ic[w] = b0 | (b1 << 8) | (b2 << 16) | (b3 << 24);
  }
}

template <int CONN, bool kForward, bool kDirty, int C>
__device__ __forceinline__ void column_chunk(WaveLds& L, uint32_t& ch, Dirty& dm, const uint32_t (&ic)[T / 4],
                                             uint32_t& prev, bool& carried, bool& carry) {
  const int l = lane();
  constexpr int y0 = (kForward ? C : T / kChunk - 1 - C) * kChunk;
  uint64_t& mine = kForward ? dm.r_cf : dm.r_cb;
  uint64_t& other = kForward ? dm.r_cb : dm.r_cf;
  if (kDirty && !carry && (mine & chunk_preds(y0, kForward)) == 0ull) {
    carried = false;
    return;
  }
  if (!carried) prev = L.J[lidx(kForward ? y0 - 1 : y0 + kChunk, l)];
  uint32_t vj[kChunk];
  const uint32_t ch0 = ch;
#pragma unroll
  for (int k = 0; k < kChunk; ++k) {
    const int s = kForward ? y0 + k : y0 + kChunk - 1 - k;
    vj[k] = L.J[lidx(s, l)];
  }
#pragma unroll
  for (int k = 0; k < kChunk; ++k) {
    const int s = kForward ? y0 + k : y0 + kChunk - 1 - k;
    const uint32_t iw = ic[s / 4];
    uint32_t m;
    if (CONN == 8) {
      // The two lane shifts of the diagonal offers are fused into the max
      // (DPP with zero fill; the s_nop gives the two wait states a DPP read
      // of a just-written register needs).
      uint32_t ml, mr;
      asm("s_nop 1\n\t"
          "v_max_u32_dpp %0, %2, %3 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_max_u32_dpp %1, %2, %2 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
          : "=&v"(ml), "=&v"(mr)
          : "v"(prev), "v"(vj[k]));
      m = umax(ml, mr);
    } else {
      m = umax(vj[k], prev);
    }
    // J <= I throughout, so min(max(J, offers), I) is the update.
    uint32_t nv;
    switch (s & 3) {
      case 0: nv = min_byte<0>(m, iw); break;
      case 1: nv = min_byte<1>(m, iw); break;
      case 2: nv = min_byte<2>(m, iw); break;
      default: nv = min_byte<3>(m, iw); break;
    }
    // Values only rise, so the sum of increases is nonzero iff something changed.
    ch += nv - vj[k];
    vj[k] = nv;
    prev = nv;
  }
  carried = true;
  const uint64_t cols = ballot(ch != ch0);
  carry = cols != 0ull;
  if (carry) {  // a chunk that changed nothing is not written back
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      const int s = kForward ? y0 + k : y0 + kChunk - 1 - k;
      L.J[lidx(s, l)] = (uint8_t)vj[k];
    }
    if (kDirty) {
      dm.c_rf |= cols;
      dm.c_rb |= cols;
      other |= 0xFFFFull << y0;
    }
  }
  asm volatile("" ::: "memory");  // keep chunks apart: bounded register use
}

template <int CONN, bool kVertical, bool kForward, bool kDirty>
__device__ __forceinline__ void scan(WaveLds& L, uint32_t& ch, Dirty& dm, const uint32_t (&ic)[T / 4]) {
  if (!kVertical) {
    row_scan<kForward, kDirty>(L, ch, dm);
    return;
  }
  uint32_t prev = 0;
  bool carried = true;  // prev holds the previous chunk's last row (the halo's zero before the first)
  bool carry = false;   // the previous chunk changed
  column_chunk<CONN, kForward, kDirty, 0>(L, ch, dm, ic, prev, carried, carry);
  column_chunk<CONN, kForward, kDirty, 1>(L, ch, dm, ic, prev, carried, carry);
  column_chunk<CONN, kForward, kDirty, 2>(L, ch, dm, ic, prev, carried, carry);
  column_chunk<CONN, kForward, kDirty, 3>(L, ch, dm, ic, prev, carried, carry);
  (kForward ? dm.r_cf : dm.r_cb) = 0ull;
  wave_sync();
}

// Sweep the tile in LDS until it is locally stable, or `max_it` iterations.
// One iteration is the four axis scans of Algorithm 5 in its order: row-wise
// forward (N^{+,0}), column-wise forward (N^{0,+}), row-wise backward
// (N^{-,0}), column-wise backward (N^{0,-}).  Every step is one elementary
// update J(p) <- max(J(p), J(q in the scan's neighbour set)) ^ I(p), so the
// tile never leaves [J ^ I, rho_I(J)].  Halo pixels are sources only, and
// `fold_halo` applies all their offers before the first scan.
//
// When the sweep stops.  With 8-connectivity the scans track what changed
// (`Dirty`): a scan with nothing to do costs nothing, and the tile is stable
// when no scan has anything left.  `all_dirty`: the tile as loaded is not
// known to be locally stable (a seed-pass tile, a tile the sweep cap stopped,
// a full round); otherwise its last visit left it stable and only the border
// pixels the halo raised start dirty.  With 4-connectivity changes spread
// over most of a tile and the bookkeeping measured slower (1.86 against
// 1.84 ms on the 16384^2 workload, against 1.54 and 1.65 ms with
// 8-connectivity): there four consecutive scans that change nothing (one of
// each direction, in any phase) mean every pixel dominates each of its
// neighbours' offers; after a scan that changed pixels three suffice, since
// that scan left its own direction satisfied and nothing has risen since.  Returns true if the tile is locally stable;
// `changed` tells whether any pixel rose.
template <int CONN>
__device__ bool sweep_tile(WaveLds& L, int max_it, uint32_t& iters, bool& changed, bool all_dirty, int start = 0) {
  constexpr bool kDirty = CONN == 8;
  uint64_t rows, cols;
  fold_halo<CONN>(L, rows, cols);
  changed = (rows | cols) != 0ull;
  Dirty dm;
  if (all_dirty || !kDirty) {
    dm.r_cf = dm.r_cb = dm.c_rf = dm.c_rb = ~0ull;
  } else {
    dm.r_cf = dm.r_cb = rows;
    dm.c_rf = dm.c_rb = cols;
  }
  uint32_t ic[T / 4];
  load_mask_column(L, ic);
  int quiet = 0;        // consecutive scans that changed nothing (4-connectivity)
  bool scanned = false;  // some scan of this visit changed a pixel
  // `start` picks the first scan (0 rows forward, 1 columns forward, 2 rows
  // backward, 3 columns backward), e.g. the one that carries a raised halo
  // side into the tile; the cyclic order is Algorithm 5's.
  for (int n = 0; n < 4 * max_it; ++n) {
    if (kDirty && dm.empty()) return true;
    if ((n & 3) == 0) iters++;
    uint32_t ch = 0;
    switch ((start + n) & 3) {
      case 0: if (!kDirty || dm.c_rf) scan<CONN, false, true, kDirty>(L, ch, dm, ic); break;
      case 1: if (!kDirty || dm.r_cf) scan<CONN, true, true, kDirty>(L, ch, dm, ic); break;
      case 2: if (!kDirty || dm.c_rb) scan<CONN, false, false, kDirty>(L, ch, dm, ic); break;
      default: if (!kDirty || dm.r_cb) scan<CONN, true, false, kDirty>(L, ch, dm, ic); break;
    }
    if (ballot(ch != 0u) != 0u) {
      changed = true;
      scanned = true;
      quiet = 0;
    } else if (!kDirty && ++quiet == (scanned ? 3 : 4)) {
      return true;
    }
  }
  return kDirty && dm.empty();
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

// Which sides' halo pixels can raise a border pixel of the tile?  (Algorithm
// 5's propagation condition read from the receiving side: J(p) < J(h) and
// J(p) < I(p), for p on the border and h a halo neighbour of p.)  A tile that
// was locally stable after its last visit can only have become raisable this
// way, because only its halo changed since.  Wave-uniform bit mask.
template <int CONN>
__device__ uint32_t border_raisable(const WaveLds& L) {
  const int l = lane();
  bool rt = false, rb = false, rl = false, rr = false;
  // p on row 0 (halo row -1), row T-1 (halo row T), column 0 (halo column -1), column T-1 (halo column T)
  const uint32_t pt = L.J[lidx(0, l)], it = L.I[lidx(0, l)];
  const uint32_t pb = L.J[lidx(T - 1, l)], ib = L.I[lidx(T - 1, l)];
  const uint32_t pl = L.J[lidx(l, 0)], il = L.I[lidx(l, 0)];
  const uint32_t pr = L.J[lidx(l, T - 1)], ir = L.I[lidx(l, T - 1)];
#pragma unroll
  for (int d = -1; d <= 1; ++d) {
    if (CONN == 4 && d != 0) continue;
    const int c = l + d;  // -1 .. 64: halo corners included
    rt |= pt < umin(L.J[lidx(-1, c)], it);
    rb |= pb < umin(L.J[lidx(T, c)], ib);
    rl |= pl < umin(L.J[lidx(c, -1)], il);
    rr |= pr < umin(L.J[lidx(c, T)], ir);
  }
  // bits: 0 top, 1 bottom, 2 left, 3 right
  return (ballot(rt) ? 1u : 0u) | (ballot(rb) ? 2u : 0u) | (ballot(rl) ? 4u : 0u) | (ballot(rr) ? 8u : 0u);
}

// ---- raisable-pixel test (full rounds of the bounded mode) -------------------------
// Dense test of the tile in LDS (region loaded with its halo).  Returns
// (wave-uniform) whether some pixel q of the tile can still be raised by a
// neighbour p, i.e. J(q) < J(p) and J(q) < I(q) -- Algorithm 5's propagation
// condition read from the receiving side -- and adds to `seeds` the number of
// pixels p meeting Algorithm 5's seed condition (some neighbour q with
// J(q) < J(p) and J(q) < I(q)).  Lane = column; rows are walked top to
// bottom keeping rows y-1, y, y+1 in registers.

// g(q) = J(q) if q can still rise (J(q) < I(q)), else 256 (never below J(p)).
__device__ __forceinline__ uint32_t gval(uint32_t j, uint32_t i) { return j < i ? j : 256u; }

template <int CONN>
__device__ bool lds_dirty(const WaveLds& L, uint32_t& seeds) {
  const int l = lane();
  const int hc = l == 0 ? -1 : T;  // fill column: lane 0 uses column -1, lane 63 column 64
  uint32_t jp = L.J[lidx(-1, l)], ip = L.I[lidx(-1, l)], fjp = L.J[lidx(-1, hc)], fip = L.I[lidx(-1, hc)];
  uint32_t jc = L.J[lidx(0, l)], ic = L.I[lidx(0, l)], fjc = L.J[lidx(0, hc)], fic = L.I[lidx(0, hc)];
  bool any = false;
  uint32_t cnt = 0;
#pragma unroll
  for (int c = 0; c < T / kChunk; ++c) {
    uint32_t nj[kChunk], ni[kChunk], nfj[kChunk], nfi[kChunk];
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      const int y = c * kChunk + k + 1;
      nj[k] = L.J[lidx(y, l)];
      ni[k] = L.I[lidx(y, l)];
      nfj[k] = L.J[lidx(y, hc)];
      nfi[k] = L.I[lidx(y, hc)];
    }
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      const uint32_t jn = nj[k], in = ni[k], fjn = nfj[k], fin = nfi[k];
      uint32_t m = umax(umax(jp, jn), umax(from_left(jc, fjc), from_right(jc, fjc)));
      const uint32_t gc = gval(jc, ic), gfc = gval(fjc, fic);
      uint32_t g = umin(umin(gval(jp, ip), gval(jn, in)), umin(from_left(gc, gfc), from_right(gc, gfc)));
      if (CONN == 8) {
        m = umax(m, umax(umax(from_left(jp, fjp), from_right(jp, fjp)), umax(from_left(jn, fjn), from_right(jn, fjn))));
        const uint32_t gp = gval(jp, ip), gfp = gval(fjp, fip), gn = gval(jn, in), gfn = gval(fjn, fin);
        g = umin(g, umin(umin(from_left(gp, gfp), from_right(gp, gfp)), umin(from_left(gn, gfn), from_right(gn, gfn))));
      }
      any |= jc < umin(m, ic);
      cnt += (uint32_t)__popcll(ballot(jc > g));
      jp = jc; ip = ic; fjp = fjc; fip = fic;
      jc = jn; ic = in; fjc = fjn; fic = fin;
    }
    asm volatile("" ::: "memory");
  }
  seeds += cnt;
  return ballot(any) != 0;
}

// ---- persistent propagation -----------------------------------------------------------
// The frontier of round r+1 while round r runs: the parity's flags and list,
// the sub-list this workgroup appends to, its capacity and lost flag.
struct Next {
  uint32_t* flags;
  uint32_t* list;
  uint32_t* count;
  uint32_t cap;
  uint32_t* lost;
};

__device__ __forceinline__ Next next_frontier(const MrArgs& a, uint32_t r) {
  const bool bounded = a.list_cap < a.ntiles;
  const uint32_t par = (r + 1u) & 1u, shard = bounded ? 0u : (blockIdx.x & (uint32_t)(kShards - 1));
  Next n;
  n.flags = a.flags + (size_t)par * a.ntiles;
  n.list = a.lists + ((size_t)par * kShards + shard) * a.ntiles;
  n.count = shard_count(a.counts, (r + 1u) % 3u, shard);
  n.cap = bounded ? a.list_cap : a.ntiles;
  n.lost = a.lost + par * 64u;
  return n;
}

// Flag the neighbours named by border mask m (see border_marks) and, if
// `unsettled`, the tile itself, for the next round (lanes 0..8 of the wave).
__device__ void mark_reach(WaveStage& s, const Next& nx, const TileRef& tr, uint32_t m, bool unsettled) {
  const int l = lane();
  int dy = 0, dx = 0;
  bool want = false;
  if (l < 8) {
    // bit order of border_marks: top, bottom, left, right, tl, tr, bl, br
    want = (m >> l) & 1u;
    dy = l < 2 ? (l == 0 ? -1 : 1) : (l < 4 ? 0 : (l < 6 ? -1 : 1));
    dx = l < 2 ? 0 : (l < 4 ? (l == 2 ? -1 : 1) : ((l & 1) ? 1 : -1));
  } else if (l == 8) {
    want = unsettled;
  }
  const int ny = tr.ty + dy, nx_ = tr.tx + dx;
  want = want && ny >= 0 && ny < tr.j.tiles_y && nx_ >= 0 && nx_ < tr.j.tiles_x;
  shard_mark(s, want, tr.j.tile_base + (uint32_t)(ny * tr.j.tiles_x + nx_), nx.flags, nx.list, nx.count, nx.cap, nx.lost);
}

// Round-0 visit: the seed pass of one tile (load from the clamped marker,
// sweep, write back) and its marks for round 1.
//
// In strip order (`fresh_top`: the tile above was written by this wave just
// before) the halo row above comes from the output; `below_next`: the tile
// below is this wave's next tile and will read this one's result, so it need
// not be flagged for this tile's bottom edge.
template <int CONN>
__device__ void seed_visit(const MrArgs& a, WaveLds& L, WaveStage& s, const Next& nx, uint32_t t, uint32_t& iters,
                           bool fresh_top = false, bool below_next = false) {
  const TileRef tr = tile_ref(a, t);
  if (fresh_top) drain();  // this wave's stores of the tile above are complete
  load_region<true>(tr, L, fresh_top);
  const int l = lane();
  const uint32_t ot = L.J[lidx(0, l)], ob = L.J[lidx(T - 1, l)];
  const uint32_t ol = L.J[lidx(l, 0)], orr = L.J[lidx(l, T - 1)];
  uint32_t it = 0;
  bool changed;
  const bool stable = sweep_tile<CONN>(L, a.seed_sweeps, it, changed, true);
  iters += it;
  store_tile(tr, L);
  store_cols(a, t, L, true);
  if (lane() == 0) cstore(a.unsettled + t, stable ? 0u : 1u);
  uint32_t m = border_marks<CONN>(L, ot, ob, ol, orr);
  if (below_next) m &= ~2u;  // bit 1: bottom
  mark_reach(s, nx, tr, m, !stable);
}

// One propagation visit: load the tile and its halo, sweep to local
// stability, write back, and flag the neighbouring tiles a border change can
// raise (and the tile itself if the sweep cap stopped it).  A tile that its
// last visit left stable needs work only if its new halo can raise its
// border (`border_raisable`); with `check` (full rounds) the whole tile is
// tested instead.
template <int CONN>
__device__ void visit_tile(const MrArgs& a, WaveLds& L, WaveStage& s, const Next& nx, uint32_t t, bool check,
                           uint32_t& visits, uint32_t& iters, uint32_t& seeds) {
  const TileRef tr = tile_ref(a, t);
  int start = 0;
  bool all_dirty = true;
  if (check) {
    load_region<false>(tr, L, false, a.cols, a.ntiles * 256u, t);
    if (!lds_dirty<CONN>(L, seeds)) return;
  } else {
    const uint32_t uns = lane() == 0 ? cload(a.unsettled + t) : 0u;
    uint32_t sides;
    if (CONN == 8) {
      // About a third of the listed 8-connected tiles turn out to need no
      // work: load the frame first and the interior only if needed.  Nearly
      // every listed 4-connected tile needs work, and the second round trip
      // measured slower there (1.85 against 1.81 ms): one load.
      load_frame(tr, L, a.cols, a.ntiles * 256u, t);
      sides = border_raisable<CONN>(L);
      if (readlane(uns, 0) == 0u && sides == 0u) return;
      load_interior(tr, L);
    } else {
      load_region<false>(tr, L, false, a.cols, a.ntiles * 256u, t);
      sides = border_raisable<CONN>(L);
      if (readlane(uns, 0) == 0u && sides == 0u) return;
    }
    all_dirty = readlane(uns, 0) != 0u;
    // First scan: the one moving away from a raisable side (top: columns
    // forward, bottom: columns backward, left: rows forward, right: rows backward).
    start = (sides & 1u) ? 1 : (sides & 2u) ? 3 : (sides & 4u) ? 0 : (sides & 8u) ? 2 : 0;
  }
  const int l = lane();
  const uint32_t ot = L.J[lidx(0, l)], ob = L.J[lidx(T - 1, l)];
  const uint32_t ol = L.J[lidx(l, 0)], orr = L.J[lidx(l, T - 1)];
  uint32_t it = 0;
  bool changed;
  const bool stable = sweep_tile<CONN>(L, a.max_sweeps, it, changed, all_dirty, start);
  iters += it;
  visits++;
  if (lane() == 0) cstore(a.unsettled + t, stable ? 0u : 1u);
  if (changed) {
    store_tile(tr, L);
    store_cols(a, t, L, false);
  }
  const uint32_t m = changed ? border_marks<CONN>(L, ot, ob, ol, orr) : 0u;
  mark_reach(s, nx, tr, m, !stable);
}

// Round 0 is the seed pass over every tile; round r >= 1 visits the tiles
// listed in round r-1 and lists the tiles of round r+1 (parity (r+1)&1,
// count slot (r+1)%3).  The list is split over kShards sub-lists, one per
// group of workgroups; a round's items (the concatenated sub-lists) are cut
// into one share per workgroup (WgShare).  Bounded mode (a capacity below
// the tile count) uses one sub-list of that capacity; a round whose list
// lost tiles is replaced by a full round that visits every tile holding a
// raisable pixel (all flags cleared first), restarting from the current
// image.  The flags and the counts must be zero when the kernel starts.
// WPB waves per workgroup.
template <int CONN, int WPB>
__global__ __launch_bounds__(64 * WPB, 16 / WPB) void k_propagate(MrArgs a) {
  __shared__ WaveLds lds[WPB];
  __shared__ uint32_t stage_mem[WPB][kStageCap];
  __shared__ uint32_t cnt[kShards];
  __shared__ uint32_t lost_sh, next_sh;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  WaveLds& L = lds[w];
  const uint32_t depth = a.stage_depth > 0u && a.stage_depth < (uint32_t)kStageCap ? a.stage_depth : (uint32_t)kStageCap;
  WaveStage s = {stage_mem[w], depth, 0u};
  L.J[lidx(lane() - 1, kZeroCol)] = 0;  // rows -1..62
  if (lane() < 2) L.J[lidx(T - 1 + lane(), kZeroCol)] = 0;  // rows 63, 64
  if (threadIdx.x == 0) next_sh = 0u;
  __syncthreads();
  const uint32_t nw = gridDim.x * WPB;  // waves of the grid
  const uint32_t cap = a.list_cap < a.ntiles ? a.list_cap : a.ntiles;
  uint32_t gen = 0, nclk = 0;
  uint32_t visits = 0, iters = 0, seed_iters = 0, rounds = 0, restarts = 0, seeds = 0, first = 0;
  clock_stamp(a.clock, nclk);
  {
    const Next nx = next_frontier(a, 0u);
    if (a.njobs == 1u) {
      // Strip order: each wave seeds vertical strips of S tiles top to bottom,
      // so the flood crosses the horizontal tile edges inside the seed pass.
      // The strips are shared by the waves of each workgroup (WgShare).
      const MrJob& j = a.job0;
      const uint32_t tx_n = (uint32_t)j.tiles_x, ty_n = (uint32_t)j.tiles_y;
      const uint32_t S = a.seed_strip > 0u ? a.seed_strip : (a.ntiles + nw - 1u) / nw;
      const uint32_t sy_n = (ty_n + S - 1) / S, nstrips = tx_n * sy_n;
      const bool cut = (j.w % T) != 0 && (j.w % T) % 16 != 0;  // right-edge tiles read bytes: stale halo there
      const WgShare share = wg_share(nstrips, &next_sh);
      for (uint32_t sid; share.take(sid);) {
        const uint32_t tx = sid % tx_n, ty0 = (sid / tx_n) * S;
        for (uint32_t k = 0; k < S && ty0 + k < ty_n; ++k) {
          const bool fresh_col = !(cut && tx + 1 == tx_n);
          const bool fresh = k > 0 && fresh_col;
          const bool below = fresh_col && k + 1 < S && ty0 + k + 1 < ty_n;  // the next tile reads this one fresh
          seed_visit<CONN>(a, L, s, nx, (ty0 + k) * tx_n + tx, seed_iters, fresh, below);
        }
      }
    } else {
      const WgShare share = wg_share(a.ntiles, &next_sh);
      for (uint32_t t; share.take(t);) seed_visit<CONN>(a, L, s, nx, t, seed_iters);
    }
    shard_flush(s, nx.list, nx.count, nx.cap, nx.flags, nx.lost);
  }
  round_work(a.clock, 0u, a.ntiles);
  bool ok = grid_barrier(a.bar, gen, a.stats);
  clock_stamp(a.clock, nclk);
  ok = ok && a.seed_only == 0u;
  for (uint32_t r = 1; ok; ++r) {
    const uint32_t par = r & 1u;
    // Every workgroup reads the same words: nothing writes them between the
    // previous barrier and this read (round r appends for round r+1).
    shard_counts(a.counts, r % 3u, cap, cnt);
    if (threadIdx.x == 0) {
      lost_sh = cload(a.lost + par * 64u);
      next_sh = 0u;  // last used before the previous barrier
    }
    __syncthreads();
    uint32_t n = 0;
    for (int x = 0; x < kShards; ++x) n += cnt[x];
    const bool full = lost_sh != 0u;
    if (!full && n == 0u) break;
    round_work(a.clock, r, full ? a.ntiles : n);
    if (r >= kMaxRounds) {  // safety limit: report instead of spinning on a logic error
      if (blockIdx.x == 0 && threadIdx.x == 0) stat_add(a.stats, kStatError, 1ull);
      break;
    }
    if (full) {
      if (!grid_barrier(a.bar, gen, a.stats)) break;  // everyone has read the decision
      for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < 2u * a.ntiles; i += gridDim.x * blockDim.x)
        cstore(a.flags + i, 0u);
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        cstore(a.lost, 0u);
        cstore(a.lost + 64, 0u);
        restarts++;
      }
      if (!grid_barrier(a.bar, gen, a.stats)) break;
    }
    // The counts of round r+2 are reused: clear them now (they were last read
    // in round r-1, and are next appended to in round r+1, after this round's barrier).
    if (blockIdx.x == 0 && threadIdx.x < (unsigned)kShards) cstore(shard_count(a.counts, (r + 2u) % 3u, threadIdx.x), 0u);
    const Next nx = next_frontier(a, r);
    const uint32_t before = visits;
    if (full) {
      const WgShare share = wg_share(a.ntiles, &next_sh);
      for (uint32_t t; share.take(t);) visit_tile<CONN>(a, L, s, nx, t, true, visits, iters, seeds);
    } else {
      const uint32_t* lists = a.lists + (size_t)par * kShards * a.ntiles;
      uint32_t* flg = a.flags + (size_t)par * a.ntiles;
      // XCD x visits the tiles XCD x listed (a bounded list is one sub-list:
      // then the whole list is cut over the grid)
      const bool bounded = a.list_cap < a.ntiles;
      const WgShare share = bounded ? wg_share(n, &next_sh) : wg_share_lists(cnt, &next_sh);
      for (uint32_t i; share.take(i);) {
        const uint32_t t = shard_item(lists, a.ntiles, cnt, i);
        if (lane() == 0) cstore(flg + t, 0u);
        visit_tile<CONN>(a, L, s, nx, t, false, visits, iters, seeds);
      }
    }
    shard_flush(s, nx.list, nx.count, nx.cap, nx.flags, nx.lost);
    if (r == 1) first = visits - before;
    rounds++;
    ok = grid_barrier(a.bar, gen, a.stats);
    clock_stamp(a.clock, nclk);
  }
  if (lane() == 0) {
    stat_add(a.stats, kStatSeeds, (unsigned long long)first);
    stat_add(a.stats, kStatItems, visits);
    stat_add(a.stats, kStatSweeps, iters + seed_iters);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    stat_add(a.stats, kStatRounds, rounds);
    stat_add(a.stats, kStatRestarts, restarts);
  }
}

// Image of every global tile, by binary search over the images' first tiles.
__global__ void k_tile_job(const MrJob* jobs, uint32_t njobs, uint32_t* tile_job, uint32_t ntiles) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = njobs;  // last job with tile_base <= t
    while (hi - lo > 1u) {
      const uint32_t mid = (lo + hi) >> 1;
      if (jobs[mid].tile_base <= t) lo = mid; else hi = mid;
    }
    tile_job[t] = lo;
  }
}

}  // namespace mr

// ---- host-side launch -----------------------------------------------------------------
int mr_launch(const MrArgs& a, int conn, int persistent_blocks, hipStream_t stream, Recorder* rec, const char** err) {
  using namespace mr;
  if (a.njobs > 1u) {
    const uint32_t b = (a.ntiles + 255u) / 256u;
    hipLaunchKernelGGL(k_tile_job, dim3(b < 1024u ? b : 1024u), dim3(256), 0, stream, a.jobs, a.njobs, a.tile_job, a.ntiles);
    if (hipGetLastError() != hipSuccess) {
      *err = "tile map launch failed";
      return -1;
    }
  }
  if (zero_words(a.flags, 2ull * a.ntiles, stream) != 0) {
    *err = "flag reset launch failed";
    return -1;
  }
  const int wpb = a.wg_waves == 8u ? 8 : 4;
  void* fn = wpb == 8 ? (conn == 8 ? reinterpret_cast<void*>(&k_propagate<8, 8>) : reinterpret_cast<void*>(&k_propagate<4, 8>))
                      : (conn == 8 ? reinterpret_cast<void*>(&k_propagate<8, 4>) : reinterpret_cast<void*>(&k_propagate<4, 4>));
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * wpb, 0) != hipSuccess || per_cu < 1) {
    *err = "occupancy query failed";
    return -1;
  }
  uint32_t blocks = persistent_grid(fn, per_cu, cus, 16 / wpb);
  if (persistent_blocks > 0 && (uint32_t)persistent_blocks < blocks) blocks = (uint32_t)persistent_blocks;
  MrArgs args = a;
  void* kargs[] = {&args};
  rec->begin(3, stream);
  const hipError_t le = launch_persistent(fn, blocks, kargs, stream, 64 * wpb);
  rec->end(stream);
  if (le != hipSuccess) {
    *err = "propagation launch failed";
    return -1;
  }
  return 0;
}

}  // namespace iwpp
