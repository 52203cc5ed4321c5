// Propagation-based Euclidean distance transform on gfx950.
//
// What is computed (Sec. 2.2, Algorithms 3 and 6): every pixel carries a
// nearest feature (the paper's VR), initially itself for features (0-pixels)
// and "none" otherwise; features propagate to neighbours in N_G when they are
// closer; the output is the squared distance to the carried feature and its
// index.  The propagation runs in level-synchronous rounds -- Algorithm 4's
// swap of input and output queues, made device-wide -- and a pixel offers the
// feature it held at the end of the previous round, so round r is the dense
// operator
//     f_r(q) = argmin over p in N_G[q] of (d2(q, f_{r-1}(p)), f_{r-1}(p))
// (lexicographic: squared distance, then feature index) and the result does
// not depend on thread order.
//
// How: K rounds per tile visit (temporal blocking).  The image is cut into
// 26x26 tiles.  A visit loads a tile with a K-pixel halo (a 34x34 region) from
// the state after round r into LDS and applies the operator K times, each time
// on a region one pixel smaller on every side, which leaves the tile exactly
// at round r + K; the tile goes to the other state buffer.  One step of the
// persistent kernel visits the listed tiles and ends in one grid barrier, so
// K rounds cost one barrier.  Which tiles a step must visit follows from two
// facts: a pixel's value only improves (its own previous feature is always a
// candidate), and a change travels at most one pixel per round.  So a tile can
// change during a step only if some pixel within K pixels of it changed in
// the last round of the previous step; such a change lists the tile that
// holds it and the neighbours within reach.  A tile that changed at all during
// a step is listed again, so that it rewrites its (then settled) values into
// the other buffer: a tile that is not visited holds equal values in both
// buffers, and every pixel a visit reads is at round r.
//
// The tiles of a step are a work list split into eight sub-lists, one per
// group of workgroups (one per XCD), appended to with one atomic per wave
// flush and consumed evenly by all waves in the next step; a per-tile flag
// keeps a tile on a step's list once.
//
// State is the feature's packed coordinates (y << 16 | x), 4 bytes per pixel.
// A candidate's squared distance is one saturating packed 16-bit subtraction
// and one 2-term dot product; "none" is the packed pair (-32768, -32768),
// whose saturated distance exceeds that of any real feature (coordinates are
// below 32767), and whose packed value exceeds any real feature's, so the
// lexicographic minimum needs no special case for it.
#include "iwpp_device.hpp"
#include "iwpp_internal.hpp"

namespace iwpp {
namespace edt {

constexpr int K = kEdtHalo;        // rounds per step = halo width
constexpr int TE = kEdtTile;       // tile side
constexpr int RP = TE + 2 * K;     // region side
constexpr int kCPR = (RP + 3) / 4; // 16-byte chunks per region row
constexpr int PE = 4 * kCPR;       // LDS row pitch (words)
constexpr int kWavesPerBlock = 4;  // the initialisation kernel
constexpr int kStageCap = 64;       // LDS work-list stage per wave (iwpp_options.stage_depth caps it)
constexpr uint32_t kMaxSteps = (1u << 20) / K;
static_assert(RP - 2 <= 32, "a round's region row must fit 32 lanes");
static_assert(K % 4 == 0, "region chunks must not straddle the image's left edge");
static_assert(K <= TE, "a change must reach no farther than the neighbouring tiles");

typedef unsigned v4u __attribute__((ext_vector_type(4)));
typedef short s2 __attribute__((ext_vector_type(2)));
typedef unsigned short u2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_yx(int y, int x) { return ((uint32_t)y << 16) | (uint32_t)x; }
__device__ __forceinline__ uint32_t umax32(uint32_t a, uint32_t b) { return a > b ? a : b; }
__device__ __forceinline__ uint32_t umin32(uint32_t a, uint32_t b) { return a < b ? a : b; }

// Coordinate arithmetic of the state words, in two forms.
//
// Narrow (sides up to 32767): coordinates are signed 16-bit fields and "none"
// is (-32768, -32768).  A squared distance is one saturating packed 16-bit
// subtraction and one 2-term dot product; none's saturated distance,
// 2 * 32767^2, exceeds that of any real feature, so it needs no special case.
//
// Wide (sides up to 46340, with (h-1)^2 + (w-1)^2 < 2^31 so that squared
// distances fit the int32 output): coordinates are unsigned 16-bit fields and
// none is all ones.  |dy|, |dx| come from packed maxima and minima, their
// squares sum in an unsigned dot product (below 2^32 for such sides), and
// none is given distance 2^32 - 1 explicitly.
template <bool kWide>
struct Coord;

template <>
struct Coord<false> {
  static constexpr uint32_t none = 0x80008000u;
  // Squared distance between q (real) and f (real or none).
  __device__ static __forceinline__ uint32_t d2(uint32_t q, uint32_t f) {
    const s2 e = __builtin_elementwise_sub_sat(__builtin_bit_cast(s2, q), __builtin_bit_cast(s2, f));
    // The three-operand dot product with a zero addend (the compiler's choice,
    // the accumulating form, needs a register cleared first).
    uint32_t r;
    asm("v_dot2_i32_i16 %0, %1, %1, 0" : "=v"(r) : "v"(__builtin_bit_cast(uint32_t, e)));
    return r;
  }
  // The lexicographically smallest (squared distance to q, feature) of the N
  // candidate features f[]: the smallest distance dm first, then the smallest
  // feature among the candidates at distance dm.  Distances are below 2^31,
  // so dm - d has its sign bit set exactly when d > dm; OR-ing that bit into
  // the feature puts every candidate farther than dm above every real feature
  // (real features are below 2^31; none has the bit already and is farthest
  // of all), and one more minimum picks the answer: 32-bit minima only, no
  // 64-bit key comparisons.
  template <int N>
  __device__ static __forceinline__ uint32_t nearest(uint32_t q, const uint32_t (&f)[N]) {
    uint32_t d[N];
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = d2(q, f[i]);
    uint32_t dm = d[0];
#pragma unroll
    for (int i = 1; i < N; ++i) dm = umin32(dm, d[i]);
    uint32_t fm = 0xFFFFFFFFu;
#pragma unroll
    for (int i = 0; i < N; ++i) fm = umin32(fm, f[i] | ((dm - d[i]) & 0x80000000u));
    return fm;
  }
};

template <>
struct Coord<true> {
  static constexpr uint32_t none = 0xFFFFFFFFu;
  __device__ static __forceinline__ uint32_t d2(uint32_t q, uint32_t f) {
    const u2 a = __builtin_bit_cast(u2, q), b = __builtin_bit_cast(u2, f);
    const u2 e = __builtin_elementwise_max(a, b) - __builtin_elementwise_min(a, b);
    const uint32_t r = __builtin_amdgcn_udot2(e, e, 0u, false);
    return f == none ? 0xFFFFFFFFu : r;
  }
  // Lexicographic minimum: the smallest distance, then the smallest feature
  // among the candidates at that distance (packed (y, x) order is index order).
  template <int N>
  __device__ static __forceinline__ uint32_t nearest(uint32_t q, const uint32_t (&f)[N]) {
    uint32_t d[N];
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = d2(q, f[i]);
    uint32_t dm = d[0];
#pragma unroll
    for (int i = 1; i < N; ++i) dm = umin32(dm, d[i]);
    uint32_t fm = 0xFFFFFFFFu;
#pragma unroll
    for (int i = 0; i < N; ++i) fm = umin32(fm, d[i] == dm ? f[i] : 0xFFFFFFFFu);
    return fm;
  }
};

struct TileRef {
  EdtJob j;
  int ty, tx;
};

__device__ __forceinline__ TileRef tile_ref(const EdtArgs& a, uint32_t t) {
  TileRef r;
  r.j = uniform(a.njobs == 1u ? a.job0 : a.jobs[a.tile_job[t]]);
  const uint32_t lt = t - r.j.tile_base;
  r.ty = (int)(lt / (uint32_t)r.j.tiles_x);
  r.tx = (int)(lt - (uint32_t)r.ty * (uint32_t)r.j.tiles_x);
  return r;
}

// Buffer resource over the image rows [row0, row0 + rows) of a per-pixel u32
// array, plus `pad` bytes after them (the state buffers are padded so that a
// 16-byte load cut by the end of the last row stays inside).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rows_rsrc(const uint32_t* base, const EdtJob& j, int row0, int rows,
                                                            uint32_t pad = 0u) {
  return make_rsrc(base + j.pix_base + (unsigned long long)row0 * (uint32_t)j.w, (uint32_t)rows * (uint32_t)j.w * 4u + pad);
}

// Offset that makes a raw buffer access fall outside every buffer (reads 0).
constexpr uint32_t kOutside = 0xFFFFFFF0u;
constexpr uint32_t kStatePad = 16u;  // readable bytes after the last pixel of a state buffer
static_assert(kStatePad <= kEdtStatePad, "state buffers must be padded");

// Per-wave LDS: the region, the change masks of two consecutive rounds (one
// bit per region pixel, a 64-bit word per row) and the active-pixel list.
constexpr int kMaxActive = (RP - 2) * (RP - 2);  // pixels of round 1
constexpr int kPerLane = (kMaxActive + kWave - 1) / kWave;
struct WaveLds {
  uint32_t F[RP * PE];
  unsigned long long chg[2][RP];
  uint16_t list[kMaxActive];
};

// Load the region of tile tr (rows and columns from K before the tile) from
// `src` into S; pixels outside the image read as none.  kCPR 16-byte chunks
// per row, all issued with no branch in between so the wave waits for memory
// once; a chunk cut by the image's right edge is loaded whole (the state
// buffers are padded) and its outside words replaced.
template <bool kWide>
__device__ void load_region(const uint32_t* src, const TileRef& tr, uint32_t* S) {
  constexpr uint32_t kNone = Coord<kWide>::none;
  const EdtJob& j = tr.j;
  const int ry0 = tr.ty * TE - K, rx0 = tr.tx * TE - K;
  const int row0 = ry0 > 0 ? ry0 : 0;
  const int row1 = ry0 + RP < j.h ? ry0 + RP : j.h;
  const __amdgpu_buffer_rsrc_t rs = rows_rsrc(src, j, row0, row1 - row0, kStatePad);
  constexpr int kChunks = RP * kCPR;
  constexpr int kPer = (kChunks + kWave - 1) / kWave;
  v4u v[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int idx = lane() + k * kWave;
    const int ry = idx / kCPR, c = idx - ry * kCPR;
    const int y = ry0 + ry, xs = rx0 + 4 * c;
    const bool ok = idx < kChunks && y >= 0 && y < j.h && xs >= 0 && xs < j.w;
    const uint32_t off = ok ? ((uint32_t)(y - row0) * (uint32_t)j.w + (uint32_t)xs) * 4u : kOutside;
    v[k] = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, kSc1));
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int idx = lane() + k * kWave;
    const int ry = idx / kCPR, c = idx - ry * kCPR;
    const int y = ry0 + ry, xs = rx0 + 4 * c;
    const bool row_ok = y >= 0 && y < j.h;
    v4u o;
#pragma unroll
    for (int b = 0; b < 4; ++b) o[b] = (row_ok && xs + b >= 0 && xs + b < j.w) ? v[k][b] : kNone;
    if (idx < kChunks) *reinterpret_cast<v4u*>(&S[ry * PE + 4 * c]) = o;
  }
  wave_sync();
}

// Zone bits of a tile pixel (cy, cx): which neighbouring tiles lie within K
// pixels of it -- 1 top, 2 bottom, 3 left, 4 right, 5 top-left, 6 top-right,
// 7 bottom-left, 8 bottom-right (bit 0, the tile itself, is set by callers).
__device__ __forceinline__ uint32_t zone_bits(int cy, int cx) {
  const bool t = cy < K, b = cy >= TE - K, l = cx < K, r = cx >= TE - K;
  return (t ? 2u : 0u) | (b ? 4u : 0u) | (l ? 8u : 0u) | (r ? 16u : 0u) | (t && l ? 32u : 0u) |
         (t && r ? 64u : 0u) | (b && l ? 128u : 0u) | (b && r ? 256u : 0u);
}

// K rounds of the operator on the region in LDS, in place.  Round i
// computes region rows and columns [i, RP-i) from round i-1's values, only at
// the pixels with a neighbour (or themselves) changed in round i-1 -- the
// others cannot change -- gathered into a list from the previous round's
// change masks; for round 1 those are the previous step's last-round changes
// over the region (`prev_step_issue` / `prev_step_finish`; for the first
// step, the contour features recorded by `k_init`).  Pixels outside the image
// never enter the list (they stay none).  Each lane computes up to kPerLane
// list pixels, kBatch at a time with their loads issued together, into
// registers, and writes the changed ones after the whole wave has read, so
// every read sees round i-1.  Accumulates the changed tile pixels (over the
// rounds), the zone mask (bit 0: a tile pixel changed; bits 1..8: a change in
// round K within K pixels of that side) and the last round (1..K) with a
// change.
constexpr int kBatch = 2;
static_assert(kPerLane % kBatch == 0, "whole batches");
template <int CONN, bool kWide>
__device__ void relax_steps(WaveLds& L, const TileRef& tr, uint32_t& changed, uint32_t& zone, uint32_t& last) {
  static_assert(RP <= 64, "one mask bit per region column");
  constexpr int NC = CONN == 8 ? 9 : 5;
  const EdtJob& j = tr.j;
  const int ry0 = tr.ty * TE - K, rx0 = tr.tx * TE - K;
  const int l = lane();
  // Region columns and this lane's region row that lie inside the image.
  const int c_lo = rx0 < 0 ? -rx0 : 0, c_hi = j.w - rx0 < RP ? j.w - rx0 : RP;
  const unsigned long long in_cols = ((c_hi >= 64 ? ~0ull : ((1ull << c_hi) - 1ull))) & ~((1ull << c_lo) - 1ull);
  const bool in_row = ry0 + l >= 0 && ry0 + l < j.h;
#pragma unroll 1
  for (int i = 1; i <= K; ++i) {
    unsigned long long* now = L.chg[i & 1];
    const unsigned long long* prev = L.chg[(i - 1) & 1];
    // The active list of round i (for round 1, chg[0] holds the previous
    // step's last-round changes over the region).
    uint32_t n;
    {
      const unsigned long long win = ((1ull << (RP - i)) - 1ull) & ~((1ull << i) - 1ull) & in_cols;  // columns [i, RP-i)
      unsigned long long m = 0;
      if (l >= i && l < RP - i && in_row) {
        m = prev[l - 1] | prev[l] | prev[l + 1];
        m = (m | (m << 1) | (m >> 1)) & win;
      }
      // exclusive prefix of the per-row counts over the lanes
      const uint32_t c = (uint32_t)__popcll(m);
      const uint32_t incl = wave_incl_sum(c);
      n = (uint32_t)readlane(incl, kWave - 1);
      uint32_t at = incl - c;
      while (m) {
        const int col = __ffsll((long long)m) - 1;
        m &= m - 1;
        L.list[at++] = (uint16_t)((l << 8) | col);
      }
    }
    if (l < RP) now[l] = 0ull;
    wave_sync();
    // Compute (reads only): batches of kBatch list pixels per lane.
    uint32_t res[kPerLane];
    uint32_t chg = 0;  // bit k: list pixel k of this lane changed
#pragma unroll
    for (int k0 = 0; k0 < kPerLane; k0 += kBatch) {
      if ((uint32_t)(k0 * kWave) < n) {  // wave-uniform
        uint32_t f[kBatch][NC], ent[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          const uint32_t idx = (uint32_t)((k0 + b) * kWave + l);
          // past the list: a harmless in-region pixel (row 1, column 1); its result is not used
          ent[b] = idx < n ? (uint32_t)L.list[idx] : 0x101u;
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          const uint32_t* c = &L.F[(int)(ent[b] >> 8) * PE + (int)(ent[b] & 0xffu)];
          f[b][0] = c[0];
          f[b][1] = c[-PE];
          f[b][2] = c[PE];
          f[b][3] = c[-1];
          f[b][4] = c[1];
          if (CONN == 8) {
            f[b][5] = c[-PE - 1];
            f[b][6] = c[-PE + 1];
            f[b][7] = c[PE - 1];
            f[b][8] = c[PE + 1];
          }
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          const uint32_t q = pack_yx(ry0 + (int)(ent[b] >> 8), rx0 + (int)(ent[b] & 0xffu));
          res[k0 + b] = Coord<kWide>::nearest(q, f[b]);
          const uint32_t idx = (uint32_t)((k0 + b) * kWave + l);
          chg |= (idx < n && res[k0 + b] != f[b][0]) ? (1u << (k0 + b)) : 0u;
        }
      }
    }
    wave_sync();
    // Write back the changed pixels, recording them.
#pragma unroll
    for (int k = 0; k < kPerLane; ++k) {
      if (!((chg >> k) & 1u)) continue;
      const uint32_t e = L.list[(uint32_t)(k * kWave + l)];
      const int row = (int)(e >> 8), col = (int)(e & 0xffu);
      L.F[row * PE + col] = res[k];
      atomicOr(&now[row], 1ull << col);
      if (row >= K && row < K + TE && col >= K && col < K + TE) {
        changed++;
        last = (uint32_t)i;
        zone |= 1u;
        if (i == K) zone |= zone_bits(row - K, col - K);
      }
    }
    wave_sync();
  }
}

// Region change mask (one 64-bit word per region row, bit = region column)
// of the pixels that changed in the last round of step m-1.  Every such pixel
// lies in a tile visited in step m-1, which recorded its last-round changes
// (`record_changes`) under that step's parity with stamp m-1; a tile whose
// stamp differs did not change.  Lane = region row: the stamps and row words
// of three tiles (left neighbour, own column, right neighbour).  Split in two
// so that the loads can be issued before the region load and waited for with
// it.
struct PrevChanges {
  uint32_t stamp[3], word[3];
};

__device__ __forceinline__ void prev_step_issue(const EdtArgs& a, const TileRef& tr, uint32_t m, PrevChanges& pc) {
  const EdtJob& j = tr.j;
  const int l = lane();
  const uint32_t par = (m - 1u) & 1u;
  const int y = tr.ty * TE - K + l;
  const bool row_ok = l < RP && y >= 0 && y < j.h;
  const int ty = row_ok ? y / TE : 0, ly = row_ok ? y - ty * TE : 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int tx = tr.tx + d - 1;
    pc.stamp[d] = 0u;
    pc.word[d] = 0u;
    if (row_ok && tx >= 0 && tx < j.tiles_x) {
      const uint32_t u = j.tile_base + (uint32_t)(ty * j.tiles_x + tx);
      pc.stamp[d] = cload(a.stamps + (size_t)par * a.ntiles + u);
      pc.word[d] = cload(a.marks + ((size_t)par * a.ntiles + u) * 32u + (uint32_t)ly);
    }
  }
}

__device__ __forceinline__ void prev_step_finish(uint32_t m, const PrevChanges& pc, unsigned long long* M) {
  const int l = lane();
  unsigned long long v = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (pc.stamp[d] != m - 1u) continue;
    const unsigned long long w = pc.word[d];
    // region column rx <-> tile column rx - K - (d - 1) * TE
    v |= d == 0 ? (w >> (TE - K)) : (d == 1 ? (w << K) : ((w & ((1ull << K) - 1ull)) << (K + TE)));
  }
  if (l < RP) M[l] = v;
  wave_sync();
}

// Record this visit's last-round changes of the tile (rows and columns
// [K, K + TE) of the round-K mask `M`) and stamp them with step m.
__device__ void record_changes(const EdtArgs& a, uint32_t t, uint32_t m, const unsigned long long* M) {
  const int l = lane();
  const uint32_t par = m & 1u;
  if (l < TE)
    cstore(a.marks + ((size_t)par * a.ntiles + t) * 32u + (uint32_t)l, (uint32_t)((M[K + l] >> K) & ((1ull << TE) - 1ull)));
  if (l == 0) cstore(a.stamps + (size_t)par * a.ntiles + t, m);
}

// Store the tile (region rows and columns [K, K + TE)) from S to `dst`.
__device__ void store_tile(const uint32_t* S, uint32_t* dst, const TileRef& tr) {
  const EdtJob& j = tr.j;
  const int y0 = tr.ty * TE, x0 = tr.tx * TE;
  const int row1 = y0 + TE < j.h ? y0 + TE : j.h;
  const __amdgpu_buffer_rsrc_t rs = rows_rsrc(dst, j, y0, row1 - y0);
  for (int idx = lane(); idx < TE * TE; idx += kWave) {
    const int cy = idx / TE, cx = idx - cy * TE;
    const int y = y0 + cy, x = x0 + cx;
    if (y < j.h && x < j.w)
      __builtin_amdgcn_raw_buffer_store_b32(S[(cy + K) * PE + cx + K], rs,
                                            ((uint32_t)cy * (uint32_t)j.w + (uint32_t)x) * 4u, 0, kSc1);
  }
}

// The list of step m+1 while step m runs (m = 0 for the initial list): the
// parity's flags and the sub-list of this workgroup's group.
struct Next {
  uint32_t* flags;
  uint32_t* list;
  uint32_t* count;
};

__device__ __forceinline__ Next next_frontier(const EdtArgs& a, uint32_t m) {
  const uint32_t par = (m + 1u) & 1u, shard = blockIdx.x & (uint32_t)(kShards - 1);
  Next n;
  n.flags = a.flags + (size_t)par * a.ntiles;
  n.list = a.lists + ((size_t)par * kShards + shard) * a.ntiles;
  n.count = shard_count(a.counts, (m + 1u) % 3u, shard);
  return n;
}

// List, for the next step, the tiles named by zone mask z of tile tr: itself
// (bit 0) and the neighbours of bits 1..8.  Lanes 0..8 of the wave each
// handle one candidate.
__device__ __forceinline__ void mark_reach(const EdtArgs& a, WaveStage& s, const Next& nx, const TileRef& tr,
                                           uint32_t z) {
  const int l = lane();
  int dy = 0, dx = 0;
  bool want = false;
  if (l == 0) {
    want = (z & 1u) != 0u;
  } else if (l <= 8) {
    // lanes 1..8: top, bottom, left, right, top-left, top-right, bottom-left, bottom-right
    const int k = l - 1;
    want = (z & (k < 4 ? (2u << k) : (32u << (k - 4)))) != 0u;
    dy = k == 0 ? -1 : (k == 1 ? 1 : (k < 4 ? 0 : (k < 6 ? -1 : 1)));
    dx = k < 2 ? 0 : (k == 2 ? -1 : (k == 3 ? 1 : ((k & 1) ? 1 : -1)));
  }
  const int ny = tr.ty + dy, nx_ = tr.tx + dx;
  want = want && ny >= 0 && ny < tr.j.tiles_y && nx_ >= 0 && nx_ < tr.j.tiles_x;
  shard_mark(s, want, tr.j.tile_base + (uint32_t)(ny * tr.j.tiles_x + nx_), nx.flags, nx.list, nx.count, a.ntiles,
             a.ovf);
}

// Initial state (features carry themselves, everything else none) in both
// buffers, the contour-feature count (Algorithm 6's initial queue), and the
// first step's list: round 1 changes exactly the non-features next to a
// feature, so their tiles and the neighbours within K pixels are listed.  The
// contour features are every tile's step-0 change record, from which the
// first step's round 1 takes its active pixels.  One wave per tile; the binary
// region (tile and one-pixel halo) is staged in LDS.  The flags, counts and
// stamps must be zero beforehand.
template <int CONN, bool kWide>
__global__ __launch_bounds__(256) void k_init(EdtArgs a) {
  constexpr int BR = TE + 2;  // binary region side
  constexpr int BP = BR + 2;  // byte pitch
  __shared__ uint8_t binl[kWavesPerBlock][BR * BP];
  __shared__ uint32_t stage_mem[kWavesPerBlock][16];
  const int w = threadIdx.x / kWave;
  const uint32_t t = blockIdx.x * kWavesPerBlock + w;
  if (t >= a.ntiles) return;
  const TileRef tr = tile_ref(a, t);
  const EdtJob& j = tr.j;
  const int y0 = tr.ty * TE, x0 = tr.tx * TE;
  uint8_t* B = binl[w];
  // Region bytes: 1 = feature, 0 = other or outside the image.
  for (int idx = lane(); idx < BR * BR; idx += kWave) {
    const int ry = idx / BR, rx = idx - ry * BR;
    const int y = y0 - 1 + ry, x = x0 - 1 + rx;
    B[ry * BP + rx] = (y >= 0 && y < j.h && x >= 0 && x < j.w && j.bin[(size_t)y * (uint32_t)j.w + (uint32_t)x] == 0) ? 1 : 0;
  }
  wave_sync();
  const int x = lane() & 31, yb = lane() >> 5;
  const int qx = x0 + x;
  uint32_t contour = 0, zone = 0;
  uint32_t* rec = a.marks + (size_t)t * 32u;  // step 0's record (parity 0; the stamps are zero)
  for (int y = yb; y < TE; y += 2) {
    const int qy = y0 + y;
    bool ct = false;
    if (x < TE && qy < j.h && qx < j.w) {
      const uint8_t* c = &B[(y + 1) * BP + x + 1];
      const bool feat = c[0] != 0;
      int nf = c[-BP] + c[BP] + c[-1] + c[1];
      int nin = (qy > 0) + (qy + 1 < j.h) + (qx > 0) + (qx + 1 < j.w);
      if (CONN == 8) {
        nf += c[-BP - 1] + c[-BP + 1] + c[BP - 1] + c[BP + 1];
        nin += (qy > 0 && qx > 0) + (qy > 0 && qx + 1 < j.w) + (qy + 1 < j.h && qx > 0) + (qy + 1 < j.h && qx + 1 < j.w);
      }
      const uint32_t v = feat ? pack_yx(qy, qx) : Coord<kWide>::none;
      const size_t p = j.pix_base + (size_t)qy * (uint32_t)j.w + (uint32_t)qx;
      a.feat0[p] = v;
      a.feat1[p] = v;
      ct = feat && nf < nin;  // a feature with a non-feature neighbour
      contour += ct ? 1u : 0u;
      if (!feat && nf > 0) zone |= 1u | zone_bits(y, x);
    }
    // Round 0's changes as round 1 sees them: only the contour features
    // offer anything new (a feature keeps itself; a pixel away from every
    // feature stays none).  Lanes 0..31 hold row y, lanes 32..63 row y + 1.
    const uint64_t bm = ballot(ct);
    if (lane() == 0 || lane() == 32) cstore(rec + y, lane() == 0 ? (uint32_t)bm : (uint32_t)(bm >> 32));
  }
  const uint32_t tot = readlane(wave_incl_sum(contour), kWave - 1);
  uint32_t z = 0;
#pragma unroll
  for (int b = 0; b < 9; ++b)
    if (ballot((zone >> b) & 1u)) z |= 1u << b;
  if (lane() == 0) {
    stat_add(a.stats, kStatSeeds, tot);
    stat_add(a.stats, kStatItems, tot);  // the first frontier
  }
  WaveStage st = {stage_mem[w], 16u, 0u};
  const Next nx = next_frontier(a, 0u);  // step 1's list
  mark_reach(a, st, nx, tr, z);
  shard_flush(st, nx.list, nx.count, a.ntiles, nx.flags, a.ovf);
}

// WPB waves per workgroup; five workgroups of four waves (or two of eight)
// fit a CU's registers and LDS.  A step's tiles are shared by the waves of a
// workgroup (WgShare).
template <int CONN, bool kWide, int WPB>
__global__ __launch_bounds__(64 * WPB, WPB == 4 ? 5 : 2) void k_rounds(EdtArgs a) {
  __shared__ WaveLds lds[WPB];
  __shared__ uint32_t stage_mem[WPB][kStageCap];
  __shared__ uint32_t cnt[kShards];
  __shared__ uint32_t last_sh;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  WaveLds& L = lds[w];
  const uint32_t depth = a.stage_depth > 0u && a.stage_depth < (uint32_t)kStageCap ? a.stage_depth : (uint32_t)kStageCap;
  WaveStage s = {stage_mem[w], depth, 0u};
  const uint32_t gw = blockIdx.x * WPB + (uint32_t)w, nw = gridDim.x * WPB;
  if (threadIdx.x == 0) last_sh = 0u;
  uint32_t gen = 0, nclk = 0;
  unsigned long long changed = 0, visits = 0;
  uint32_t last_round = 0;  // this wave's last round with a change
  clock_stamp(a.clock, nclk);
  for (uint32_t m = 1;; ++m) {
    // Every workgroup reads the same words: nothing writes them between the
    // previous barrier and this read (step m appends for step m+1).
    shard_counts(a.counts, m % 3u, a.ntiles, cnt);
    __syncthreads();
    uint32_t n = 0;
    for (int x = 0; x < kShards; ++x) n += cnt[x];
    if (n == 0u) break;
    round_work(a.clock, m - 1u, n);
    if (m >= kMaxSteps) {  // safety limit: report instead of spinning on a logic error
      if (blockIdx.x == 0 && threadIdx.x == 0) stat_add(a.stats, kStatError, 1ull);
      break;
    }
    // The counts of step m+2 are reused: clear them now (they were last read
    // at the start of step m-1 and are next appended to in step m+1, after
    // this step's barrier).
    if (blockIdx.x == 0 && threadIdx.x < (unsigned)kShards) cstore(shard_count(a.counts, (m + 2u) % 3u, threadIdx.x), 0u);
    const uint32_t* rd = (m & 1u) ? a.feat0 : a.feat1;  // buffer (m-1)&1
    uint32_t* wr = (m & 1u) ? a.feat1 : a.feat0;        // buffer m&1
    const uint32_t par = m & 1u;
    const uint32_t* lists = a.lists + (size_t)par * kShards * a.ntiles;
    uint32_t* flg = a.flags + (size_t)par * a.ntiles;
    const Next nx = next_frontier(a, m);
    // Items are dealt round-robin over the waves of the grid: workgroup
    // pooling, and items kept on the XCD that listed them, were both measured
    // slower here (1.36 and 1.38 against 1.34 ms on the 4096^2 workload).
    // The next item's list entry is loaded while the current tile is visited.
    uint32_t t_next = gw < n ? shard_item(lists, a.ntiles, cnt, gw) : 0u;
    for (uint32_t i = gw; i < n; i += nw) {
      const uint32_t t = t_next;
      if (i + nw < n) t_next = shard_item(lists, a.ntiles, cnt, i + nw);
      if (lane() == 0) cstore(flg + t, 0u);
      const TileRef tr = tile_ref(a, t);
      PrevChanges pc;
      prev_step_issue(a, tr, m, pc);
      load_region<kWide>(rd, tr, L.F);
      prev_step_finish(m, pc, L.chg[0]);
      uint32_t c = 0, zone = 0, lr = 0;
      relax_steps<CONN, kWide>(L, tr, c, zone, lr);
      record_changes(a, t, m, L.chg[K & 1]);
      changed += c;
      visits++;
      uint32_t z = 0;
#pragma unroll
      for (int b = 0; b < 9; ++b)
        if (ballot((zone >> b) & 1u)) z |= 1u << b;
      uint32_t lw = 0;  // the wave's last round with a change (lr is 0..K per lane)
      for (uint32_t v = (uint32_t)K; v > 0u; --v)
        if (ballot(lr >= v) != 0u) {
          lw = v;
          break;
        }
      if (lw) last_round = umax32(last_round, (m - 1u) * (uint32_t)K + lw);
      store_tile(L.F, wr, tr);
      mark_reach(a, s, nx, tr, z);
      wave_sync();  // LDS is reloaded by the next visit
    }
    shard_flush(s, nx.list, nx.count, a.ntiles, nx.flags, a.ovf);
    if (!grid_barrier(a.bar, gen, a.stats)) return;
    clock_stamp(a.clock, nclk);
  }
  // Both buffers now agree everywhere; write the outputs.
  const uint32_t* fin = a.feat0;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t jj = 0; jj < a.njobs; ++jj) {
    const EdtJob& j = a.njobs == 1u ? a.job0 : a.jobs[jj];
    const uint32_t npx = (uint32_t)j.h * (uint32_t)j.w;
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += stride) {
      const uint32_t f = cload(fin + j.pix_base + p);
      if (f == Coord<kWide>::none) {
        j.sqdist[p] = -1;
        j.nearest[p] = -1;
      } else {
        const uint32_t y = p / (uint32_t)j.w, x = p - y * (uint32_t)j.w;
        j.sqdist[p] = (int32_t)Coord<kWide>::d2(pack_yx((int)y, (int)x), f);
        j.nearest[p] = (int32_t)((f >> 16) * (uint32_t)j.w + (f & 0xffffu));
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) changed += __shfl_xor(changed, o);
  if (lane() == 0) {
    stat_add(a.stats, kStatItems, changed);  // pixels changed in a round join the next frontier
    stat_add(a.stats, kStatUpdates, changed);
    stat_add(a.stats, kStatSweeps, visits);
    atomicMax(&last_sh, last_round);
  }
  __syncthreads();
  // Rounds: the last round in which any pixel changed -- a maximum, kept in
  // shard 0 so that the host's sum over the shards leaves it unchanged.
  if (threadIdx.x == 0 && last_sh) atomic_max(a.stats + kStatRounds, (unsigned long long)last_sh);
}

// Image of every global tile, by binary search over the images' first tiles.
__global__ void k_tile_job(const EdtJob* jobs, uint32_t njobs, uint32_t* tile_job, uint32_t ntiles) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = njobs;
    while (hi - lo > 1u) {
      const uint32_t mid = (lo + hi) >> 1;
      if (jobs[mid].tile_base <= t) lo = mid; else hi = mid;
    }
    tile_job[t] = lo;
  }
}

}  // namespace edt

int edt_launch(const EdtArgs& a, int conn, int persistent_blocks, hipStream_t stream, Recorder* rec, const char** err) {
  using namespace edt;
  if (a.njobs > 1u) {
    const uint32_t b = (a.ntiles + 255u) / 256u;
    hipLaunchKernelGGL(k_tile_job, dim3(b < 1024u ? b : 1024u), dim3(256), 0, stream, a.jobs, a.njobs, a.tile_job, a.ntiles);
    if (hipGetLastError() != hipSuccess) {
      *err = "tile map launch failed";
      return -1;
    }
  }
  if (zero_words(a.flags, 2ull * a.ntiles, stream) != 0 || zero_words(a.stamps, 2ull * a.ntiles, stream) != 0) {
    *err = "flag reset launch failed";
    return -1;
  }
  // eight XCD parts of ceil(ntiles / 8) tiles, kWavesPerBlock tiles per workgroup
  const uint32_t init_blocks = (a.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
  rec->begin(4, stream);
  if (conn == 8 && !a.wide)
    hipLaunchKernelGGL((k_init<8, false>), dim3(init_blocks), dim3(256), 0, stream, a);
  else if (conn == 8)
    hipLaunchKernelGGL((k_init<8, true>), dim3(init_blocks), dim3(256), 0, stream, a);
  else if (!a.wide)
    hipLaunchKernelGGL((k_init<4, false>), dim3(init_blocks), dim3(256), 0, stream, a);
  else
    hipLaunchKernelGGL((k_init<4, true>), dim3(init_blocks), dim3(256), 0, stream, a);
  rec->end(stream);
  if (hipGetLastError() != hipSuccess) {
    *err = "EDT init launch failed";
    return -1;
  }
  const int wpb = a.wg_waves == 8u ? 8 : 4;
  void* fn;
  if (wpb == 8)
    fn = conn == 8 ? (a.wide ? reinterpret_cast<void*>(&k_rounds<8, true, 8>) : reinterpret_cast<void*>(&k_rounds<8, false, 8>))
                   : (a.wide ? reinterpret_cast<void*>(&k_rounds<4, true, 8>) : reinterpret_cast<void*>(&k_rounds<4, false, 8>));
  else
    fn = conn == 8 ? (a.wide ? reinterpret_cast<void*>(&k_rounds<8, true, 4>) : reinterpret_cast<void*>(&k_rounds<8, false, 4>))
                   : (a.wide ? reinterpret_cast<void*>(&k_rounds<4, true, 4>) : reinterpret_cast<void*>(&k_rounds<4, false, 4>));
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * wpb, 0) != hipSuccess || per_cu < 1) {
    *err = "occupancy query failed";
    return -1;
  }
  uint32_t blocks = persistent_grid(fn, per_cu, cus, wpb == 4 ? 5 : 2);
  if (persistent_blocks > 0 && (uint32_t)persistent_blocks < blocks) blocks = (uint32_t)persistent_blocks;
  EdtArgs args = a;
  void* kargs[] = {&args};
  rec->begin(5, stream);
  const hipError_t le = launch_persistent(fn, blocks, kargs, stream, 64 * wpb);
  rec->end(stream);
  if (le != hipSuccess) {
    *err = "EDT rounds launch failed";
    return -1;
  }
  return 0;
}

uint32_t persistent_grid(const void* fn, int per_cu, int cus, int max_per_cu) {
  hipFuncAttributes fa{};
  int lim = per_cu < max_per_cu ? per_cu : max_per_cu;
  if (hipFuncGetAttributes(&fa, fn) == hipSuccess && fa.sharedSizeBytes > 0) {
    const int by_lds = (int)((160u * 1024u) / (unsigned)fa.sharedSizeBytes);  // LDS per CU
    if (by_lds < lim) lim = by_lds;
  }
  if (lim < 1) lim = 1;
  return (uint32_t)lim * (uint32_t)cus;
}

hipError_t launch_persistent(const void* fn, uint32_t blocks, void** args, hipStream_t s, uint32_t threads) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive)
    return hipLaunchKernel(fn, dim3(blocks), dim3(threads), args, 0, s);
  return hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(threads), args, 0, s);
}

// Zero a range of 32-bit words with a kernel (no memset node, so the sequence
// can be captured into a graph).
__global__ void k_zero(uint32_t* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}

int zero_words(uint32_t* p, size_t nwords, hipStream_t stream) {
  size_t blocks = (nwords + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks == 0) return 0;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, stream, p, nwords);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace iwpp
