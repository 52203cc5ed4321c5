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
// How.  The image is cut into 32x32 tiles.  A round visits only the tiles
// whose pixels or one-pixel halo changed in the previous round: one wave loads
// the tile and its halo from the previous round's buffer into LDS, recomputes
// every pixel of the tile with the operator above, writes the tile to the other
// buffer, and flags itself and the neighbouring tiles its changes can reach for
// the next round.  Nothing writes the buffer a round reads, so no atomics touch
// pixels.  A tile that is not visited in a round keeps equal values in both
// buffers: a tile changes only in rounds it is visited, and after a round in
// which it changed it is visited again, so it stops being visited only after a
// round in which it (re)wrote its unchanged values.  The tiles of a round are
// a work list split into eight sub-lists, one per group of workgroups (one
// per XCD), appended to with one atomic per wave flush and consumed evenly by
// all waves in the next round; a per-tile flag keeps a tile on a round's list
// once.
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

constexpr int TE = kEdtTile;      // tile side
constexpr int RP = TE + 2;        // region side with the halo
constexpr int kWavesPerBlock = 4;
constexpr int kStageCap = 128;
constexpr uint32_t kNone = 0x80008000u;
constexpr uint32_t kMaxRounds = 1u << 20;

typedef unsigned v4u __attribute__((ext_vector_type(4)));
typedef short s2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_yx(int y, int x) { return ((uint32_t)y << 16) | (uint32_t)x; }

// Squared distance between packed points q and f (0 <= coordinates < 32767
// for q; f real or kNone).
__device__ __forceinline__ uint32_t d2(uint32_t q, uint32_t f) {
  const s2 e = __builtin_elementwise_sub_sat(__builtin_bit_cast(s2, q), __builtin_bit_cast(s2, f));
  return (uint32_t)__builtin_amdgcn_sdot2(e, e, 0, false);
}

// Offer candidate f to the best (distance << 32 | feature) key of pixel q.
__device__ __forceinline__ void offer(uint32_t q, uint32_t f, unsigned long long& best) {
  const unsigned long long key = ((unsigned long long)d2(q, f) << 32) | f;
  best = key < best ? key : best;
}

struct TileRef {
  EdtJob j;
  int ty, tx;
};

__device__ __forceinline__ TileRef tile_ref(const EdtArgs& a, uint32_t t) {
  TileRef r;
  r.j = a.njobs == 1u ? a.job0 : a.jobs[a.tile_job[t]];
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

// Region in LDS: 34 rows; row pitch 40 words, tile column x at word 4 + x
// (the halo at words 3 and 36), so that a row is ten aligned 16-byte chunks
// starting at tile column -4.
constexpr int PE = 40;
constexpr int kC0 = 4;
struct WaveLds {
  uint32_t F[RP * PE];
};

// Offset that makes a raw buffer access fall outside every buffer (reads 0).
constexpr uint32_t kOutside = 0xFFFFFFF0u;
constexpr uint32_t kStatePad = 16u;  // readable bytes after the last pixel of a state buffer
static_assert(kStatePad <= kEdtStatePad, "state buffers must be padded");

// Load the tile of `src` and its halo into LDS (kNone outside the image).
// 34 rows x 10 chunks of four words, six per lane, all as 16-byte loads with
// no branches between them, so the wave waits for memory once per visit.
// Chunks reaching outside the image are loaded anyway (or pointed outside the
// buffer) and their outside words replaced by kNone.
__device__ void load_region(const uint32_t* src, const TileRef& tr, WaveLds& L) {
  const EdtJob& j = tr.j;
  const int y0 = tr.ty * TE, x0 = tr.tx * TE;
  const int row0 = y0 > 0 ? y0 - 1 : 0;
  const int row1 = y0 + TE + 1 < j.h ? y0 + TE + 1 : j.h;
  const __amdgpu_buffer_rsrc_t rs = rows_rsrc(src, j, row0, row1 - row0, kStatePad);
  constexpr int kChunks = RP * 10;
  constexpr int kPer = (kChunks + kWave - 1) / kWave;
  v4u v[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int idx = lane() + k * kWave;
    const int ry = idx / 10, c = idx - ry * 10;
    const int y = y0 - 1 + ry, xs = x0 - kC0 + 4 * c;
    const bool ok = idx < kChunks && y >= 0 && y < j.h && xs >= 0 && xs < j.w;
    const uint32_t off = ok ? ((uint32_t)(y - row0) * (uint32_t)j.w + (uint32_t)xs) * 4u : kOutside;
    v[k] = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, kSc1));
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int idx = lane() + k * kWave;
    const int ry = idx / 10, c = idx - ry * 10;
    const int y = y0 - 1 + ry, xs = x0 - kC0 + 4 * c;
    const bool row_ok = y >= 0 && y < j.h;
    v4u o;
#pragma unroll
    for (int b = 0; b < 4; ++b) o[b] = (row_ok && xs + b >= 0 && xs + b < j.w) ? v[k][b] : kNone;
    if (idx < kChunks) *reinterpret_cast<v4u*>(&L.F[ry * PE + 4 * c]) = o;
  }
  wave_sync();
}

// One round of the operator on the tile in LDS.  Lane l handles column l & 31
// of rows (l >> 5), (l >> 5) + 2, ...; the new values go to `dst` (the other
// buffer), unconditionally.  Returns a bit mask of where something changed:
// bit 0 anywhere, 1 row 0, 2 last row, 3 column 0, 4 last column, 5..8 the
// corners (top-left, top-right, bottom-left, bottom-right); `changed` counts
// the changed pixels.
template <int CONN>
__device__ uint32_t relax_tile(const WaveLds& L, uint32_t* dst, const TileRef& tr, uint32_t& changed) {
  const EdtJob& j = tr.j;
  const int y0 = tr.ty * TE, x0 = tr.tx * TE;
  const int x = lane() & (TE - 1), yb = lane() >> 5;
  const int qx = x0 + x;
  const int row0 = y0 > 0 ? y0 - 1 : 0;
  const int row1 = y0 + TE + 1 < j.h ? y0 + TE + 1 : j.h;
  const __amdgpu_buffer_rsrc_t rs = rows_rsrc(dst, j, row0, row1 - row0);
  uint32_t any = 0, n = 0;
#pragma unroll 4
  for (int k = 0; k < TE / 2; ++k) {
    const int y = yb + 2 * k;
    const int qy = y0 + y;
    const uint32_t q = pack_yx(qy, qx);
    const uint32_t* c = &L.F[(y + 1) * PE + kC0 + x];
    const uint32_t old = c[0];
    unsigned long long best = ((unsigned long long)d2(q, old) << 32) | old;
    offer(q, c[-PE], best);
    offer(q, c[PE], best);
    offer(q, c[-1], best);
    offer(q, c[1], best);
    if (CONN == 8) {
      offer(q, c[-PE - 1], best);
      offer(q, c[-PE + 1], best);
      offer(q, c[PE - 1], best);
      offer(q, c[PE + 1], best);
    }
    const uint32_t bf = (uint32_t)best;
    const bool inside = qy < j.h && qx < j.w;
    if (inside)
      __builtin_amdgcn_raw_buffer_store_b32(bf, rs, ((uint32_t)(qy - row0) * (uint32_t)j.w + (uint32_t)qx) * 4u, 0, kSc1);
    if (inside && bf != old) {
      n++;
      any |= 1u;
      if (y == 0) any |= 2u;
      if (y == TE - 1) any |= 4u;
      if (x == 0) any |= 8u;
      if (x == TE - 1) any |= 16u;
      if (y == 0 && x == 0) any |= 32u;
      if (y == 0 && x == TE - 1) any |= 64u;
      if (y == TE - 1 && x == 0) any |= 128u;
      if (y == TE - 1 && x == TE - 1) any |= 256u;
    }
  }
  changed += n;
  uint32_t m = 0;
#pragma unroll
  for (int b = 0; b < 9; ++b)
    if (ballot((any >> b) & 1u)) m |= 1u << b;
  return m;
}

// The list of round r+1 while round r runs (r = 0 for the initial frontier):
// the parity's flags and the sub-list of this workgroup's group.
struct Next {
  uint32_t* flags;
  uint32_t* list;
  uint32_t* count;
};

__device__ __forceinline__ Next next_frontier(const EdtArgs& a, uint32_t r) {
  const uint32_t par = (r + 1u) & 1u, shard = blockIdx.x & (uint32_t)(kShards - 1);
  Next n;
  n.flags = a.flags + (size_t)par * a.ntiles;
  n.list = a.lists + ((size_t)par * kShards + shard) * a.ntiles;
  n.count = shard_count(a.counts, (r + 1u) % 3u, shard);
  return n;
}

// List, for the next round, the tiles that the changes of tile tr (mask m of
// relax_tile, or of the initial state) reach: itself (bit 0) and each
// neighbour whose halo holds a changed pixel.  Lanes 0..8 of the wave each
// handle one candidate.
__device__ __forceinline__ void mark_reach(const EdtArgs& a, WaveStage& s, const Next& nx, const TileRef& tr,
                                           uint32_t m) {
  const int l = lane();
  int dy = 0, dx = 0;
  bool want = false;
  if (l == 0) {
    want = (m & 1u) != 0u;
  } else if (l <= 8) {
    // lanes 1..8: top, bottom, left, right, top-left, top-right, bottom-left, bottom-right
    const int k = l - 1;
    want = (m & (k < 4 ? (2u << k) : (32u << (k - 4)))) != 0u;
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
// first round's list: the tiles holding a non-feature pixel next to a
// feature (exactly the pixels round 1 changes) and the neighbours whose halo
// holds one.  One wave per tile; the binary region is staged in LDS.  The
// flags and counts must be zero beforehand.
template <int CONN>
__global__ __launch_bounds__(256) void k_init(EdtArgs a) {
  constexpr int BP = RP + 2;  // byte pitch
  __shared__ uint8_t binl[kWavesPerBlock][RP * BP];
  __shared__ uint32_t stage_mem[kWavesPerBlock][16];
  const int w = threadIdx.x / kWave;
  const uint32_t t = blockIdx.x * kWavesPerBlock + w;
  if (t >= a.ntiles) return;
  const TileRef tr = tile_ref(a, t);
  const EdtJob& j = tr.j;
  const int y0 = tr.ty * TE, x0 = tr.tx * TE;
  uint8_t* B = binl[w];
  // Region bytes: 1 = feature, 0 = other or outside the image.
  for (int idx = lane(); idx < RP * RP; idx += kWave) {
    const int ry = idx / RP, rx = idx - ry * RP;
    const int y = y0 - 1 + ry, x = x0 - 1 + rx;
    B[ry * BP + rx] = (y >= 0 && y < j.h && x >= 0 && x < j.w && j.bin[(size_t)y * (uint32_t)j.w + (uint32_t)x] == 0) ? 1 : 0;
  }
  wave_sync();
  const int x = lane() & (TE - 1), yb = lane() >> 5;
  const int qx = x0 + x;
  uint32_t contour = 0, any = 0;
  for (int k = 0; k < TE / 2; ++k) {
    const int y = yb + 2 * k;
    const int qy = y0 + y;
    if (qy >= j.h || qx >= j.w) continue;
    const uint8_t* c = &B[(y + 1) * BP + x + 1];
    const bool feat = c[0] != 0;
    int nf = c[-BP] + c[BP] + c[-1] + c[1];
    int nin = (qy > 0) + (qy + 1 < j.h) + (qx > 0) + (qx + 1 < j.w);
    if (CONN == 8) {
      nf += c[-BP - 1] + c[-BP + 1] + c[BP - 1] + c[BP + 1];
      nin += (qy > 0 && qx > 0) + (qy > 0 && qx + 1 < j.w) + (qy + 1 < j.h && qx > 0) + (qy + 1 < j.h && qx + 1 < j.w);
    }
    const uint32_t v = feat ? pack_yx(qy, qx) : kNone;
    const size_t p = j.pix_base + (size_t)qy * (uint32_t)j.w + (uint32_t)qx;
    a.feat0[p] = v;
    a.feat1[p] = v;
    contour += (feat && nf < nin) ? 1u : 0u;  // a feature with a non-feature neighbour
    if (!feat && nf > 0) {
      any |= 1u;
      if (y == 0) any |= 2u;
      if (y == TE - 1) any |= 4u;
      if (x == 0) any |= 8u;
      if (x == TE - 1) any |= 16u;
      if (y == 0 && x == 0) any |= 32u;
      if (y == 0 && x == TE - 1) any |= 64u;
      if (y == TE - 1 && x == 0) any |= 128u;
      if (y == TE - 1 && x == TE - 1) any |= 256u;
    }
  }
  uint32_t tot = contour;
  for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
  uint32_t m = 0;
#pragma unroll
  for (int b = 0; b < 9; ++b)
    if (ballot((any >> b) & 1u)) m |= 1u << b;
  if (lane() == 0) {
    stat_add(a.stats, kStatSeeds, tot);
    stat_add(a.stats, kStatItems, tot);  // the first frontier
  }
  WaveStage st = {stage_mem[w], 16u, 0u};
  const Next nx = next_frontier(a, 0u);  // round 1's list
  mark_reach(a, st, nx, tr, m);
  shard_flush(st, nx.list, nx.count, a.ntiles, nx.flags, a.ovf);
}

template <int CONN>
__global__ __launch_bounds__(256) void k_rounds(EdtArgs a) {
  __shared__ WaveLds lds[kWavesPerBlock];
  __shared__ uint32_t stage_mem[kWavesPerBlock][kStageCap];
  __shared__ uint32_t cnt[kShards];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  WaveLds& L = lds[w];
  WaveStage s = {stage_mem[w], (uint32_t)kStageCap, 0u};
  const uint32_t gw = blockIdx.x * kWavesPerBlock + (uint32_t)w, nw = gridDim.x * kWavesPerBlock;
  uint32_t gen = 0;
  unsigned long long changed = 0, visits = 0;
  uint32_t r = 1;
  for (;; ++r) {
    // Every workgroup reads the same words: nothing writes them between the
    // previous barrier and this read (round r appends for round r+1).
    shard_counts(a.counts, r % 3u, a.ntiles, cnt);
    __syncthreads();
    uint32_t n = 0;
    for (int x = 0; x < kShards; ++x) n += cnt[x];
    if (n == 0u) break;
    if (r >= kMaxRounds) {  // safety limit: report instead of spinning on a logic error
      if (blockIdx.x == 0 && threadIdx.x == 0) stat_add(a.stats, kStatError, 1ull);
      break;
    }
    // The counts of round r+2 are reused: clear them now (they were last read
    // at the start of round r-1 and are next appended to in round r+1, after
    // this round's barrier).
    if (blockIdx.x == 0 && threadIdx.x < (unsigned)kShards) cstore(shard_count(a.counts, (r + 2u) % 3u, threadIdx.x), 0u);
    const uint32_t* rd = (r & 1u) ? a.feat0 : a.feat1;  // buffer (r-1)&1
    uint32_t* wr = (r & 1u) ? a.feat1 : a.feat0;        // buffer r&1
    const uint32_t par = r & 1u;
    const uint32_t* lists = a.lists + (size_t)par * kShards * a.ntiles;
    uint32_t* flg = a.flags + (size_t)par * a.ntiles;
    const Next nx = next_frontier(a, r);
    for (uint32_t i = gw; i < n; i += nw) {
      const uint32_t t = shard_item(lists, a.ntiles, cnt, i);
      if (lane() == 0) cstore(flg + t, 0u);
      const TileRef tr = tile_ref(a, t);
      load_region(rd, tr, L);
      uint32_t c = 0;
      const uint32_t m = relax_tile<CONN>(L, wr, tr, c);
      changed += c;
      visits++;
      mark_reach(a, s, nx, tr, m);
      wave_sync();  // LDS is reloaded by the next visit
    }
    shard_flush(s, nx.list, nx.count, a.ntiles, nx.flags, a.ovf);
    if (!grid_barrier(a.bar, gen, a.stats)) return;
  }
  // Both buffers now agree everywhere; write the outputs.
  const uint32_t* fin = a.feat0;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t jj = 0; jj < a.njobs; ++jj) {
    const EdtJob& j = a.njobs == 1u ? a.job0 : a.jobs[jj];
    const uint32_t npx = (uint32_t)j.h * (uint32_t)j.w;
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += stride) {
      const uint32_t f = cload(fin + j.pix_base + p);
      if (f == kNone) {
        j.sqdist[p] = -1;
        j.nearest[p] = -1;
      } else {
        const uint32_t y = p / (uint32_t)j.w, x = p - y * (uint32_t)j.w;
        j.sqdist[p] = (int32_t)d2(pack_yx((int)y, (int)x), f);
        j.nearest[p] = (int32_t)((f >> 16) * (uint32_t)j.w + (f & 0xffffu));
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) changed += __shfl_xor(changed, o);
  if (lane() == 0) {
    stat_add(a.stats, kStatItems, changed);  // pixels changed in a round join the next frontier
    stat_add(a.stats, kStatUpdates, changed);
    stat_add(a.stats, kStatSweeps, visits);
  }
  // Round r found an empty list: round r-1 changed nothing, rounds 1..r-2 did.
  if (blockIdx.x == 0 && threadIdx.x == 0) stat_add(a.stats, kStatRounds, r >= 2u ? r - 2u : 0u);
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
  if (zero_words(a.flags, 2ull * a.ntiles, stream) != 0) {
    *err = "flag reset launch failed";
    return -1;
  }
  const uint32_t init_blocks = (a.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
  rec->begin(4, stream);
  if (conn == 8)
    hipLaunchKernelGGL(k_init<8>, dim3(init_blocks), dim3(256), 0, stream, a);
  else
    hipLaunchKernelGGL(k_init<4>, dim3(init_blocks), dim3(256), 0, stream, a);
  rec->end(stream);
  if (hipGetLastError() != hipSuccess) {
    *err = "EDT init launch failed";
    return -1;
  }
  void* fn = conn == 8 ? reinterpret_cast<void*>(&k_rounds<8>) : reinterpret_cast<void*>(&k_rounds<4>);
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0) != hipSuccess || per_cu < 1) {
    *err = "occupancy query failed";
    return -1;
  }
  uint32_t blocks = persistent_grid(fn, per_cu, cus);
  if (persistent_blocks > 0 && (uint32_t)persistent_blocks < blocks) blocks = (uint32_t)persistent_blocks;
  EdtArgs args = a;
  void* kargs[] = {&args};
  rec->begin(5, stream);
  const hipError_t le = launch_persistent(fn, blocks, kargs, stream);
  rec->end(stream);
  if (le != hipSuccess) {
    *err = "EDT rounds launch failed";
    return -1;
  }
  return 0;
}

uint32_t persistent_grid(const void* fn, int per_cu, int cus) {
  hipFuncAttributes fa{};
  int lim = per_cu < 4 ? per_cu : 4;
  if (hipFuncGetAttributes(&fa, fn) == hipSuccess && fa.sharedSizeBytes > 0) {
    const int by_lds = (int)((160u * 1024u) / (unsigned)fa.sharedSizeBytes);  // LDS per CU
    if (by_lds < lim) lim = by_lds;
  }
  if (lim < 1) lim = 1;
  return (uint32_t)lim * (uint32_t)cus;
}

hipError_t launch_persistent(const void* fn, uint32_t blocks, void** args, hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive)
    return hipLaunchKernel(fn, dim3(blocks), dim3(256), args, 0, s);
  return hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(256), args, 0, s);
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
