// Device-side building blocks shared by the reconstruction and distance
// transform kernels (gfx950, wave64).
//
// Cross-workgroup coherence.  On MI355X every XCD has its own L2 and the L2s
// are not coherent with each other while a kernel runs, so plain loads can
// return stale lines for data another XCD wrote during the same launch.  The
// persistent kernels therefore move all data that other workgroups of the same
// launch read or write with device-scope ("sc1") loads and stores, and publish
// it by draining the store counter (s_waitcnt vmcnt(0)) before the atomic
// that makes it reachable.  The alternative -- agent-scope acquire/release,
// which writes back and invalidates the whole L2 -- costs roughly ten times
// more per handoff.  Kernel boundaries are coherence points, so data written
// by an earlier kernel may be read with plain loads.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace iwpp {

constexpr int kWave = 64;
constexpr int kSc1 = 16;  // buffer-instruction cache policy bit: device scope

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}

// Wait until every store/atomic this wave issued has completed.
__device__ __forceinline__ void drain() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// ---- device-coherent scalar accesses (one element per lane) -----------------
template <typename T>
__device__ __forceinline__ T cload(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void cstore(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T atomic_add(T* p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T atomic_or(T* p, T v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T atomic_min(T* p, T v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T atomic_max(T* p, T v) {
  return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- wave helpers -------------------------------------------------------------
__device__ __forceinline__ int lane() { return (int)__lane_id(); }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int mbcnt(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
// lane i receives v from lane i-1; lane 0 receives `fill`.
__device__ __forceinline__ uint32_t from_left(uint32_t v, uint32_t fill) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)v, 0x138 /* wave_shr:1 */, 0xf, 0xf, false);
}
// lane i receives v from lane i+1; lane 63 receives `fill`.
__device__ __forceinline__ uint32_t from_right(uint32_t v, uint32_t fill) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)v, 0x130 /* wave_shl:1 */, 0xf, 0xf, false);
}
// lane i receives v from lane i-1 (i+1); lane 0 (63) receives 0, the identity
// of an unsigned max, so a max of the result folds into one DPP instruction.
__device__ __forceinline__ uint32_t from_left0(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138 /* wave_shr:1 */, 0xf, 0xf, true);
}
__device__ __forceinline__ uint32_t from_right0(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130 /* wave_shl:1 */, 0xf, 0xf, true);
}
// A value the wave holds in common, moved to scalar registers word by word
// (e.g. a job descriptor read through a per-tile table), so that buffer
// resources built from it need no per-lane loop.
template <class V>
__device__ __forceinline__ V uniform(const V& v) {
  static_assert(sizeof(V) % 4 == 0, "whole words");
  uint32_t w[sizeof(V) / 4];
  __builtin_memcpy(w, &v, sizeof(V));
#pragma unroll
  for (int i = 0; i < (int)(sizeof(V) / 4); ++i) w[i] = (uint32_t)__builtin_amdgcn_readfirstlane((int)w[i]);
  V r;
  __builtin_memcpy(&r, w, sizeof(V));
  return r;
}
// Inclusive prefix sum over the 64 lanes with DPP (no LDS round trips):
// shifts by 1, 2, 4 and 8 inside each row of 16 lanes (zero-filled), then row
// 0's total into row 1 and row 2's into row 3 (row_bcast:15), then the total of
// rows 0-1 into rows 2-3 (row_bcast:31).
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111 /* row_shr:1 */, 0xf, 0xf, true);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112 /* row_shr:2 */, 0xf, 0xf, true);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114 /* row_shr:4 */, 0xf, 0xf, true);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118 /* row_shr:8 */, 0xf, 0xf, true);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142 /* row_bcast:15 */, 0xa, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143 /* row_bcast:31 */, 0xc, 0xf, false);
  return x;
}
__device__ __forceinline__ uint32_t readlane(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

// ---- statistics: sharded counters (8 copies, one per workgroup group) ---------
// Fields are summed over the shards by the host.
enum StatField : int {
  kStatSeeds = 0,
  kStatItems = 1,
  kStatSweeps = 2,
  kStatRounds = 3,
  kStatUpdates = 4,
  kStatRestarts = 5,
  kStatError = 6,
  kStatFields = 16
};
constexpr int kStatShards = 8;

__device__ __forceinline__ void stat_add(unsigned long long* stats, int field, unsigned long long v) {
  if (v) atomic_add(stats + (blockIdx.x & (kStatShards - 1)) * kStatFields + field, v);
}

// ---- grid barrier ---------------------------------------------------------------
// Hierarchical sense-counting barrier for a co-resident (cooperative) grid:
// workgroups arrive on one of 8 group counters (blockIdx & 7), the last of a
// group arrives on the top counter, and the last group bumps the generation.
// Counters sit 256 bytes apart so they do not share a cache line.  Every wait
// is bounded: on timeout (or when another workgroup raised `abort`) the
// barrier returns false and the caller must leave the kernel.
//
// The barrier can also OR one flag per workgroup over the grid: an arrival
// adds 1 to the low half of its counter and, when the flag is set, 1 to the
// high half, so the last arrival of a group knows the group's OR and passes it
// on to the top counter, whose last arrival publishes the grid's OR before it
// bumps the generation.  No other word is written, so a grid-wide "did anyone
// do X" costs nothing beyond the barrier.
struct GridBarrier {
  uint32_t group[8][64];
  uint32_t top[64];
  uint32_t gen[64];
  uint32_t abort[64];
  uint32_t result[64];
};

constexpr uint32_t kSpinLimit = 1u << 24;  // ~ seconds of polling, far beyond any real wait
constexpr uint32_t kArriveFlag = 1u << 16;  // an arrival's flag in the high half of a counter

// `flag` (LDS word, or null) is read after every wave of the workgroup has
// arrived and is reset to 0; the grid's OR of it is returned in `any`.
__device__ __forceinline__ bool grid_barrier_or(GridBarrier* b, uint32_t& gen, unsigned long long* stats,
                                                uint32_t* flag, bool& any) {
  __shared__ uint32_t ok, anyv;
  __syncthreads();
  if (threadIdx.x == 0) {
    drain();
    const bool mine = flag != nullptr && *flag != 0u;
    if (flag) *flag = 0u;
    const uint32_t nwg = gridDim.x;
    const uint32_t g = blockIdx.x & 7u;
    const uint32_t in_group = (nwg - g + 7u) >> 3;
    const uint32_t groups = nwg < 8u ? nwg : 8u;
    uint32_t res = 1;
    const uint32_t old = atomic_add(&b->group[g][0], 1u + (mine ? kArriveFlag : 0u));
    if ((old & (kArriveFlag - 1u)) == in_group - 1) {
      const bool gany = mine || (old >> 16) != 0u;
      cstore(&b->group[g][0], 0u);
      drain();
      const uint32_t old2 = atomic_add(&b->top[0], 1u + (gany ? kArriveFlag : 0u));
      if ((old2 & (kArriveFlag - 1u)) == groups - 1) {
        cstore(&b->top[0], 0u);
        cstore(&b->result[0], (gany || (old2 >> 16) != 0u) ? 1u : 0u);
        drain();
        cstore(&b->gen[0], gen + 1);
      }
    }
    uint32_t spins = 0;
    while (cload(&b->gen[0]) == gen) {
      if (cload(&b->abort[0])) { res = 0; break; }
      __builtin_amdgcn_s_sleep(2);
      if (++spins > kSpinLimit) {
        cstore(&b->abort[0], 1u);
        atomic_add(stats + kStatError, 1ull);
        res = 0;
        break;
      }
    }
    gen += 1;
    ok = res;
    anyv = res ? cload(&b->result[0]) : 0u;
  }
  __syncthreads();
  any = anyv != 0u;
  return ok != 0;
}

__device__ __forceinline__ bool grid_barrier(GridBarrier* b, uint32_t& gen, unsigned long long* stats) {
  bool unused;
  return grid_barrier_or(b, gen, stats, nullptr, unused);
}

// Compiler + memory ordering point for lanes of one wave that exchange data
// through LDS (LDS instructions of a wave execute in order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ---- per-wave staged append ---------------------------------------------------
// A wave collects items in an LDS buffer with ballot + mbcnt (no atomics) and
// flushes it to a global list with one atomic per flush.  `cap_global` bounds
// the global list; items past it are dropped and *ovf is set.  The fill level
// `n` is wave-uniform and lives in a register.
template <typename Item>
struct WaveStageT {
  Item* items;  // LDS, `cap` entries
  uint32_t cap;
  uint32_t n;
};
using WaveStage = WaveStageT<uint32_t>;

template <typename Item>
__device__ __forceinline__ void stage_flush(WaveStageT<Item>& s, Item* list, uint32_t* count, uint32_t cap_global,
                                            uint32_t* ovf) {
  const uint32_t n = s.n;
  if (n == 0) return;
  wave_sync();
  uint32_t base = 0;
  if (lane() == 0) base = atomic_add(count, n);
  base = readlane(base, 0);
  for (uint32_t i = lane(); i < n; i += kWave) {
    uint32_t slot = base + i;
    if (slot < cap_global) cstore(list + slot, s.items[i]);
  }
  if (base + n > cap_global && lane() == 0) cstore(ovf, 1u);
  wave_sync();
  s.n = 0;
}

// Append `item` for every lane with `pred`; flushes first if the stage could overflow.
template <typename Item>
__device__ __forceinline__ void stage_append(WaveStageT<Item>& s, bool pred, Item item, Item* list, uint32_t* count,
                                             uint32_t cap_global, uint32_t* ovf) {
  const uint64_t m = ballot(pred);
  if (m == 0) return;
  const uint32_t k = (uint32_t)__popcll(m);
  if (s.n + k > s.cap) stage_flush(s, list, count, cap_global, ovf);
  if (pred) s.items[s.n + mbcnt(m)] = item;
  s.n += k;
}

// ---- round timeline -----------------------------------------------------------
// Workgroup 0 stamps the realtime clock (a constant-rate counter) at kernel
// start and after every grid barrier into words 1..255 (word 0 counts the
// stamps), and the work of each phase (tiles visited) into words 256 + phase.
// Costs one or two stores per round.
constexpr uint32_t kClockStamps = 256;
__device__ __forceinline__ void clock_stamp(unsigned long long* clock, uint32_t& n) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && n + 1u < kClockStamps) {
    n++;
    clock[n] = __builtin_amdgcn_s_memrealtime();
    clock[0] = n;
  }
}
__device__ __forceinline__ void round_work(unsigned long long* clock, uint32_t phase, uint32_t tiles) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && phase < kClockStamps) clock[kClockStamps + phase] = tiles;
}

// Work of a round shared by the waves of a workgroup: the workgroup owns a
// contiguous range [lo, hi) of the round's items, and its waves take the next
// item from an LDS counter, so a wave whose visits were cheap takes more.
// Ranges are cut XCD-major: workgroup b runs on XCD b mod 8, and the eight
// XCDs own eight contiguous parts of the items, so the tiles an XCD visits
// together are neighbours whose shared cache lines (the other half of a
// 128-byte line, the halo rows and border columns) its own L2 holds.
// (One device-scope atomic per item instead, shared by all workgroups, was
// measured to double the dense rounds: its latency under contention exceeds
// the imbalance it removes; items dealt round-robin over the workgroups made
// the seed pass 40% slower than neighbouring strips on one XCD.)
struct WgShare {
  uint32_t lo, hi;
  uint32_t* next;  // LDS, zeroed before the round
  __device__ bool take(uint32_t& i) const {
    uint32_t k = 0;
    if (lane() == 0) k = atomicAdd(next, 1u);
    k = readlane(k, 0);
    i = lo + k;
    return i < hi;
  }
};

constexpr uint32_t kXcds = 8;  // workgroup b runs on XCD b mod 8

// Workgroups of the grid on XCD x, and this workgroup's rank among them.
__device__ __forceinline__ uint32_t xcd_groups(uint32_t x) { return (gridDim.x + kXcds - 1u - x) / kXcds; }

// This workgroup's share of the items [base, base + n) owned by its XCD.
__device__ __forceinline__ WgShare share_of(uint32_t base, uint32_t n, uint32_t* next) {
  const uint32_t l = blockIdx.x / kXcds, L = xcd_groups(blockIdx.x % kXcds);
  WgShare w;
  w.lo = base + (uint32_t)(((uint64_t)n * l) / L);
  w.hi = base + (uint32_t)(((uint64_t)n * (l + 1u)) / L);
  w.next = next;
  return w;
}

// n items cut into eight XCD parts (when the grid covers all XCDs).
__device__ __forceinline__ WgShare wg_share(uint32_t n, uint32_t* next) {
  if (gridDim.x < kXcds) {
    WgShare w;
    w.lo = (uint32_t)(((uint64_t)n * blockIdx.x) / gridDim.x);
    w.hi = (uint32_t)(((uint64_t)n * (blockIdx.x + 1u)) / gridDim.x);
    w.next = next;
    return w;
  }
  const uint32_t x = blockIdx.x % kXcds;
  const uint32_t lo = (uint32_t)(((uint64_t)n * x) / kXcds), hi = (uint32_t)(((uint64_t)n * (x + 1u)) / kXcds);
  return share_of(lo, hi - lo, next);
}

// A round's list, whose sub-list x (cnt[x] items) was appended by XCD x:
// XCD x takes its own sub-list, where the neighbours of the tiles it visited
// last round are.  Items are indices into the concatenated sub-lists.
__device__ __forceinline__ WgShare wg_share_lists(const uint32_t* cnt, uint32_t* next) {
  if (gridDim.x < kXcds) {
    uint32_t n = 0;
    for (uint32_t x = 0; x < kXcds; ++x) n += cnt[x];
    return wg_share(n, next);
  }
  const uint32_t x = blockIdx.x % kXcds;
  uint32_t base = 0;
  for (uint32_t y = 0; y < x; ++y) base += cnt[y];
  return share_of(base, cnt[x], next);
}

// ---- sharded tile frontier --------------------------------------------------------
// A round's work list of tiles is split into kShards sub-lists, one per group of
// workgroups (blockIdx & 7, i.e. one per XCD).  A wave stages its appends in LDS
// and flushes them into its group's sub-list with one atomic on that sub-list's
// counter, so each counter sees an eighth of the flushes.  Consumers read the
// kShards counters and split the concatenation evenly over all waves, so a
// round's work is balanced whatever the tiles' positions.  A per-tile flag word
// (set with atomic_or) keeps a tile on a round's list at most once.
constexpr int kShards = 8;

// Counter of (round slot, shard): 256 bytes apart.
__device__ __forceinline__ uint32_t* shard_count(uint32_t* counts, uint32_t slot, uint32_t shard) {
  return counts + (slot * (uint32_t)kShards + shard) * 64u;
}

// Flush the stage into sub-list `list` (capacity `cap`) counted by `count`.
// Items past the capacity are dropped: their flag is cleared (so a later mark
// can list them again) and *lost is set.
__device__ inline void shard_flush(WaveStage& s, uint32_t* list, uint32_t* count, uint32_t cap, uint32_t* flags,
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

// Stage tile t (every lane with `pred`) unless it is already on the list
// whose flags are `flags`; flushes first if the stage could overflow.
__device__ inline void shard_mark(WaveStage& s, bool pred, uint32_t t, uint32_t* flags, uint32_t* list,
                                  uint32_t* count, uint32_t cap, uint32_t* lost) {
  const bool fresh = pred && atomic_or(flags + t, 1u) == 0u;
  const uint64_t m = ballot(fresh);
  if (m == 0) return;
  const uint32_t k = (uint32_t)__popcll(m);
  if (s.n + k > s.cap) shard_flush(s, list, count, cap, flags, lost);
  if (fresh) s.items[s.n + mbcnt(m)] = t;
  s.n += k;
}

// Length of round slot `slot`'s list: per-shard counts (capped) into `cnt`
// (kShards entries in LDS, filled by threads 0..kShards-1 of the workgroup).
__device__ __forceinline__ void shard_counts(uint32_t* counts, uint32_t slot, uint32_t cap, uint32_t* cnt) {
  if (threadIdx.x < (unsigned)kShards) {
    const uint32_t c = cload(shard_count(counts, slot, threadIdx.x));
    cnt[threadIdx.x] = c < cap ? c : cap;
  }
}

// Item i of the concatenated sub-lists of one parity (lists: [kShards][stride]).
__device__ __forceinline__ uint32_t shard_item(const uint32_t* lists, uint32_t stride, const uint32_t* cnt, uint32_t i) {
  uint32_t x = 0;
  while (x + 1 < (uint32_t)kShards && i >= cnt[x]) {
    i -= cnt[x];
    ++x;
  }
  return cload(lists + (size_t)x * stride + i);
}

}  // namespace iwpp
