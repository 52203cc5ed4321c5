// Reconstruction by dilation with the paper's pixel queue, for comparison
// with the tile design (iwpp_morph_recon_queue_u8).
//
// After a seed pass (the tile seed pass of the main kernel, swept a given
// number of times: the analogue of the number of initial raster scans that
// Table 1 varies), the image is copied to 32-bit words and every pixel that
// can raise a neighbour (Algorithm 5's seed condition, over the full
// neighbourhood) is queued.  A persistent kernel then runs the queue in
// rounds, one item per lane (the in/out queue swap of Algorithm 4, made
// device-wide): popping p, every neighbour q with J(q) < J(p) and J(q) < I(q)
// is raised with an atomic maximum to min(J(p), I(q)), and queued when that
// atomic raised it (Algorithm 5's propagation).  Three ways to append to the
// round's queue (Sec. 3.2 and Table 1):
//   naive   -- one global atomic per appended item;
//   ballot  -- one global atomic per wave and append step (wave prefix sum
//              by ballot and mbcnt);
//   staged  -- items staged in an LDS buffer per wave and flushed with one
//              global atomic per flush (the paper's per-block queue).
// The queue has a fixed capacity: appends past it are dropped and flagged;
// the propagation goes on with what the queues hold, and once they drain the
// queue is rebuilt from the current image by the dense seed detection, which
// is the paper's restart from a partial output after a global-queue overflow
// (Sec. 3.2, Sec. 5.2.4).  The result is rho_I(J) like every other schedule.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include "../../include/iwpp.h"
#include "iwpp_device.hpp"
#include "iwpp_internal.hpp"
#include "iwpp_runtime.hpp"

namespace iwpp {
namespace mrq {

constexpr int kWavesPerBlock = 4;
constexpr int kStageCap = 256;  // staged mode: LDS items per wave before a flush
constexpr uint32_t kMaxRounds = 1u << 22;

struct QArgs {
  const uint8_t* mask;
  uint8_t* out;       // the seed pass result on entry, rho_I(J) on exit
  uint32_t* J;        // [h*w] working copy, 32-bit words (atomic maximum)
  uint32_t* q[2];     // round queues, `cap` items each
  uint32_t* counts;   // [3 slots][64]: word 0 the slot's fill level, word 32 its lost flag
  GridBarrier* bar;
  unsigned long long* stats;
  unsigned long long* clock;
  uint32_t cap;
  int32_t h, w;
  int32_t mode;       // IWPP_QUEUE_NAIVE / _BALLOT / _STAGED
};

// Round r's queue is counted in slot r % 3 (appended during round r - 1);
// its lost flag is set when an append past the capacity was dropped.
__device__ __forceinline__ uint32_t* count_of(const QArgs& a, uint32_t slot) { return a.counts + slot * 64u; }
__device__ __forceinline__ uint32_t* lost_of(const QArgs& a, uint32_t slot) { return a.counts + slot * 64u + 32u; }

// Append `item` for every lane with `pred` to queue `qi` (counted by `cnt`),
// in the way `mode` says; returns nothing, drops past the capacity.
struct Appender {
  const QArgs& a;
  uint32_t* list;
  uint32_t* cnt;
  uint32_t* lost;
  WaveStage& st;
  __device__ void push(bool pred, uint32_t item) {
    if (a.mode == IWPP_QUEUE_NAIVE) {
      if (pred) {
        // One device-scope atomic per item.  Written out because the
        // compiler would otherwise combine the wave's increments of one
        // address into a single atomic (mbcnt offsets), which is the ballot
        // mode; the wait is inside the same statement.
        uint32_t slot;
        asm volatile("global_atomic_add %0, %1, %2, off sc0\n\ts_waitcnt vmcnt(0)"
                     : "=&v"(slot)
                     : "v"(cnt), "v"(1u)
                     : "memory");
        if (slot < a.cap) cstore(list + slot, item);
        else cstore(lost, 1u);
      }
    } else if (a.mode == IWPP_QUEUE_BALLOT) {
      const uint64_t m = ballot(pred);
      if (m == 0) return;
      uint32_t base = 0;
      if (lane() == 0) base = atomic_add(cnt, (uint32_t)__popcll(m));
      base = readlane(base, 0);
      if (pred) {
        const uint32_t slot = base + (uint32_t)mbcnt(m);
        if (slot < a.cap) cstore(list + slot, item);
        else cstore(lost, 1u);
      }
    } else {
      stage_append(st, pred, item, list, cnt, a.cap, lost);
    }
  }
  __device__ void flush() {
    if (a.mode == IWPP_QUEUE_STAGED) stage_flush(st, list, cnt, a.cap, lost);
  }
};

// Pixel p can raise a neighbour: some in-image q in N_G(p) with J(q) < J(p)
// and J(q) < I(q) (Algorithm 5's seed condition).  `J` is read with
// device-scope loads (other workgroups raise it during the kernel).
template <int CONN, bool kWords>
__device__ __forceinline__ bool is_seed(const QArgs& a, uint32_t p) {
  const int y = (int)(p / (uint32_t)a.w), x = (int)(p - (uint32_t)y * (uint32_t)a.w);
  const uint32_t jp = kWords ? cload(a.J + p) : (uint32_t)a.out[p];
  bool s = false;
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      if ((dy == 0 && dx == 0) || (CONN == 4 && dy != 0 && dx != 0)) continue;
      const int qy = y + dy, qx = x + dx;
      if (qy < 0 || qy >= a.h || qx < 0 || qx >= a.w) continue;
      const uint32_t q = (uint32_t)qy * (uint32_t)a.w + (uint32_t)qx;
      const uint32_t jq = kWords ? cload(a.J + q) : (uint32_t)a.out[q];
      s |= jq < jp && jq < (uint32_t)a.mask[q];
    }
  return s;
}

// The 32-bit working copy and the initial queue (round 0's, parity 0, slot 0).
template <int CONN>
__global__ __launch_bounds__(256) void k_init(QArgs a) {
  __shared__ uint32_t stage_mem[kWavesPerBlock][kStageCap];
  const int w = threadIdx.x / kWave;
  WaveStage st = {stage_mem[w], (uint32_t)kStageCap, 0u};
  Appender ap{a, a.q[0], count_of(a, 0u), lost_of(a, 0u), st};
  const uint32_t n = (uint32_t)a.h * (uint32_t)a.w;
  uint32_t seeds = 0;
  // whole waves iterate together (the appends are wave-wide)
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < n; base += stride) {
    const uint32_t p = base + (uint32_t)lane();
    bool s = false;
    if (p < n) {
      a.J[p] = a.out[p];
      s = is_seed<CONN, false>(a, p);
    }
    seeds += s ? 1u : 0u;
    ap.push(s, p);
  }
  ap.flush();
  for (int o = 32; o > 0; o >>= 1) seeds += __shfl_xor(seeds, o);
  if (lane() == 0) stat_add(a.stats, kStatSeeds, seeds);
}

// Rounds: pop every item of the round's queue (one per lane), raise the
// neighbours it can raise, queue those it raised.  When a queue lost items
// (capacity), the propagation continues with what it holds; once a round
// finds its queue empty after such a loss, it rebuilds the queue from the
// current image by dense seed detection (the restart from a partial output),
// and the propagation ends when a queue is empty with no loss outstanding.
// Every workgroup reads the same counts and flags after each barrier, so all
// take the same decisions.
template <int CONN>
__global__ __launch_bounds__(256) void k_prop(QArgs a) {
  __shared__ uint32_t stage_mem[kWavesPerBlock][kStageCap];
  __shared__ uint32_t nin_sh, lost_sh;
  const int w = threadIdx.x / kWave;
  WaveStage st = {stage_mem[w], (uint32_t)kStageCap, 0u};
  const uint32_t gw = blockIdx.x * kWavesPerBlock + (uint32_t)w, nw = gridDim.x * kWavesPerBlock;
  const uint32_t npx = (uint32_t)a.h * (uint32_t)a.w;
  uint32_t gen = 0, nclk = 0;
  unsigned long long pops = 0, raises = 0;
  uint32_t rounds = 0, restarts = 0;
  bool pending_loss = false;  // a queue lost items and no rebuild has followed yet
  clock_stamp(a.clock, nclk);
  for (uint32_t r = 0;; ++r) {
    const uint32_t par = r & 1u, slot = r % 3u;
    if (threadIdx.x == 0) {
      const uint32_t c = cload(count_of(a, slot));
      nin_sh = c < a.cap ? c : a.cap;
      lost_sh = cload(lost_of(a, slot));
    }
    __syncthreads();
    const uint32_t nin = nin_sh;
    pending_loss |= lost_sh != 0u;
    const bool rebuild = nin == 0u && pending_loss;
    if (nin == 0u && !rebuild) break;
    if (r >= kMaxRounds) {
      if (blockIdx.x == 0 && threadIdx.x == 0) stat_add(a.stats, kStatError, 1ull);
      break;
    }
    round_work(a.clock, r, rebuild ? npx : nin);
    // Slot (r+2)%3 was last read in round r-1 and is next appended to in
    // round r+1, after this round's barrier.
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      cstore(count_of(a, (r + 2u) % 3u), 0u);
      cstore(lost_of(a, (r + 2u) % 3u), 0u);
    }
    Appender ap{a, a.q[par ^ 1u], count_of(a, (r + 1u) % 3u), lost_of(a, (r + 1u) % 3u), st};
    if (rebuild) {
      for (uint32_t base = gw * kWave; base < npx; base += nw * kWave) {
        const uint32_t p = base + (uint32_t)lane();
        const bool s = p < npx && is_seed<CONN, true>(a, p);
        ap.push(s, p);
      }
      pending_loss = false;
      restarts++;
    } else {
      const uint32_t* qin = a.q[par];
      for (uint32_t base = gw * kWave; base < nin; base += nw * kWave) {
        const uint32_t i = base + (uint32_t)lane();
        uint32_t raised = 0u;  // bit k: neighbour k raised by this lane
        uint32_t qs[8] = {};
        if (i < nin) {
          const uint32_t p = cload(qin + i);
          pops++;
          const int y = (int)(p / (uint32_t)a.w), x = (int)(p - (uint32_t)y * (uint32_t)a.w);
          const uint32_t jp = cload(a.J + p);
          int k = 0;
#pragma unroll
          for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
              if ((dy == 0 && dx == 0) || (CONN == 4 && dy != 0 && dx != 0)) continue;
              const int qy = y + dy, qx = x + dx;
              if (qy >= 0 && qy < a.h && qx >= 0 && qx < a.w) {
                const uint32_t q = (uint32_t)qy * (uint32_t)a.w + (uint32_t)qx;
                const uint32_t iq = a.mask[q], jq = cload(a.J + q);
                const uint32_t v = jp < iq ? jp : iq;
                if (jq < v && atomic_max(a.J + q, v) < v) raised |= 1u << k;
                qs[k] = q;
              }
              ++k;
            }
        }
#pragma unroll
        for (int k = 0; k < (CONN == 8 ? 8 : 4); ++k) {
          const bool pred = (raised >> k) & 1u;
          raises += pred ? 1u : 0u;
          ap.push(pred, qs[k]);
        }
      }
    }
    ap.flush();
    rounds++;
    if (!grid_barrier(a.bar, gen, a.stats)) return;
    clock_stamp(a.clock, nclk);
  }
  // The result back to bytes.
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += gridDim.x * blockDim.x)
    a.out[p] = (uint8_t)cload(a.J + p);
  for (int o = 32; o > 0; o >>= 1) {
    pops += __shfl_xor(pops, o);
    raises += __shfl_xor(raises, o);
  }
  if (lane() == 0) {
    stat_add(a.stats, kStatItems, pops);
    stat_add(a.stats, kStatUpdates, raises);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    stat_add(a.stats, kStatRounds, rounds);
    stat_add(a.stats, kStatRestarts, restarts);
  }
}

}  // namespace mrq
}  // namespace iwpp

using namespace iwpp::rt;

extern "C" int32_t iwpp_morph_recon_queue_u8(iwpp_ctx* ctx, const uint8_t* marker, const uint8_t* mask, uint8_t* out,
                                             int32_t height, int32_t width, int32_t conn,
                                             const iwpp_queue_options* qopt, void* stream) {
  using namespace iwpp;
  if (!ctx) return IWPP_EINVAL;
  if (ctx->server) return fail(ctx, IWPP_EBUSY, "morph_recon_queue: the context is serving");
  if (!marker || !mask || !out) return fail(ctx, IWPP_EINVAL, "morph_recon_queue: NULL image pointer");
  iwpp_queue_options q{};
  q.append_mode = IWPP_QUEUE_STAGED;
  if (qopt) q = *qopt;
  if (q.append_mode < IWPP_QUEUE_NAIVE || q.append_mode > IWPP_QUEUE_STAGED || q.capacity < 0 || q.seed_sweeps < 0)
    return fail(ctx, IWPP_EINVAL, "morph_recon_queue: bad queue options");
  const uint64_t np = (uint64_t)(height > 0 ? height : 0) * (uint64_t)(width > 0 ? width : 0);
  if (np >= (1ull << 31)) return fail(ctx, IWPP_EINVAL, "morph_recon_queue: at most 2^31 - 1 pixels");
  iwpp_job j{IWPP_OP_RECON, conn, height, width, marker, mask, out, nullptr};
  Plan plan;
  int32_t rc = build_plan(ctx, &j, 1, "morph_recon_queue", plan);
  if (rc != IWPP_OK) return rc;
  const uint64_t cap = q.capacity > 0 ? (uint64_t)q.capacity : 2 * np + 64;
  if (cap >= (1ull << 32)) return fail(ctx, IWPP_EINVAL, "morph_recon_queue: capacity above 2^32 - 1");
  // scratch: the seed pass's group scratch | J words | two queues
  const size_t sb = align256(plan.scratch_bytes);
  const size_t jb = align256(4 * np), qb = align256(4 * cap);
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, IWPP_EDEVICE, "morph_recon_queue: cannot select the context's device");
  if ((rc = ensure_scratch(ctx, sb + jb + 2 * qb)) != IWPP_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // 1. the tile seed pass only, `seed_sweeps` sweep iterations per tile
  iwpp_options saved = ctx->opt;
  ctx->opt.mr_seed_sweeps = q.seed_sweeps;
  Group seed = plan.groups[0];
  rc = launch_group(ctx, seed, ctx->scratch, ctx->fixed, nullptr, st, true, &ctx->rec, /*seed_only=*/true);
  ctx->opt = saved;
  if (rc != IWPP_OK) return rc;
  // 2. working copy and initial queue; 3. rounds (the statistics of the seed
  // pass are cleared: the counters describe the queue)
  mrq::QArgs a{};
  a.mask = mask;
  a.out = out;
  a.J = reinterpret_cast<uint32_t*>(ctx->scratch + sb);
  a.q[0] = reinterpret_cast<uint32_t*>(ctx->scratch + sb + jb);
  a.q[1] = reinterpret_cast<uint32_t*>(ctx->scratch + sb + jb + qb);
  a.counts = reinterpret_cast<uint32_t*>(ctx->fixed + kOffCounts);
  a.bar = reinterpret_cast<iwpp::GridBarrier*>(ctx->fixed + kOffBarrier);
  a.stats = reinterpret_cast<unsigned long long*>(ctx->fixed + kOffStats);
  a.clock = reinterpret_cast<unsigned long long*>(ctx->fixed + kOffClock);
  a.cap = (uint32_t)cap;
  a.h = height;
  a.w = width;
  a.mode = q.append_mode;
  ctx->rec.begin(IWPP_K_RESET, st);
  const int zr = zero_words(reinterpret_cast<uint32_t*>(ctx->fixed), kFixedBytes / 4, st);
  ctx->rec.end(st);
  if (zr != 0) return fail(ctx, IWPP_EDEVICE, "morph_recon_queue: reset launch failed");
  const uint32_t blocks_init = (uint32_t)((np + 255) / 256 < 8192 ? (np + 255) / 256 : 8192);
  ctx->rec.begin(IWPP_K_MRQ_INIT, st);
  if (conn == 8)
    hipLaunchKernelGGL(mrq::k_init<8>, dim3(blocks_init), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(mrq::k_init<4>, dim3(blocks_init), dim3(256), 0, st, a);
  ctx->rec.end(st);
  if (hipGetLastError() != hipSuccess) return fail(ctx, IWPP_EDEVICE, "morph_recon_queue: init launch failed");
  const void* fn = conn == 8 ? reinterpret_cast<const void*>(&mrq::k_prop<8>) : reinterpret_cast<const void*>(&mrq::k_prop<4>);
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0) != hipSuccess || per_cu < 1)
    return fail(ctx, IWPP_EDEVICE, "morph_recon_queue: occupancy query failed");
  uint32_t blocks = persistent_grid(fn, per_cu, cus);
  if (ctx->opt.persistent_blocks > 0 && (uint32_t)ctx->opt.persistent_blocks < blocks)
    blocks = (uint32_t)ctx->opt.persistent_blocks;
  void* kargs[] = {&a};
  ctx->rec.begin(IWPP_K_MRQ_PROPAGATE, st);
  const hipError_t le = launch_persistent(fn, blocks, kargs, st);
  ctx->rec.end(st);
  if (le != hipSuccess) return fail(ctx, IWPP_EDEVICE, "morph_recon_queue: propagation launch failed");
  ctx->last_stream = st;
  ctx->last_fixed = ctx->fixed;
  ctx->last_op = 1;
  ctx->have_call = true;
  return IWPP_OK;
}
