// Propagation-based Euclidean distance transform on gfx950.
//
// What is computed (Sec. 2.2, Algorithms 3 and 6): every pixel carries a
// nearest feature (the paper's VR), initially itself for features (0-pixels)
// and "none" otherwise; features are propagated to neighbours in N_G when they
// are closer; the output is the squared distance to the carried feature and
// its index.  The propagation runs in level-synchronous rounds -- Algorithm 4's
// swap of input and output queues, made device-wide -- and a pixel offers the
// feature it held at the end of the previous round.  Round r therefore equals
// the dense operator key_r(q) = min over p in N_G[q] of (d2(q, f_{r-1}(p)),
// f_{r-1}(p)), so the result does not depend on thread order.
//
// State.  A pixel's key is the 64-bit word (d2 << 32) | (fy << 16) | fx;
// unsigned comparison orders keys by squared distance, then by feature row,
// then column -- i.e. by (d2, feature index) -- and the CAS-retry loop of
// Algorithm 6 becomes one 64-bit atomic min.  Two key buffers alternate per
// round: round r reads buffer (r-1)&1, which no one writes during the round,
// and lowers buffer r&1 with atomic min.  Buffer r&1 holds the state of round
// r-2; a pixel that changed in round r-1 is brought up to date by its own
// frontier item with one more atomic min, and min makes the order of that
// catch-up and the offers irrelevant.
//
// Frontier.  A pixel joins the next round's frontier the first time an offer
// improves it in a round (a round stamp, updated with atomic max, makes the
// frontier a set).  Items are staged per wave in LDS and flushed with one
// atomic per batch.  Rounds are separated by a grid barrier.
#include "iwpp_device.hpp"
#include "iwpp_internal.hpp"

namespace iwpp {
namespace edt {

constexpr int kWavesPerBlock = 4;
constexpr int kStageCap = 1024;
constexpr unsigned long long kNone = ~0ull;
constexpr uint32_t kMaxRounds = 1u << 20;

__device__ __forceinline__ uint32_t pack_yx(int y, int x) { return ((uint32_t)y << 16) | (uint32_t)x; }

// Neighbour k of N_G (raster order; 4-connectivity uses the 4 axis neighbours).
template <int CONN>
__device__ __forceinline__ void nb_off(int k, int& dy, int& dx) {
  if (CONN == 8) {
    dy = k < 3 ? -1 : (k < 5 ? 0 : 1);
    dx = (k == 0 || k == 3 || k == 5) ? -1 : ((k == 1 || k == 6) ? 0 : 1);
  } else {
    dy = k == 0 ? -1 : (k == 3 ? 1 : 0);
    dx = k == 1 ? -1 : (k == 2 ? 1 : 0);
  }
}

__device__ __forceinline__ unsigned long long make_item(uint32_t job, int y, int x) {
  return ((unsigned long long)job << 32) | pack_yx(y, x);
}

__device__ __forceinline__ const EdtJob& job_of(const EdtArgs& a, uint32_t j) { return a.njobs == 1u ? a.job0 : a.jobs[j]; }

// Initial state and the first frontier: the contour features (features with a
// non-feature neighbour, Algorithm 6 initialisation).  blockIdx.y = image.
template <int CONN>
__global__ __launch_bounds__(256) void k_init(EdtArgs a) {
  __shared__ unsigned long long stage_mem[kWavesPerBlock][kStageCap];
  const int w = threadIdx.x / kWave;
  WaveStageT<unsigned long long> s = {stage_mem[w], (uint32_t)kStageCap, 0u};
  const uint32_t j = blockIdx.y;
  const EdtJob job = job_of(a, j);
  const uint32_t npx = (uint32_t)job.h * (uint32_t)job.w;
  unsigned long long* list1 = a.lists + a.npix;  // the first frontier is read by round 1: list parity 1, count slot 1
  uint32_t contour = 0;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < npx; base += stride) {
    const uint32_t p = base + (uint32_t)lane();
    const bool valid = p < npx;
    bool c = false;
    int y = 0, x = 0;
    if (valid) {
      y = (int)(p / (uint32_t)job.w);
      x = (int)(p - (uint32_t)y * (uint32_t)job.w);
      const bool feat = job.bin[p] == 0;
      const unsigned long long k0 = feat ? (unsigned long long)pack_yx(y, x) : kNone;
      a.key0[job.pix_base + p] = k0;
      a.key1[job.pix_base + p] = k0;
      a.stamp[job.pix_base + p] = 0u;
      if (feat) {
#pragma unroll
        for (int k = 0; k < CONN; ++k) {
          int dy, dx;
          nb_off<CONN>(k, dy, dx);
          const int qy = y + dy, qx = x + dx;
          if (qy >= 0 && qy < job.h && qx >= 0 && qx < job.w &&
              job.bin[(uint32_t)qy * (uint32_t)job.w + (uint32_t)qx] != 0)
            c = true;
        }
      }
      contour += c ? 1u : 0u;
    }
    stage_append(s, c, make_item(j, y, x), list1, a.counts + 64, a.npix, a.ovf);
  }
  stage_flush(s, list1, a.counts + 64, a.npix, a.ovf);
  uint32_t tot = contour;
  for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
  if (lane() == 0) stat_add(a.stats, kStatSeeds, tot);
}

template <int CONN>
__global__ __launch_bounds__(256) void k_rounds(EdtArgs a) {
  __shared__ unsigned long long stage_mem[kWavesPerBlock][kStageCap];
  __shared__ uint32_t nshared;
  const int w = threadIdx.x / kWave;
  WaveStageT<unsigned long long> s = {stage_mem[w], (uint32_t)kStageCap, 0u};
  const uint32_t gw = blockIdx.x * kWavesPerBlock + w, nw = gridDim.x * kWavesPerBlock;
  uint32_t gen = 0;
  unsigned long long items = 0, updates = 0;
  uint32_t r = 1;
  for (;; ++r) {
    if (threadIdx.x == 0) nshared = cload(a.counts + (r % 3u) * 64u);
    __syncthreads();
    uint32_t n = nshared;
    if (n == 0u) break;
    if (r >= kMaxRounds) {  // safety limit: report instead of spinning on a logic error
      if (blockIdx.x == 0 && threadIdx.x == 0) stat_add(a.stats, kStatError, 1ull);
      break;
    }
    if (n > a.npix) n = a.npix;
    items += n;
    if (blockIdx.x == 0 && threadIdx.x == 0) cstore(a.counts + ((r + 2u) % 3u) * 64u, 0u);
    const unsigned long long* rd = (r & 1u) ? a.key0 : a.key1;  // buffer (r-1)&1
    unsigned long long* wr = (r & 1u) ? a.key1 : a.key0;        // buffer r&1
    const unsigned long long* list = a.lists + (size_t)(r & 1u) * a.npix;
    unsigned long long* nlist = a.lists + (size_t)((r + 1u) & 1u) * a.npix;
    uint32_t* ncount = a.counts + ((r + 1u) % 3u) * 64u;
    for (uint32_t base = gw * kWave; base < n; base += nw * kWave) {
      const uint32_t i = base + (uint32_t)lane();
      const bool valid = i < n;
      const unsigned long long it = valid ? cload(list + i) : 0ull;
      const uint32_t j = (uint32_t)(it >> 32);
      const int py = (int)((uint32_t)it >> 16), px = (int)((uint32_t)it & 0xffffu);
      int h = 1, wd = 1;
      uint32_t pb = 0;
      if (valid) {
        const EdtJob& job = job_of(a, j);
        h = job.h;
        wd = job.w;
        pb = job.pix_base;
      }
      const uint32_t p = pb + (uint32_t)py * (uint32_t)wd + (uint32_t)px;
      // Issue every independent access of the item together (one round trip
      // each for: its own key and its neighbours' previous keys; the atomic
      // mins; the stamps) instead of one chain per neighbour.
      uint32_t q[CONN];
      bool in[CONN];
      unsigned long long prev[CONN];
#pragma unroll
      for (int k = 0; k < CONN; ++k) {
        int dy, dx;
        nb_off<CONN>(k, dy, dx);
        const int qy = py + dy, qx = px + dx;
        in[k] = valid && qy >= 0 && qy < h && qx >= 0 && qx < wd;
        q[k] = in[k] ? pb + (uint32_t)qy * (uint32_t)wd + (uint32_t)qx : 0u;
      }
      const unsigned long long sk = valid ? cload(rd + p) : kNone;
#pragma unroll
      for (int k = 0; k < CONN; ++k) prev[k] = in[k] ? cload(rd + q[k]) : 0ull;
      if (valid && r > 1u) atomic_min(wr + p, sk);  // catch up: this pixel changed in round r-1
      const uint32_t f = (uint32_t)sk;
      const int fy = (int)(f >> 16), fx = (int)(f & 0xffffu);
      unsigned long long cand[CONN], old[CONN];
#pragma unroll
      for (int k = 0; k < CONN; ++k) {
        int dy, dx;
        nb_off<CONN>(k, dy, dx);
        const int ey = py + dy - fy, ex = px + dx - fx;
        cand[k] = ((unsigned long long)(uint32_t)(ey * ey + ex * ex) << 32) | f;
        old[k] = (in[k] && cand[k] < prev[k]) ? atomic_min(wr + q[k], cand[k]) : 0ull;
      }
      bool fresh[CONN];
#pragma unroll
      for (int k = 0; k < CONN; ++k) {
        const bool improved = in[k] && cand[k] < prev[k] && cand[k] < old[k];
        fresh[k] = improved ? atomic_max(a.stamp + q[k], r) < r : false;
        updates += fresh[k] ? 1u : 0u;
      }
#pragma unroll
      for (int k = 0; k < CONN; ++k) {
        int dy, dx;
        nb_off<CONN>(k, dy, dx);
        stage_append(s, fresh[k], make_item(j, py + dy, px + dx), nlist, ncount, a.npix, a.ovf);
      }
    }
    stage_flush(s, nlist, ncount, a.npix, a.ovf);
    if (!grid_barrier(a.bar, gen, a.stats)) return;
  }
  // Finalize: buffer (r-1)&1 holds the state after the last round.
  const unsigned long long* fin = (r & 1u) ? a.key0 : a.key1;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t j = 0; j < a.njobs; ++j) {
    const EdtJob& job = job_of(a, j);
    const uint32_t npx = (uint32_t)job.h * (uint32_t)job.w;
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += stride) {
      const unsigned long long k = cload(fin + job.pix_base + p);
      if (k == kNone) {
        job.sqdist[p] = -1;
        job.nearest[p] = -1;
      } else {
        const uint32_t f = (uint32_t)k;
        job.sqdist[p] = (int32_t)(k >> 32);
        job.nearest[p] = (int32_t)((f >> 16) * (uint32_t)job.w + (f & 0xffffu));
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) updates += __shfl_xor(updates, o);
  if (lane() == 0) stat_add(a.stats, kStatUpdates, updates);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    stat_add(a.stats, kStatItems, items);
    stat_add(a.stats, kStatRounds, r >= 2u ? r - 2u : 0u);
  }
}

}  // namespace edt

int edt_launch(const EdtArgs& a, int conn, int persistent_blocks, hipStream_t stream, Recorder* rec, const char** err) {
  using namespace edt;
  // blocks per image: enough to fill the device when spread over the images
  uint32_t per_job = (2048u + a.njobs - 1u) / a.njobs;
  const uint32_t avg = (a.npix / a.njobs + 255u) / 256u;
  if (per_job > avg) per_job = avg;
  if (per_job < 1u) per_job = 1u;
  rec->begin(4, stream);
  if (conn == 8)
    hipLaunchKernelGGL(k_init<8>, dim3(per_job, a.njobs), dim3(256), 0, stream, a);
  else
    hipLaunchKernelGGL(k_init<4>, dim3(per_job, a.njobs), dim3(256), 0, stream, a);
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
  const hipError_t le = hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(256), kargs, 0, stream);
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
    const int by_lds = (int)((128u * 1024u) / (unsigned)fa.sharedSizeBytes);
    if (by_lds < lim) lim = by_lds;
  }
  if (lim < 1) lim = 1;
  return (uint32_t)lim * (uint32_t)cus;
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
