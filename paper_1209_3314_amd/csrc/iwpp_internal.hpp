// Internal declarations shared by the host library and the kernel sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace iwpp {

struct GridBarrier;

// Tile geometry shared by the host plans and the kernels.
constexpr int kMrTile = 64;   // reconstruction tiles: 64 x 64 pixels
constexpr int kEdtHalo = 4;   // EDT rounds per tile visit (= halo width; 8 measured slower)
constexpr int kEdtTile = 26;  // EDT tiles: 26 x 26 pixels (a 34 x 34 region with the halo)
constexpr size_t kEdtStatePad = 256;  // bytes after each EDT state buffer (16-byte loads may cross the end)

// One reconstruction image of a launch.
struct MrJob {
  const uint8_t* marker;
  const uint8_t* mask;
  uint8_t* out;
  int32_t h, w;
  int32_t tiles_y, tiles_x;
  uint32_t tile_base;  // first global tile id of this image
  // 0 for reconstruction by dilation; all ones for reconstruction by
  // erosion, computed as the dilation of the complemented images (every
  // image byte is complemented as it is loaded and stored).
  uint32_t inv;
};

// Reconstruction launch arguments (device pointers, scratch owned by the context).
// A launch processes njobs images; global tile ids run over all of them.
struct MrArgs {
  MrJob job0;                // the image when njobs == 1 (no table lookup)
  const MrJob* jobs;         // [njobs] device table when njobs > 1
  uint32_t* tile_job;        // [ntiles] image of each global tile when njobs > 1
  uint32_t njobs;
  uint32_t ntiles;           // total tiles over all images
  uint32_t list_cap;         // capacity of each round's tile list (<= ntiles)
  int32_t max_sweeps;        // sweep iterations per propagation visit before re-listing
  int32_t seed_sweeps;       // sweep iterations per tile in the seed pass
  uint32_t seed_only;        // nonzero: stop after the seed pass (round 0)
  uint32_t seed_strip;       // seed pass: tiles per strip (0 = automatic)
  uint32_t stage_depth;      // work-list items staged per wave before a flush (0 = the LDS maximum)
  uint32_t wg_waves;         // waves per workgroup: 4 or 8
  uint32_t* flags;           // [2][ntiles] tile on the round's list, per round parity
  uint32_t* lists;           // [2][8 shards][ntiles] tile lists per round parity
  uint32_t* unsettled;       // [ntiles] the tile's last visit stopped at the sweep cap
  uint8_t* cols;             // [ntiles][4][64] each tile's border columns: J left, J right, I left, I right
  uint32_t* counts;          // [3 round slots][8 shards][64] list fill levels (256 B apart)
  uint32_t* lost;            // [2][64] a listed tile was dropped (capacity), per parity
  GridBarrier* bar;
  unsigned long long* stats;  // [8 shards][16 fields]
  unsigned long long* clock;  // [kClockWords] round timeline (see kClockWords)
};

// One distance-transform image of a launch.
struct EdtJob {
  const uint8_t* bin;
  int32_t* sqdist;
  int32_t* nearest;
  int32_t h, w;
  int32_t tiles_y, tiles_x;  // kEdtTile x kEdtTile tiles
  uint32_t tile_base;        // first global tile id of this image
  uint32_t pad;
  unsigned long long pix_base;  // first global pixel id of this image
};

// Distance-transform launch arguments.  Global pixel id = pix_base + y*w + x;
// global tile ids run over all images.
struct EdtArgs {
  EdtJob job0;                // the image when njobs == 1
  const EdtJob* jobs;         // [njobs] device table when njobs > 1
  uint32_t* tile_job;         // [ntiles] image of each global tile when njobs > 1
  uint32_t njobs;
  uint32_t ntiles;
  uint32_t wide;              // nonzero: wide coordinate fields (an image side above 32767)
  uint32_t pad0;
  unsigned long long npix;    // total pixels over all images
  uint32_t* feat0;            // [npix] nearest feature (y << 16 | x), ~0 = none; round parity 0
  uint32_t* feat1;            // [npix] round parity 1
  uint32_t* flags;            // [2][ntiles] tile on the round's list, per round parity
  uint32_t* lists;            // [2][8 shards][ntiles] tile lists per round parity
  uint32_t* stamps;           // [2][ntiles] step of the tile's last visit, per step parity (0 = none)
  uint32_t* marks;            // [2][ntiles][32] that visit's last-round change mask, one word per tile row
  uint32_t* counts;           // [3 round slots][8 shards][64] list fill levels (256 B apart)
  uint32_t* ovf;              // never set: a list holds each tile once
  uint32_t stage_depth;       // work-list items staged per wave before a flush (0 = the LDS maximum)
  uint32_t wg_waves;          // waves per workgroup of the rounds kernel: 4 or 8
  GridBarrier* bar;
  unsigned long long* stats;
  unsigned long long* clock;  // [kClockWords] round timeline (see kClockWords)
};

// Bytes of the scratch areas the kernels expect.
constexpr size_t kBarrierBytes = 4096;
constexpr size_t kCountsBytes = 3 * 8 * 64 * 4;
// Round timeline: word 0 = stamps written, words 1..255 realtime-clock stamps
// (kernel start, then after every grid barrier) of one workgroup, words
// 256 + i the tiles visited in phase i.
constexpr int kClockWords = 512;
constexpr size_t kLostBytes = 2 * 64 * 4;
constexpr size_t kStatsBytes = 8 * 16 * 8;

// Optional per-launch event timing (iwpp_options.profile).  begin/end bracket
// one kernel launch on `s`; both are no-ops when disabled or full.
class Recorder {
 public:
  static constexpr int kCap = 4096;
  bool enabled = false;
  void begin(int kernel, hipStream_t s);
  void end(hipStream_t s);
  // Completed records since the last read: returns the count written.
  int read(int* kernels, float* ms, int max);
  void release();

 private:
  hipEvent_t start_[kCap] = {};
  hipEvent_t stop_[kCap] = {};
  int kernel_[kCap] = {};
  int created_ = 0;
  int count_ = 0;
  bool open_ = false;
};

int mr_launch(const MrArgs& a, int conn, int persistent_blocks, hipStream_t stream, Recorder* rec, const char** err);
int edt_launch(const EdtArgs& a, int conn, int persistent_blocks, hipStream_t stream, Recorder* rec, const char** err);
int zero_words(uint32_t* p, size_t nwords, hipStream_t stream);

// Workgroups for a cooperative (persistent) launch of `fn`: every one must be
// resident at once, since they meet at grid barriers.  The runtime's occupancy
// figure is capped by the 160 KiB of LDS of a CU and by `max_per_cu`
// workgroups per CU (4 unless the kernel's registers and LDS fit more); grids
// sized from the raw figure (8 per CU for a 16 KiB kernel) were measured not
// to be co-resident on MI355X, while these caps are.
uint32_t persistent_grid(const void* fn, int per_cu, int cus, int max_per_cu = 4);

// Launch a persistent kernel: a cooperative launch (the runtime checks that the
// whole grid is resident), or a plain launch of the same grid while `s` is being
// captured into a graph.  Inside a graph, residency then rests on the grid
// fitting the device when the graph runs alone; a grid that does not fit makes
// the grid barrier time out and report an error instead of waiting forever.
hipError_t launch_persistent(const void* fn, uint32_t blocks, void** args, hipStream_t s, uint32_t threads = 256);

}  // namespace iwpp
