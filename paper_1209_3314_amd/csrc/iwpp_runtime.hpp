// Host runtime shared by the C ABI entry points and the serving loop:
// the context, launch plans (images grouped by operation and connectivity),
// scratch layout and group launches.  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/iwpp.h"
#include "iwpp_internal.hpp"

namespace iwpp::rt {

constexpr size_t kOffBarrier = 0;
constexpr size_t kOffCounts = kOffBarrier + iwpp::kBarrierBytes;
constexpr size_t kOffLost = kOffCounts + iwpp::kCountsBytes;
constexpr size_t kOffOvf = kOffLost + iwpp::kLostBytes;
constexpr size_t kOffStats = kOffOvf + 256;
constexpr size_t kOffClock = kOffStats + iwpp::kStatsBytes;  // round timeline of the last group
constexpr size_t kFixedBytes = kOffClock + iwpp::kClockWords * 8;
static_assert(kOffStats % 8 == 0, "stats must be 8-byte aligned");

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// One (operation, connectivity) group of a plan.
struct Group {
  int op = 0;
  int conn = 8;
  std::vector<iwpp::MrJob> mr;
  std::vector<iwpp::EdtJob> edt;
  uint64_t ntiles = 0;
  uint64_t npix = 0;
  size_t table_off = 0;  // offset of this group's job table in the table area

  uint32_t njobs() const { return (uint32_t)(op == IWPP_OP_RECON ? mr.size() : edt.size()); }
  size_t table_bytes() const {
    return njobs() > 1 ? align256(op == IWPP_OP_RECON ? mr.size() * sizeof(iwpp::MrJob) : edt.size() * sizeof(iwpp::EdtJob))
                       : 0;
  }
  // Scratch layout (T = tiles, arrays of u32, each 256-byte aligned).
  // Recon: flags[2][T] | lists[2][8][T] | unsettled[T] | tile_job[T] | cols[T][256 B].
  // EDT: feat0 | feat1 | flags[2][T] | lists[2][8][T] | tile_job[T] | stamps[2][T] | marks[2][T][128 B].
  size_t scratch_bytes() const {
    const size_t tb = align256(ntiles * 4);
    return op == IWPP_OP_EDT ? 2 * (align256(npix * 4) + iwpp::kEdtStatePad) + 21 * tb + ntiles * 256
                             : 20 * tb + ntiles * 256;
  }
};

struct Plan {
  std::vector<Group> groups;
  size_t scratch_bytes = 0;  // max over groups (groups run one after another)
  size_t table_bytes = 0;    // sum over groups
};

// Sides the distance transform accepts: at most 46340 each, and every squared
// distance ((h-1)^2 + (w-1)^2 at most) below 2^31 so it fits the int32 output.
bool edt_dims_ok(int32_t h, int32_t w);

// Scratch bytes one image adds to a group (upper bound, used for admission).
size_t job_scratch_bytes(int op, int32_t h, int32_t w);

// Makes `dev` current for the duration of a call and restores the caller's device.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev);
  ~DeviceGuard();
};

}  // namespace iwpp::rt

struct iwpp_server;

struct iwpp_ctx {
  int device = 0;
  iwpp_options opt{};
  std::string err;
  uint8_t* fixed = nullptr;    // barrier | counts | lost | ovf | stats
  uint8_t* scratch = nullptr;  // growable: group scratch, then job tables
  size_t scratch_bytes = 0;
  hipStream_t last_stream = nullptr;
  uint8_t* last_fixed = nullptr;  // fixed area of the last call (the context's, or the static one)
  int last_op = 0;
  bool have_call = false;
  iwpp_server* server = nullptr;  // a running server owns the context
  uint8_t* noalloc = nullptr;     // device address of the static work area on this device (null: unavailable)
  iwpp::Recorder rec;
};

namespace iwpp::rt {

int32_t fail(iwpp_ctx* ctx, int32_t code, const std::string& msg);
// Validate the jobs and group them by (op, conn).  `who` prefixes messages.
int32_t build_plan(iwpp_ctx* ctx, const iwpp_job* jobs, int32_t n, const char* who, Plan& plan);
// Copy every group's job table from host `src` tables (or the plan itself when
// `host` is null) into `tables` (device) on `st`; `sync` waits for the copy.
int32_t upload_tables(iwpp_ctx* ctx, const Plan& plan, uint8_t* tables, hipStream_t st, bool sync);
// Serialise the plan's job tables into `host` (plan.table_bytes bytes).
void pack_tables(const Plan& plan, uint8_t* host);
// Launch the kernels of one group on `st`; `first` also clears the statistics;
// `seed_only` stops a reconstruction group after its seed pass.
int32_t launch_group(iwpp_ctx* ctx, const Group& g, uint8_t* scratch, uint8_t* fixed, uint8_t* tables, hipStream_t st,
                     bool first, iwpp::Recorder* rec, bool seed_only = false);
// Grow the context's scratch to at least `bytes` (waits for the device first
// if a smaller buffer must be freed).
int32_t ensure_scratch(iwpp_ctx* ctx, size_t bytes);
// Sum the sharded statistics words copied from a fixed area.
// (The round timeline is read by iwpp_round_times.)
void fold_stats(const unsigned long long* shards, int op, iwpp_stats* out);
// Look up the static work area of iwpp_morph_recon_u8_noalloc on the context's
// device (which must be current) once per device and store it in ctx->noalloc.
int32_t noalloc_setup(iwpp_ctx* ctx);
// Bytes of the static area left for a group's scratch after its fixed area.
size_t noalloc_group_limit();

}  // namespace iwpp::rt
