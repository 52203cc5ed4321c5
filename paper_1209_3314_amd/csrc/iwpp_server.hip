// Serving loop: jobs arrive one by one from the host, are admitted against a
// device-memory budget and a slot limit, uploaded on a copy stream, run in
// batches on a compute stream (all admitted jobs that are not yet running
// form the next batch: continuous batching) and downloaded on a second copy
// stream.  A resident server takes jobs whose images are already on the
// device and skips the copies.  The paper's runtime hands independent tiles to
// whichever device is free, first come first served (Sec. 4); here one device
// takes them in batches, which fills it with many small tiles at once.
//
// Concurrency: one worker thread owns the device side (streams, arena,
// batches); submit/poll/drain/stats take a mutex shared with it.  A batch
// takes the admitted jobs whose uploads have finished; at most two batches are
// queued on the compute stream, so the device goes from one batch to the next
// without a host round trip while later arrivals still join the batch after,
// and uploads, computation and downloads of successive batches overlap.  While
// a batch computes and uploads are still arriving, the next batch waits until
// it is at least as large as the computing one (bursts form large batches),
// and an idle device takes the oldest job alone (it completes as a plain call
// would; the others follow in the next batch).
// Batches share the context's fixed area and one scratch buffer: they run one
// after another in stream order.  A batch runs as one launch sequence per
// (operation, connectivity) group; each group's jobs are downloaded and
// completed as soon as that group's kernels end, so a small reconstruction
// does not wait for a large distance transform launched after it.
#include <hip/hip_runtime.h>
#include <time.h>

#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/iwpp.h"
#include "iwpp_device.hpp"
#include "iwpp_internal.hpp"
#include "iwpp_runtime.hpp"

namespace {

using iwpp::rt::align256;

int64_t mono_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (int64_t)ts.tv_sec * 1000000000ll + ts.tv_nsec;
}

// First-fit allocator over one device range, 256-byte granules, coalescing frees.
class Arena {
 public:
  void init(size_t bytes) {
    free_.clear();
    size_ = bytes & ~size_t(255);
    if (size_) free_[0] = size_;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align256(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(bytes ? bytes : 1);
    used_ -= bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  std::map<size_t, size_t> free_;  // offset -> length
  size_t size_ = 0;
  size_t used_ = 0;
};

size_t job_buffer_bytes(const iwpp_job& j) {
  const size_t np = (size_t)j.height * (size_t)j.width;
  // recon: mask | marker (the output is written in place over the marker copy)
  // EDT: binary | sqdist | nearest
  return j.op != IWPP_OP_EDT ? 2 * align256(np) : align256(np) + 2 * align256(4 * np);
}

struct SJob {
  iwpp_job host{};  // caller's host buffers
  int64_t arrival_ns = 0;
  int64_t done_ns = 0;
  int32_t state = IWPP_JOB_QUEUED;
  size_t off = 0, bytes = 0;
  iwpp_job dev{};             // the same job on device buffers
  hipEvent_t up = nullptr;    // recorded after the job's uploads
  hipEvent_t ready = nullptr; // recorded on the caller's stream at submit
};

// The jobs of one (operation, connectivity) group of a batch.
struct Part {
  std::vector<uint64_t> tickets;
  hipEvent_t done = nullptr;  // the group's kernels (and its statistics copy) ended
  hipEvent_t down = nullptr;  // its outputs are on the host
};

struct Batch {
  std::vector<Part> parts;
  size_t jobs = 0;
  size_t next = 0;  // first part not yet complete
  int slot = -1;
  bool failed = false;  // the launch sequence could not be enqueued
};

constexpr int kSlots = 4;             // pinned table/statistics slots = batches in flight at most
constexpr int kMaxGroups = 4;         // (operation, connectivity) groups of a plan
constexpr int kMaxComputingBatches = 2;  // batches queued or running on the compute stream
constexpr size_t kStatWords = iwpp::kStatShards * iwpp::kStatFields;

}  // namespace

struct iwpp_server {
  iwpp_ctx* ctx = nullptr;
  iwpp_server_options opt{};
  size_t budget = 0, scratch_cap = 0;
  uint8_t* arena_base = nullptr;
  uint8_t* scratch = nullptr;
  hipStream_t h2d = nullptr, comp = nullptr, d2h = nullptr;
  uint8_t* pinned = nullptr;  // kSlots x (tables | stats)
  size_t slot_bytes = 0, table_cap = 0;
  bool slot_busy[kSlots] = {};
  std::vector<hipEvent_t> event_pool;

  // worker-only state
  iwpp_ctx wctx;  // the worker's view of the context (own error string)
  Arena arena;
  std::deque<uint64_t> admitted;
  std::deque<Batch> inflight;
  bool broken = false;

  // shared state
  std::mutex mu;
  std::condition_variable cv;
  std::deque<SJob> jobs;  // index = ticket
  std::deque<uint64_t> pending;
  std::vector<hipEvent_t> ready_pool;  // submit-side events (under mu)
  bool stop = false;
  std::string error;
  iwpp_server_stats st{};
  std::thread worker;

  hipEvent_t get_event() {
    if (!event_pool.empty()) {
      hipEvent_t e = event_pool.back();
      event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return e;
  }
  void put_event(hipEvent_t e) {
    if (e) event_pool.push_back(e);
  }
  uint8_t* slot_tables(int s) { return pinned + (size_t)s * slot_bytes; }
  // Statistics snapshot after group g of the batch in slot s (cumulative over
  // the batch's groups 0..g).
  unsigned long long* slot_stats(int s, int g) {
    return reinterpret_cast<unsigned long long*>(pinned + (size_t)s * slot_bytes + table_cap +
                                                 (size_t)g * align256(kStatWords * 8));
  }

  void set_error(const std::string& m) {
    std::lock_guard<std::mutex> g(mu);
    if (error.empty()) error = m;
  }

  // Finish, in launch order, the batch parts whose downloads are complete.
  bool complete() {
    bool progress = false;
    while (!inflight.empty()) {
      Batch& b = inflight.front();
      while (b.next < b.parts.size()) {
        Part& p = b.parts[b.next];
        const hipError_t q = b.failed ? hipSuccess : hipEventQuery(p.down);
        if (q == hipErrorNotReady) break;
        const int64_t now = mono_ns();
        bool ok = q == hipSuccess && !b.failed;
        if (q != hipSuccess) {
          (void)hipGetLastError();
          broken = true;
          set_error("serving: device error in a batch");
        } else if (ok) {
          iwpp_stats s;
          iwpp::rt::fold_stats(slot_stats(b.slot, (int)b.next), 3, &s);
          if (s.status != IWPP_OK) {
            ok = false;
            set_error("serving: a batch hit a kernel safety limit");
          }
        }
        {
          std::lock_guard<std::mutex> g(mu);
          for (uint64_t t : p.tickets) {
            SJob& j = jobs[t];
            j.state = ok ? IWPP_JOB_DONE : IWPP_JOB_FAILED;
            j.done_ns = now;
            put_event(j.up);
            j.up = nullptr;
            if (j.ready) ready_pool.push_back(j.ready);
            j.ready = nullptr;
            if (j.bytes) arena.release(j.off, j.bytes);
            if (ok)
              st.completed++;
            else
              st.failed++;
            st.admitted_now--;
          }
        }
        put_event(p.done);
        put_event(p.down);
        p.done = p.down = nullptr;
        b.next++;
        progress = true;
        cv.notify_all();
      }
      if (b.next < b.parts.size()) break;
      slot_busy[b.slot] = false;
      inflight.pop_front();
    }
    return progress;
  }

  // Admit queued jobs in arrival order while memory and slots allow.
  bool admit() {
    bool progress = false;
    for (;;) {
      uint64_t t;
      SJob* j;
      {
        std::lock_guard<std::mutex> g(mu);
        if (pending.empty()) break;
        t = pending.front();
        j = &jobs[t];
        if (broken) {
          pending.pop_front();
          if (j->ready) ready_pool.push_back(j->ready);
          j->ready = nullptr;
          j->state = IWPP_JOB_FAILED;
          j->done_ns = mono_ns();
          st.failed++;
          st.queued_now--;
          cv.notify_all();
          progress = true;
          continue;
        }
        if (st.admitted_now >= opt.max_inflight) break;
      }
      if (opt.resident) {  // device buffers already: nothing to allocate or upload
        std::lock_guard<std::mutex> g(mu);
        pending.pop_front();
        j->off = 0;
        j->bytes = 0;
        j->dev = j->host;
        j->up = nullptr;
        j->state = IWPP_JOB_ADMITTED;
        st.queued_now--;
        st.admitted_now++;
        if ((int64_t)scratch_cap > st.peak_bytes) st.peak_bytes = (int64_t)scratch_cap;
        admitted.push_back(t);
        progress = true;
        continue;
      }
      const size_t bytes = job_buffer_bytes(j->host);
      size_t off = 0;
      if (!arena.alloc(bytes, &off)) break;
      const size_t np = (size_t)j->host.height * (size_t)j->host.width;
      uint8_t* base = arena_base + off;
      iwpp_job d = j->host;
      // The copies wait for the caller's work queued before the submit.
      bool ok = hipStreamWaitEvent(h2d, j->ready, 0) == hipSuccess;
      if (d.op != IWPP_OP_EDT) {
        uint8_t* mask = base;
        uint8_t* marker = base + align256(np);  // overwritten by the result
        d.in1 = mask;
        d.in0 = marker;
        d.out0 = marker;
        ok = ok && hipMemcpyAsync(mask, j->host.in1, np, hipMemcpyHostToDevice, h2d) == hipSuccess &&
             hipMemcpyAsync(marker, j->host.in0, np, hipMemcpyHostToDevice, h2d) == hipSuccess;
      } else {
        d.in0 = base;
        d.out0 = base + align256(np);
        d.out1 = base + align256(np) + align256(4 * np);
        ok = ok && hipMemcpyAsync(base, j->host.in0, np, hipMemcpyHostToDevice, h2d) == hipSuccess;
      }
      hipEvent_t up = ok ? get_event() : nullptr;
      ok = ok && up && hipEventRecord(up, h2d) == hipSuccess;
      if (!ok) {
        (void)hipGetLastError();
        put_event(up);
        arena.release(off, bytes);
        broken = true;
        set_error("serving: upload failed");
        continue;  // the job fails on the next pass through `broken`
      }
      {
        std::lock_guard<std::mutex> g(mu);
        pending.pop_front();
        j->off = off;
        j->bytes = bytes;
        j->dev = d;
        j->up = up;
        j->state = IWPP_JOB_ADMITTED;
        st.queued_now--;
        st.admitted_now++;
        const int64_t used = (int64_t)(arena.used() + scratch_cap);
        if (used > st.peak_bytes) st.peak_bytes = used;
      }
      admitted.push_back(t);
      progress = true;
    }
    return progress;
  }

  // Launch the admitted jobs as one batch when the compute stream has room.
  bool launch() {
    if (admitted.empty() || broken) return false;
    int computing = 0;  // batches whose last group has not finished computing
    size_t computing_jobs = 0;
    for (const Batch& q : inflight)
      if (!q.failed && !q.parts.empty() && q.parts.back().done &&
          hipEventQuery(q.parts.back().done) == hipErrorNotReady) {
        computing++;
        computing_jobs = q.jobs > computing_jobs ? q.jobs : computing_jobs;
      }
    if (computing >= kMaxComputingBatches) return false;
    int slot = -1;
    for (int s = 0; s < kSlots; ++s)
      if (!slot_busy[s]) {
        slot = s;
        break;
      }
    if (slot < 0) return false;
    // The batch takes the admitted jobs, in order, whose uploads have
    // finished: while it computes, later uploads and the previous batch's
    // downloads proceed on the copy streams.
    std::vector<iwpp_job> dj;
    std::vector<uint64_t> tk;
    bool uploading = false;  // a later admitted job's upload has not finished
    {
      std::lock_guard<std::mutex> g(mu);
      for (uint64_t t : admitted) {
        if ((int)dj.size() >= opt.max_batch) break;
        const hipError_t q = jobs[t].up ? hipEventQuery(jobs[t].up) : hipSuccess;
        if (q == hipErrorNotReady) {
          uploading = true;
          break;
        }
        if (q != hipSuccess) {
          (void)hipGetLastError();
          broken = true;
          error = error.empty() ? "serving: upload failed on the device" : error;
          return false;
        }
        dj.push_back(jobs[t].dev);
        tk.push_back(t);
      }
    }
    if (dj.empty()) return false;
    // While a batch computes and uploads are still arriving (a burst), wait
    // until the next batch is at least as large as the computing one: every
    // launch sequence has a fixed cost, and small batches launched one after
    // another would pay it per handful of jobs.  An idle device launches at
    // once, so light load keeps its latency.
    if (computing > 0 && uploading && dj.size() < computing_jobs && (int)dj.size() < opt.max_batch) return false;
    // An idle device takes the oldest job alone, so that it completes as a
    // plain call would; the jobs ready with it form the next batch, queued
    // right behind it.
    if (computing == 0 && dj.size() > 1) {
      dj.resize(1);
      tk.resize(1);
    }
    iwpp::rt::Plan plan;
    size_t n = dj.size();
    for (;;) {  // shrink the batch until its scratch and tables fit
      plan = iwpp::rt::Plan();
      if (iwpp::rt::build_plan(&wctx, dj.data(), (int32_t)n, "serve", plan) != IWPP_OK) {
        broken = true;
        set_error(wctx.err);
        return false;
      }
      if (align256(plan.scratch_bytes) + plan.table_bytes <= scratch_cap && plan.table_bytes <= table_cap) break;
      if (n == 1) {
        broken = true;
        set_error("serving: a job does not fit the scratch area");
        return false;
      }
      n = n / 2;
    }
    tk.resize(n);
    Batch b;
    b.slot = slot;
    b.jobs = n;
    // One part per plan group, holding that group's tickets in plan order
    // (build_plan keeps the jobs' order inside a group).
    for (const iwpp::rt::Group& g : plan.groups) {
      Part p;
      for (size_t i = 0; i < n; ++i)
        if ((dj[i].op == IWPP_OP_EDT ? IWPP_OP_EDT : IWPP_OP_RECON) == g.op && dj[i].conn == g.conn)
          p.tickets.push_back(tk[i]);
      p.done = get_event();
      p.down = get_event();
      b.parts.push_back(std::move(p));
    }
    const size_t sb = align256(plan.scratch_bytes);
    uint8_t* tables = scratch + sb;
    iwpp::rt::pack_tables(plan, slot_tables(slot));
    iwpp::Recorder off;
    bool ok = (int)b.parts.size() <= kMaxGroups;
    for (const Part& p : b.parts) ok = ok && p.done && p.down;
    if (ok && opt.resident) {
      // A resident job's buffers are the caller's: its batch waits for the
      // work the caller queued on its stream before the submit (inputs being
      // written, earlier users of the output memory).
      std::lock_guard<std::mutex> g(mu);
      for (size_t i = 0; i < n && ok; ++i) ok = hipStreamWaitEvent(comp, jobs[tk[i]].ready, 0) == hipSuccess;
    }
    if (ok && plan.table_bytes)
      ok = hipMemcpyAsync(tables, slot_tables(slot), plan.table_bytes, hipMemcpyHostToDevice, comp) == hipSuccess;
    for (size_t gi = 0; gi < plan.groups.size() && ok; ++gi) {
      Part& p = b.parts[gi];
      ok = iwpp::rt::launch_group(&wctx, plan.groups[gi], scratch, wctx.fixed, tables, comp, gi == 0, &off) == IWPP_OK;
      ok = ok &&
           hipMemcpyAsync(slot_stats(slot, (int)gi), wctx.fixed + iwpp::rt::kOffStats, kStatWords * 8,
                          hipMemcpyDeviceToHost, comp) == hipSuccess &&
           hipEventRecord(p.done, comp) == hipSuccess && hipStreamWaitEvent(d2h, p.done, 0) == hipSuccess;
      if (!ok) break;
      std::lock_guard<std::mutex> g(mu);
      for (uint64_t t : p.tickets) {
        SJob& j = jobs[t];
        const size_t np = (size_t)j.host.height * (size_t)j.host.width;
        if (opt.resident) {
          // outputs are the caller's device buffers
        } else if (j.host.op != IWPP_OP_EDT) {
          ok = ok && hipMemcpyAsync(j.host.out0, j.dev.out0, np, hipMemcpyDeviceToHost, d2h) == hipSuccess;
        } else {
          ok = ok && hipMemcpyAsync(j.host.out0, j.dev.out0, 4 * np, hipMemcpyDeviceToHost, d2h) == hipSuccess &&
               hipMemcpyAsync(j.host.out1, j.dev.out1, 4 * np, hipMemcpyDeviceToHost, d2h) == hipSuccess;
        }
        j.state = IWPP_JOB_RUNNING;
      }
      ok = ok && hipEventRecord(p.down, d2h) == hipSuccess;
    }
    if (ok) {
      std::lock_guard<std::mutex> g(mu);
      st.batches++;
      if ((int64_t)n > st.max_batch_jobs) st.max_batch_jobs = (int64_t)n;
    }
    for (size_t i = 0; i < n; ++i) admitted.pop_front();
    slot_busy[slot] = true;
    if (!ok) {
      (void)hipGetLastError();
      broken = true;
      b.failed = true;
      set_error(std::string("serving: batch launch failed: ") + wctx.err);
      // Wait for what was enqueued, then let complete() fail the batch.
      (void)hipStreamSynchronize(comp);
      (void)hipStreamSynchronize(d2h);
      (void)hipGetLastError();
    }
    inflight.push_back(b);
    return true;
  }

  void run() {
    (void)hipSetDevice(ctx->device);
    for (;;) {
      bool progress = complete();
      progress |= admit();
      progress |= launch();
      if (broken) {
        // Fail everything admitted but not launched.
        std::lock_guard<std::mutex> g(mu);
        while (!admitted.empty()) {
          SJob& j = jobs[admitted.front()];
          admitted.pop_front();
          j.state = IWPP_JOB_FAILED;
          j.done_ns = mono_ns();
          put_event(j.up);
          j.up = nullptr;
          if (j.ready) ready_pool.push_back(j.ready);
          j.ready = nullptr;
          if (j.bytes) arena.release(j.off, j.bytes);
          st.failed++;
          st.admitted_now--;
          progress = true;
        }
        cv.notify_all();
      }
      if (!progress) {
        std::unique_lock<std::mutex> g(mu);
        if (stop && pending.empty() && admitted.empty() && inflight.empty()) break;
        // Sleep briefly; a submit wakes the loop at once.
        cv.wait_for(g, std::chrono::microseconds(inflight.empty() ? 500 : 20));
      }
    }
  }
};

namespace {

void free_server(iwpp_server* s) {
  for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : s->ready_pool) (void)hipEventDestroy(e);
  for (SJob& j : s->jobs)
    if (j.ready) (void)hipEventDestroy(j.ready);
  if (s->pinned) (void)hipHostFree(s->pinned);
  if (s->h2d) (void)hipStreamDestroy(s->h2d);
  if (s->comp) (void)hipStreamDestroy(s->comp);
  if (s->d2h) (void)hipStreamDestroy(s->d2h);
  if (s->arena_base) (void)hipFree(s->arena_base);
  if (s->scratch) (void)hipFree(s->scratch);
  (void)hipGetLastError();
  delete s;
}

}  // namespace

extern "C" {

int32_t iwpp_server_start(iwpp_ctx* ctx, const iwpp_server_options* opt, iwpp_server** out) {
  using iwpp::rt::fail;
  if (!ctx) return IWPP_EINVAL;
  if (!out) return fail(ctx, IWPP_EINVAL, "server_start: out is NULL");
  *out = nullptr;
  if (ctx->server) return fail(ctx, IWPP_EBUSY, "server_start: the context already runs a server");
  iwpp_server_options o{};
  if (opt) o = *opt;
  if (o.hbm_budget_bytes < 0 || o.scratch_bytes < 0 || o.max_inflight < 0 || o.max_batch < 0)
    return fail(ctx, IWPP_EINVAL, "server_start: negative option");
  if (o.resident != 0 && o.resident != 1) return fail(ctx, IWPP_EINVAL, "server_start: resident must be 0 or 1");
  if (o.hbm_budget_bytes == 0) o.hbm_budget_bytes = 64ll << 30;
  if (o.max_inflight == 0) o.max_inflight = 4096;
  if (o.max_batch == 0) o.max_batch = 512;
  if (o.scratch_bytes == 0) o.scratch_bytes = o.hbm_budget_bytes / 4;
  if (o.scratch_bytes >= o.hbm_budget_bytes || o.hbm_budget_bytes < (8ll << 20))
    return fail(ctx, IWPP_EINVAL, "server_start: budget below 8 MiB or scratch not below the budget");
  iwpp::rt::DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(ctx, IWPP_EDEVICE, "server_start: cannot select the context's device");
  iwpp_server* s = new (std::nothrow) iwpp_server();
  if (!s) return fail(ctx, IWPP_ENOMEM, "server_start: out of host memory");
  s->ctx = ctx;
  s->opt = o;
  s->wctx.device = ctx->device;
  s->wctx.opt = ctx->opt;
  s->wctx.opt.profile = 0;
  s->wctx.fixed = ctx->fixed;
  s->budget = (size_t)o.hbm_budget_bytes;
  s->scratch_cap = (size_t)o.scratch_bytes & ~size_t(255);
  s->table_cap = align256((size_t)o.max_batch * (sizeof(iwpp::EdtJob) > sizeof(iwpp::MrJob) ? sizeof(iwpp::EdtJob)
                                                                                                 : sizeof(iwpp::MrJob)) +
                          4 * 256);
  s->slot_bytes = s->table_cap + kMaxGroups * align256(kStatWords * 8);
  void* a = nullptr;
  void* sc = nullptr;
  void* pin = nullptr;
  const size_t arena_bytes = o.resident ? 0 : s->budget - s->scratch_cap;
  bool ok = arena_bytes == 0 || hipMalloc(&a, arena_bytes) == hipSuccess;
  if (ok) s->arena_base = static_cast<uint8_t*>(a);
  ok = ok && hipMalloc(&sc, s->scratch_cap) == hipSuccess;
  if (ok) s->scratch = static_cast<uint8_t*>(sc);
  ok = ok && hipHostMalloc(&pin, s->slot_bytes * kSlots, hipHostMallocDefault) == hipSuccess;
  if (ok) s->pinned = static_cast<uint8_t*>(pin);
  if (!ok) {
    free_server(s);
    return fail(ctx, IWPP_ENOMEM, "server_start: cannot allocate the budget on the device");
  }
  ok = hipStreamCreateWithFlags(&s->h2d, hipStreamNonBlocking) == hipSuccess &&
       hipStreamCreateWithFlags(&s->comp, hipStreamNonBlocking) == hipSuccess &&
       hipStreamCreateWithFlags(&s->d2h, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    free_server(s);
    return fail(ctx, IWPP_EDEVICE, "server_start: stream creation failed");
  }
  s->arena.init(arena_bytes);
  try {
    s->worker = std::thread([s] { s->run(); });
  } catch (...) {
    free_server(s);
    return fail(ctx, IWPP_ENOMEM, "server_start: cannot start the worker thread");
  }
  ctx->server = s;
  *out = s;
  return IWPP_OK;
}

int32_t iwpp_server_submit(iwpp_server* s, const iwpp_job* job, int64_t arrival_ns, void* stream, uint64_t* ticket) {
  using iwpp::rt::fail;
  if (!s) return IWPP_EINVAL;
  iwpp_ctx* ctx = s->ctx;
  if (!job || !ticket) return fail(ctx, IWPP_EINVAL, "server_submit: NULL argument");
  const iwpp_job& j = *job;
  if (j.op != IWPP_OP_RECON && j.op != IWPP_OP_RECON_ERODE && j.op != IWPP_OP_EDT)
    return fail(ctx, IWPP_EINVAL, "server_submit: op must be RECON, RECON_ERODE or EDT");
  if (j.conn != 4 && j.conn != 8) return fail(ctx, IWPP_EINVAL, "server_submit: conn must be 4 or 8");
  if (j.height < 1 || j.width < 1) return fail(ctx, IWPP_EINVAL, "server_submit: height and width must be >= 1");
  if (j.op != IWPP_OP_EDT && (!j.in0 || !j.in1 || !j.out0 || j.out1))
    return fail(ctx, IWPP_EINVAL, "server_submit: reconstruction needs in0, in1, out0 and no out1");
  if (j.op == IWPP_OP_EDT && (!j.in0 || j.in1 || !j.out0 || !j.out1))
    return fail(ctx, IWPP_EINVAL, "server_submit: EDT needs in0, out0, out1 and no in1");
  if (j.op == IWPP_OP_EDT && !iwpp::rt::edt_dims_ok(j.height, j.width))
    return fail(ctx, IWPP_EINVAL, "server_submit: EDT sides must be <= 46340 with (h-1)^2 + (w-1)^2 < 2^31");
  if ((uint64_t)j.height * (uint64_t)j.width > 0xFFFFFFFFull)
    return fail(ctx, IWPP_EINVAL, "server_submit: image larger than 2^32 - 1 pixels");
  const size_t need = s->opt.resident ? 0 : job_buffer_bytes(j);
  const size_t sc = iwpp::rt::job_scratch_bytes(j.op, j.height, j.width) + 64 * 256;
  if (need > s->arena.size() || sc > s->scratch_cap)
    return fail(ctx, IWPP_EINVAL, "server_submit: the job can never fit the server's memory budget");
  if (s->opt.resident) {
    const void* bufs[4] = {j.in0, j.in1, j.out0, j.out1};
    for (const void* b : bufs) {
      if (!b) continue;
      hipPointerAttribute_t at{};
      const bool dev_ok = hipPointerGetAttributes(&at, b) == hipSuccess && at.type == hipMemoryTypeDevice &&
                          at.device == ctx->device;
      (void)hipGetLastError();
      if (!dev_ok) return fail(ctx, IWPP_EINVAL, "server_submit: a resident server takes device buffers of its device");
    }
  }
  iwpp::rt::DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(ctx, IWPP_EDEVICE, "server_submit: cannot select the context's device");
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return fail(ctx, IWPP_EBUSY, "server_submit: the server is stopping");
    hipEvent_t ready = nullptr;
    if (!s->ready_pool.empty()) {
      ready = s->ready_pool.back();
      s->ready_pool.pop_back();
    } else if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, IWPP_EDEVICE, "server_submit: event creation failed");
    }
    if (hipEventRecord(ready, static_cast<hipStream_t>(stream)) != hipSuccess) {
      (void)hipGetLastError();
      s->ready_pool.push_back(ready);
      return fail(ctx, IWPP_EDEVICE, "server_submit: cannot record on the caller's stream");
    }
    SJob sj;
    sj.ready = ready;
    sj.host = j;
    sj.arrival_ns = arrival_ns > 0 ? arrival_ns : mono_ns();
    *ticket = (uint64_t)s->jobs.size();
    s->jobs.push_back(sj);
    s->pending.push_back(*ticket);
    s->st.submitted++;
    s->st.queued_now++;
  }
  s->cv.notify_all();
  return IWPP_OK;
}

int32_t iwpp_server_poll(iwpp_server* s, uint64_t ticket, int32_t* state, double* latency_ms) {
  using iwpp::rt::fail;
  if (!s) return IWPP_EINVAL;
  if (!state) return fail(s->ctx, IWPP_EINVAL, "server_poll: state is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  if (ticket >= s->jobs.size()) return fail(s->ctx, IWPP_EINVAL, "server_poll: unknown ticket");
  const SJob& j = s->jobs[ticket];
  *state = j.state;
  if (latency_ms)
    *latency_ms = (j.state == IWPP_JOB_DONE || j.state == IWPP_JOB_FAILED) ? (j.done_ns - j.arrival_ns) * 1e-6 : -1.0;
  if (j.state == IWPP_JOB_FAILED) s->ctx->err = s->error;
  return IWPP_OK;
}

int32_t iwpp_server_drain(iwpp_server* s, int64_t timeout_ms) {
  using iwpp::rt::fail;
  if (!s) return IWPP_EINVAL;
  std::unique_lock<std::mutex> g(s->mu);
  auto done = [s] { return s->st.completed + s->st.failed == s->st.submitted; };
  if (timeout_ms < 0) {
    s->cv.wait(g, done);
  } else if (!s->cv.wait_for(g, std::chrono::milliseconds(timeout_ms), done)) {
    s->ctx->err = "server_drain: timed out";
    return IWPP_EBUSY;
  }
  if (s->st.failed) {
    s->ctx->err = s->error;
    return IWPP_EDEVICE;
  }
  return IWPP_OK;
}

int32_t iwpp_server_get_stats(iwpp_server* s, iwpp_server_stats* out) {
  if (!s) return IWPP_EINVAL;
  if (!out) return iwpp::rt::fail(s->ctx, IWPP_EINVAL, "server_get_stats: out is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  *out = s->st;
  return IWPP_OK;
}

int32_t iwpp_server_stop(iwpp_server* s) {
  if (!s) return IWPP_EINVAL;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  iwpp_ctx* ctx = s->ctx;
  const bool failed = s->st.failed != 0;
  std::string err = s->error;
  {
    iwpp::rt::DeviceGuard dg(ctx->device);
    (void)hipStreamSynchronize(s->comp);
    (void)hipStreamSynchronize(s->d2h);
    free_server(s);
  }
  ctx->server = nullptr;
  if (failed) {
    ctx->err = err;
    return IWPP_EDEVICE;
  }
  return IWPP_OK;
}

}  // extern "C"
