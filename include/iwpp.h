/*
 * iwpp.h -- C ABI of the MI355X (gfx950) irregular wavefront propagation library.
 *
 * Two instances of the irregular wavefront propagation pattern (IWPP) of
 * Teodoro et al., "Efficient Irregular Wavefront Propagation Algorithms on
 * Hybrid CPU-GPU Machines" (arXiv 1209.3314):
 *
 *   - grayscale morphological reconstruction by dilation, rho_I(J)
 *     (Sec. 2.1 and Algorithms 2 and 5), 4- or 8-connected, and its dual,
 *     reconstruction by erosion (one of the pattern's other users, Sec. 1);
 *   - the propagation-based Euclidean distance transform that carries the
 *     nearest feature of every pixel (Sec. 2.2 and Algorithms 3 and 6).
 *
 * Every symbol is extern "C"; no C++ type or exception crosses this boundary
 * and the library never aborts the process.
 *
 * Memory.  Image arguments are DEVICE pointers on the context's device, owned
 * by the caller, row-major with row stride == width (contiguous).  The context
 * owns its scratch memory (queues, keys, counters), which it grows on demand
 * and frees in iwpp_destroy.
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the default
 * stream).  Compute calls only enqueue work on it and return; results are
 * valid once the stream has been synchronised.  A context serves one call at a
 * time: calls on one context must not overlap (their scratch is shared), so
 * either use one stream per context or order the calls.
 *
 * Errors.  Argument errors return IWPP_EINVAL before anything is enqueued; a
 * HIP error from a launch returns IWPP_EDEVICE.  A device-side failure (a
 * safety limit hit inside a kernel) is reported by iwpp_get_stats through the
 * `status` field.  iwpp_last_error gives a message for the last non-OK status.
 */
#ifndef IWPP_H
#define IWPP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct iwpp_ctx iwpp_ctx;
typedef struct iwpp_graph iwpp_graph;
typedef struct iwpp_server iwpp_server;

typedef enum {
  IWPP_OK = 0,
  IWPP_EINVAL = -1,  /* bad argument: nothing was enqueued */
  IWPP_ENOMEM = -2,  /* scratch allocation failed */
  IWPP_EDEVICE = -3, /* HIP launch/runtime error, or a device-side failure */
  IWPP_EBUSY = -4    /* the operation needs an idle context */
} iwpp_status;

/* Tunables.  Zero means "library default" for every field.  None of them can
 * change a result: reconstruction is unique (Sec. 2.1) and the distance
 * transform follows fixed round semantics, so every setting yields the same
 * bytes; they only change speed (and, for the capacity, force the overflow
 * path of Sec. 3.2 so it can be tested). */
typedef struct {
  /* Capacity, in tiles, of each round's work list of the reconstruction
   * propagation.  When a round needs more, the excess is dropped, a flag is
   * raised and the work list is rebuilt from the current image by a dense
   * seed detection, as the paper re-runs propagation from its partial output
   * after its global queue overflows (Sec. 3.2, Sec. 5.2.4).  0 = no limit. */
  int64_t mr_list_capacity;
  /* Cap on sweep iterations per tile visit before the tile is re-queued
   * (0 = 2). */
  int32_t mr_max_sweeps;
  /* Workgroups of the persistent kernels (0 = fill the device). */
  int32_t persistent_blocks;
  /* Nonzero: record a HIP event pair around every kernel launch so that
   * iwpp_profile_read can report per-kernel device times.  Costs two event
   * records per launch. */
  int32_t profile;
  /* Cap on sweep iterations per tile in the reconstruction seed pass (the
   * number of raster/anti-raster scan pairs before the queue takes over; the
   * paper varies the number of initial scans in Table 1; 0 = 1 with
   * 8-connectivity, 2 with 4-connectivity). */
  int32_t mr_seed_sweeps;
  /* Waves per workgroup of the persistent kernels, 4 or 8 (0 = 4): the
   * workgroup size (the paper's threads per block; a wave holds one tile). */
  int32_t wg_waves;
  /* Work-list items a wave stages in LDS before one global atomic appends
   * them (the depth of the paper's per-block queue): 1 .. 64 (0 = 64). */
  int32_t stage_depth;
  /* Reconstruction seed pass: tiles of 64 x 64 per vertical strip that a
   * wave sweeps top to bottom, each tile reading the one above it fresh (the
   * seed pass's tiling; 0 = automatic). */
  int32_t mr_seed_strip;
  int32_t reserved[3];
} iwpp_options;

/* Counters of the last compute call on a context (see iwpp_get_stats). */
typedef struct {
  int32_t status;            /* IWPP_OK, or IWPP_EDEVICE if a kernel hit a safety limit */
  int32_t op;                /* 1 = reconstruction, 2 = distance transform, 3 = batch */
  int64_t seeds;             /* MR: tiles the seed pass left to propagation (visited in round 1);
                                EDT: contour features (initial frontier) */
  int64_t items;             /* MR: tile visits in propagation; EDT: frontier items over all rounds */
  int64_t sweeps;            /* MR: sweep iterations over all tile visits */
  int64_t rounds;            /* MR: propagation rounds; EDT: rounds that changed a pixel */
  int64_t updates;           /* EDT: successful key improvements */
  int64_t overflow_restarts; /* MR: dense re-seeds after a work-list overflow */
  int64_t reserved[6];
} iwpp_stats;

/* One timed kernel launch (see iwpp_options.profile). */
typedef struct {
  int32_t kernel; /* IWPP_K_* */
  float ms;       /* device time between the events around the launch */
} iwpp_kernel_time;

enum {
  IWPP_K_RESET = 0,        /* counter reset at the start of every call */
  IWPP_K_MR_SEED = 1,      /* reserved (the seed pass is round 0 of IWPP_K_MR_PROPAGATE) */
  IWPP_K_MR_DETECT = 2,    /* reserved (no separate seed detection) */
  IWPP_K_MR_PROPAGATE = 3, /* reconstruction: persistent kernel, seed pass + propagation */
  IWPP_K_EDT_INIT = 4,     /* distance transform initialisation */
  IWPP_K_EDT_ROUNDS = 5,   /* distance transform rounds + finalisation */
  IWPP_K_MRQ_INIT = 6,     /* pixel-queue reconstruction: working copy + initial queue */
  IWPP_K_MRQ_PROPAGATE = 7, /* pixel-queue reconstruction: queue rounds */
  IWPP_K_XEDT = 8            /* exact EDT: column and row passes together */
};

/* Library version, (major << 16) | minor. */
int32_t iwpp_version(void);

/* Create a context on HIP device `device`.  `opt` may be NULL.  On success
 * *out receives the context.  Errors: IWPP_EINVAL (bad device, NULL out),
 * IWPP_EDEVICE. */
int32_t iwpp_create(int32_t device, const iwpp_options* opt, iwpp_ctx** out);

/* Free a context and its scratch memory.  NULL is allowed.  Waits for the
 * context's work to finish first. */
void iwpp_destroy(iwpp_ctx* ctx);

/* Message for the last non-OK status on `ctx` (or for iwpp_create when ctx is
 * NULL).  The pointer stays valid until the next call on the context. */
const char* iwpp_last_error(const iwpp_ctx* ctx);

/* Grayscale morphological reconstruction by dilation of mask I from marker J,
 * rho_I(J): the limit of J(p) <- max{J(q) : q in N_G(p) U {p}} ^ I(p) applied
 * until nothing changes (Sec. 2.1).  The steps of Algorithm 5, re-planned for
 * the GPU: a seed pass of raster and anti-raster scans swept to local
 * stability inside 64x64 tiles held in LDS (one wave per tile), seed
 * detection reduced to tests of the tile borders that rose, and propagation
 * in rounds over a work list of tiles (the frontier, kept at tile
 * granularity; a tile is listed when a border change can raise it) until the
 * list is empty.  No pixel is updated atomically: a tile has one owner per
 * round.  A bounded list (options.mr_list_capacity) drops, flags and rebuilds
 * its frontier from the current image, as the paper's fixed-size global queue
 * does on overflow (Sec. 3.2).
 *
 *   marker, mask : const uint8_t[height*width] (device)
 *   out          : uint8_t[height*width] (device); may alias marker (in place),
 *                  must not alias mask
 *   height,width : >= 1; width <= 2^25 and at most 2^24 - 1 tiles of 64x64
 *                  (about 68 G pixels): whole slides beyond 2^32 pixels are
 *                  one call (the tile rounds carry the propagation across
 *                  tiles, the border propagation of Sec. 4)
 *   conn         : 4 or 8
 * A marker above the mask is clamped first (the result is rho_I(min(J, I))).
 * Pixels outside the image are not neighbours.  The result is unique, so it is
 * bit-exact whatever the schedule.
 * Errors: IWPP_EINVAL (NULL pointer, dims < 1, conn not 4/8, out aliasing
 * mask), IWPP_ENOMEM, IWPP_EDEVICE. */
int32_t iwpp_morph_recon_u8(iwpp_ctx* ctx, const uint8_t* marker, const uint8_t* mask, uint8_t* out,
                            int32_t height, int32_t width, int32_t conn, void* stream);

/* Bytes of the static device work area of iwpp_morph_recon_u8_noalloc (one
 * per device, held until the process ends). */
#define IWPP_NOALLOC_SCRATCH_BYTES (32u << 20)

/* iwpp_morph_recon_u8 for callers that cannot allocate device memory during a
 * call: code under HIP stream/graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, rules and result bytes as
 * iwpp_morph_recon_u8, but the work lists, flags, counters and grid barrier
 * live in a static device array of IWPP_NOALLOC_SCRATCH_BYTES instead of the
 * context's growable scratch; the call performs no hipMalloc, hipFree or
 * event creation (the context's profile recording does not apply to it).
 * The array's device address is looked up once per device by iwpp_create.
 *
 * Limit: the image's tile scratch (about 336 bytes per 64x64 tile) must fit
 * the area, i.e. at most about 99,800 tiles -- e.g. 16384 x 24576
 * (98,304 tiles) fits, 20480 x 20480 (102,400 tiles) does not; a larger image
 * returns IWPP_EINVAL with the sizes in iwpp_last_error.
 *
 * Sharing: every call on a device uses that device's one array, which keeps
 * the last call's contents (counters are cleared at the start of each call).
 * Calls that overlap on one device -- from any context, on any stream -- race
 * and give wrong results: order them (one stream, or events).  iwpp_get_stats
 * and iwpp_round_times on the context read the last such call's counters
 * until another call on the device replaces them.
 * Errors: as iwpp_morph_recon_u8, plus IWPP_EINVAL for an image above the
 * limit and IWPP_EDEVICE if the area could not be set up. */
int32_t iwpp_morph_recon_u8_noalloc(iwpp_ctx* ctx, const uint8_t* marker, const uint8_t* mask, uint8_t* out,
                                    int32_t height, int32_t width, int32_t conn, void* stream);

/* Grayscale morphological reconstruction by erosion of mask I from marker J,
 * rho*_I(J): the limit of J(p) <- max(min{J(q) : q in N_G(p) U {p}}, I(p))
 * applied until nothing changes -- the dual of reconstruction by dilation and
 * another instance of the pattern (Sec. 1).  Computed by the reconstruction
 * kernels on complemented bytes (rho*_I(J) = 255 - rho_{255-I}(255-J)): each
 * image byte is complemented as it is loaded and as the result is stored, so
 * the arguments, layout, limits and errors are those of iwpp_morph_recon_u8.
 * A marker below the mask is raised to it first (the result is
 * rho*_I(max(J, I))).  In batches its op is IWPP_OP_RECON_ERODE; it shares
 * the launches of the 4- or 8-connected dilation group. */
int32_t iwpp_morph_recon_erode_u8(iwpp_ctx* ctx, const uint8_t* marker, const uint8_t* mask, uint8_t* out,
                                  int32_t height, int32_t width, int32_t conn, void* stream);

/* How the pixel-queue reconstruction appends to a round's queue. */
enum {
  IWPP_QUEUE_NAIVE = 0,  /* one global atomic per appended item */
  IWPP_QUEUE_BALLOT = 1, /* one global atomic per wave and append step (ballot + mbcnt offsets) */
  IWPP_QUEUE_STAGED = 2  /* items staged per wave in LDS, one global atomic per flush */
};

typedef struct {
  int32_t append_mode; /* IWPP_QUEUE_* */
  int32_t seed_sweeps; /* sweep iterations per tile of the seed pass (0 = as iwpp_morph_recon_u8) */
  int64_t capacity;    /* items per round queue; appends past it are dropped and recovered (0 = 2*h*w + 64) */
  int32_t reserved[4];
} iwpp_queue_options;

/* Reconstruction by dilation with the paper's pixel queue (Algorithm 5's
 * propagation, Sec. 3.2), kept to compare with the tile design of
 * iwpp_morph_recon_u8 (same result, bit for bit; it is slower).  After the
 * same tile seed pass (`seed_sweeps` iterations: the analogue of the number
 * of initial scans of Table 1), every pixel with a neighbour it can raise is
 * queued; rounds then pop one item per lane, raise each neighbour q with
 * J(q) < J(p) and J(q) < I(q) by an atomic maximum on a 32-bit working copy,
 * and queue q when that atomic raised it.  `append_mode` selects how items
 * enter a round's queue.  A queue that reaches `capacity` drops, flags, and
 * once the queues drain is rebuilt from the current image by dense seed
 * detection (the restart of Sec. 3.2 / Sec. 5.2.4; counted in
 * iwpp_stats.overflow_restarts).  iwpp_get_stats: seeds = initial queue,
 * items = pops, updates = successful atomic raises, rounds = queue rounds.
 * Scratch: 4 bytes per pixel plus 8 bytes per capacity item.
 *   arguments as iwpp_morph_recon_u8; at most 2^31 - 1 pixels; qopt may be
 *   NULL (staged appends, default capacity).
 * Errors: as iwpp_morph_recon_u8, plus IWPP_EINVAL for bad queue options. */
int32_t iwpp_morph_recon_queue_u8(iwpp_ctx* ctx, const uint8_t* marker, const uint8_t* mask, uint8_t* out,
                                  int32_t height, int32_t width, int32_t conn, const iwpp_queue_options* qopt,
                                  void* stream);

/* Euclidean distance transform by propagation of the nearest feature
 * (Sec. 2.2, Algorithms 3 and 6).  Features (the paper's background, the
 * targets of the distance) are the 0-pixels of `binary`; every pixel receives
 * the squared distance to the feature it ends up carrying and that feature's
 * index y*width + x.
 *
 * Semantics: level-synchronous rounds.  Round r offers, from every pixel that
 * changed in round r-1 (initially the contour features), the feature that
 * pixel held at the end of round r-1 to each in-image neighbour in N_G; a
 * neighbour keeps the smallest (squared distance, feature index) pair.  Rounds
 * stop when nothing changes.  These semantics make the parallel result unique
 * (the paper's equidistant-choice argument does not hold for the propagation
 * approximation), so the output is reproducible bit for bit.
 *
 *   binary        : const uint8_t[height*width] (device), 0 = feature
 *   sqdist        : int32_t[height*width] (device), squared distance
 *   nearest       : int32_t[height*width] (device), y*width + x of the feature
 *   height,width  : 1 .. 46340 with (height-1)^2 + (width-1)^2 < 2^31, so
 *                   every squared distance fits the int32 output; images with
 *                   a side above 32767 use wider coordinate fields (slower)
 *   conn          : 4 or 8
 * If the image has no feature, sqdist and nearest are -1 everywhere.
 * Errors: IWPP_EINVAL (NULL pointer, dims out of range, conn not 4/8, outputs
 * aliasing each other or the input), IWPP_ENOMEM, IWPP_EDEVICE. */
int32_t iwpp_edt(iwpp_ctx* ctx, const uint8_t* binary, int32_t* sqdist, int32_t* nearest, int32_t height,
                 int32_t width, int32_t conn, void* stream);

/* The exact Euclidean distance transform.  The propagation of iwpp_edt is an
 * approximation (Sec. 2.2: the 8-neighbour propagation misses some nearest
 * features; exact distances need further processing).  This call computes the
 * exact transform by the separable method of Meijster, Roerdink and
 * Hesselink (2000): per column the nearest feature in the column, then per
 * row the lower envelope of the parabolas (x - x')^2 + dy(x')^2, in integer
 * arithmetic.  sqdist is the exact squared distance to the nearest feature;
 * nearest is y*width + x of a feature at exactly that distance (of several,
 * the one in the smallest column, then the smallest row).  No counters
 * (iwpp_get_stats reports zeros).  Scratch: about 16 bytes per pixel.
 *   binary, sqdist, nearest, height, width : as iwpp_edt (no connectivity)
 * If the image has no feature, sqdist and nearest are -1 everywhere.
 * Errors: as iwpp_edt. */
int32_t iwpp_edt_exact(iwpp_ctx* ctx, const uint8_t* binary, int32_t* sqdist, int32_t* nearest, int32_t height,
                       int32_t width, void* stream);

/* One image of a batch (see iwpp_run_batch). */
typedef struct {
  int32_t op;          /* IWPP_OP_RECON, IWPP_OP_RECON_ERODE or IWPP_OP_EDT */
  int32_t conn;        /* 4 or 8 */
  int32_t height;
  int32_t width;
  const uint8_t* in0;  /* recon (either): marker; EDT: binary (0 = feature) */
  const uint8_t* in1;  /* recon (either): mask; EDT: NULL */
  void* out0;          /* recon (either): uint8 result (may equal in0); EDT: int32 sqdist */
  void* out1;          /* recon: NULL; EDT: int32 nearest */
} iwpp_job;

enum { IWPP_OP_RECON = 1, IWPP_OP_EDT = 2, IWPP_OP_RECON_ERODE = 3 };

/* Process many images of mixed sizes and both operations with few launches:
 * jobs are grouped by (op, conn) and every group runs as one seed pass and
 * one persistent propagation launch over all of its images (reconstruction)
 * or one initialisation and one persistent round launch (EDT), so small
 * images share the device instead of each leaving it mostly idle.  Every
 * result is identical to the corresponding single-image call (each image's
 * reconstruction is unique; EDT images advance in the same rounds, each by its
 * own round semantics).
 *   jobs : host array of n descriptors (copied before the call returns)
 *   n    : >= 1
 * Each job obeys the rules of iwpp_morph_recon_u8 / iwpp_edt; in addition no
 * output may overlap another job's input or output.  Counters from
 * iwpp_get_stats cover the whole batch.
 * Errors: IWPP_EINVAL (bad job: the message names its index), IWPP_ENOMEM,
 * IWPP_EDEVICE. */
int32_t iwpp_run_batch(iwpp_ctx* ctx, const iwpp_job* jobs, int32_t n, void* stream);

/* Replace the context's options for later calls (for per-call tuning).
 * Errors: IWPP_EINVAL for NULL or negative fields. */
int32_t iwpp_set_options(iwpp_ctx* ctx, const iwpp_options* opt);

/* Capture a batch (same rules as iwpp_run_batch) into a HIP graph that can be
 * replayed with one launch: the job tables are uploaded once, every kernel of
 * every group is recorded, and the graph owns its scratch memory and counters,
 * so replays do not depend on the context's later calls.  The graph reads and
 * writes the buffers named in `jobs` on every launch.  Inside the graph the
 * persistent kernels are plain launches of a device-filling grid: launch the
 * graph when the device is not busy with other work (if the grid cannot all be
 * resident, the kernels stop with status IWPP_EDEVICE rather than waiting).
 * Errors: as iwpp_run_batch; IWPP_EDEVICE if capture is not possible. */
int32_t iwpp_batch_graph_create(iwpp_ctx* ctx, const iwpp_job* jobs, int32_t n, iwpp_graph** out);

/* Enqueue one replay of the graph on `stream` (hipStream_t as void*). */
int32_t iwpp_batch_graph_launch(iwpp_graph* graph, void* stream);

/* Counters of the graph's last replay (synchronises with its stream). */
int32_t iwpp_batch_graph_stats(iwpp_graph* graph, iwpp_stats* out);

/* Free the graph and its memory (waits for the device).  NULL is allowed. */
void iwpp_batch_graph_destroy(iwpp_graph* graph);

/* ---- serving ------------------------------------------------------------
 * A request loop on one context, after the paper's demand-driven runtime that
 * hands independent tiles to whichever device is free in arrival order
 * (Sec. 4).  Jobs come with HOST buffers; a worker thread admits them in
 * arrival order while the device-memory budget and the in-flight slot limit
 * allow, uploads them on a copy stream, runs every admitted job that is not
 * yet running as one batch (continuous batching: jobs that arrive while a
 * batch runs form the next one), downloads the outputs on a second copy
 * stream and timestamps completion.  Results are the same bytes as the single
 * image calls.  While a server runs, the other calls on its context return
 * IWPP_EBUSY. */
typedef struct {
  /* Device memory the server holds: admitted jobs' buffers plus one scratch
   * area shared by the batches (0 = 64 GiB). */
  int64_t hbm_budget_bytes;
  /* Part of the budget kept as the batches' scratch area; it bounds the
   * pixels of one batch (0 = a quarter of the budget). */
  int64_t scratch_bytes;
  int32_t max_inflight; /* admitted jobs not yet complete (0 = 4096) */
  int32_t max_batch;    /* jobs per launch; 1 = one job per launch (0 = 512) */
  /* Nonzero: device-resident jobs.  Jobs then come with DEVICE buffers on the
   * context's device (images already resident: no copies), the server
   * allocates only the scratch area, admission is bounded by the in-flight
   * limit, and a job is complete when its batch's computation is.  The
   * outputs of jobs in flight together must not overlap any buffer of another
   * of them (a batch containing such jobs fails). */
  int32_t resident;
  int32_t reserved[5];
} iwpp_server_options;

typedef struct {
  int64_t submitted, completed, failed;
  int64_t batches;        /* launches (batches) so far */
  int64_t max_batch_jobs; /* largest batch */
  int64_t peak_bytes;     /* high-water mark of device memory in use */
  int64_t admitted_now;   /* admitted, not complete */
  int64_t queued_now;     /* submitted, not admitted */
  int64_t reserved[4];
} iwpp_server_stats;

enum { IWPP_JOB_QUEUED = 0, IWPP_JOB_ADMITTED = 1, IWPP_JOB_RUNNING = 2, IWPP_JOB_DONE = 3, IWPP_JOB_FAILED = 4 };

/* Allocate the budget on the context's device and start the worker thread.
 * Errors: IWPP_EINVAL (bad options), IWPP_EBUSY (already serving),
 * IWPP_ENOMEM (the budget cannot be allocated). */
int32_t iwpp_server_start(iwpp_ctx* ctx, const iwpp_server_options* opt, iwpp_server** out);

/* Queue one job.  `job` has the layout of iwpp_run_batch's jobs but HOST
 * pointers (page-locked memory lets the copies overlap the computation), or
 * device pointers on a resident server (each buffer is checked to be device
 * memory of the context's device); the caller must not change the inputs or
 * read the outputs before the job is done.  `arrival_ns` is the request's
 * arrival time on CLOCK_MONOTONIC (0 = now); latency is measured from it.
 * `stream` (hipStream_t as void*, NULL = the default stream) is the caller's
 * stream: an event is recorded on it at submit, and the job's work (its
 * uploads; on a resident server its batch) waits for that event, so inputs
 * that the caller's queued kernels are still writing, and output memory that
 * its queued kernels still use, are safe to submit without synchronising.
 * Errors: IWPP_EINVAL (bad job, one that can never fit the budget, or a
 * buffer of the wrong kind), IWPP_EBUSY (stopping), IWPP_EDEVICE (the event
 * cannot be recorded on `stream`). */
int32_t iwpp_server_submit(iwpp_server* server, const iwpp_job* job, int64_t arrival_ns, void* stream,
                           uint64_t* ticket);

/* State of a ticket (IWPP_JOB_*) and, once done or failed, its latency:
 * completion of the output download (resident: of the batch) minus arrival,
 * in ms (else -1). */
int32_t iwpp_server_poll(iwpp_server* server, uint64_t ticket, int32_t* state, double* latency_ms);

/* Wait until every submitted job is done or failed (timeout_ms < 0: no
 * limit).  IWPP_EBUSY on timeout, IWPP_EDEVICE if a job failed. */
int32_t iwpp_server_drain(iwpp_server* server, int64_t timeout_ms);

int32_t iwpp_server_get_stats(iwpp_server* server, iwpp_server_stats* out);

/* Finish every submitted job, stop the worker and free the budget; the
 * context is usable again.  IWPP_EDEVICE if any job failed. */
int32_t iwpp_server_stop(iwpp_server* server);

/* Timeline of the last persistent kernel of the last call on the context:
 * us[i] = device time of phase i in microseconds, where phase 0 runs from the
 * kernel's start to its first grid barrier and phase i from barrier i to
 * barrier i+1 (reconstruction: phase 0 is the seed pass and phase r round r;
 * distance transform: phase i is step i+1).  Stamps are taken by one
 * workgroup on the device's constant-rate clock.  Synchronises with the last
 * call's stream.  *n = phases written (at most max). */
int32_t iwpp_round_times(iwpp_ctx* ctx, double* us, int32_t max, int32_t* n);

/* iwpp_round_times plus the work of each phase: tiles[i] = tiles visited
 * in phase i (reconstruction: every tile in the seed pass and in a full
 * round after a work-list overflow, else the round's work list; distance
 * transform: the step's work list).  At most 254 phases are recorded.
 * Errors: IWPP_EINVAL (NULL arguments), IWPP_EDEVICE. */
int32_t iwpp_round_work(iwpp_ctx* ctx, double* us, int64_t* tiles, int32_t max, int32_t* n);

/* The same timeline for the last replay of a batch graph: the last
 * persistent kernel of the graph (its last group).  Synchronises with the
 * stream of that replay.  *n = 0 before the first replay.
 * Errors: IWPP_EINVAL (NULL arguments), IWPP_EDEVICE. */
int32_t iwpp_batch_graph_round_times(iwpp_graph* graph, double* us, int32_t max, int32_t* n);

/* Per-kernel device times recorded since the previous read (needs
 * iwpp_options.profile).  Synchronises with every stream the recorded
 * launches used, writes up to `max` entries in launch order to out[], sets
 * *n to the number written and clears the record.  Launches beyond the
 * record's capacity (4096) are not recorded.
 * Errors: IWPP_EINVAL (NULL arguments), IWPP_EDEVICE. */
int32_t iwpp_profile_read(iwpp_ctx* ctx, iwpp_kernel_time* out, int32_t max, int32_t* n);

/* Copy the counters of the last compute call into *out.  Synchronises with
 * the stream of that call first.  Errors: IWPP_EINVAL (NULL), IWPP_EDEVICE. */
int32_t iwpp_get_stats(iwpp_ctx* ctx, iwpp_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* IWPP_H */
