/*
 * pxcl.h -- per-event pixel clustering on MI355X behind a non-blocking
 * acquire / produce boundary.
 *
 * The boundary follows the offload pattern of "Bringing heterogeneity to the CMS
 * software framework" (arXiv:2004.04334):
 *
 *  - Sec. 2 (External Worker): a module's work is split into acquire(), which only
 *    reads its inputs and launches the offloaded work, and produce(), which runs
 *    after completion.  The continuation is released by a reference-counted holder
 *    that non-framework threads may signal and that can carry an error.
 *    -> pxcl_acquire() enqueues all device work and returns without blocking;
 *       pxcl_done_cb fires exactly once, from the context's completion thread,
 *       with a status;
 *       pxcl_produce() hands back the results without blocking.
 *  - Sec. 4.1 (asynchronous execution): during event processing only asynchronous
 *    copies, memsets and kernel launches are issued, on the caller's stream; no
 *    allocation and no synchronisation happens on the event path; completion is
 *    signalled by a callback queued into the stream after the work.
 *    -> here an event is recorded into the stream after the work instead, and one
 *       thread per context polls the events of the launches in flight and runs the
 *       callbacks: queuing a host function costs the caller ~30 us per launch on
 *       this platform and fires ~45-75 us after the work ends; polling an event
 *       costs ~0.1 us and sees the end ~10 us after it.
 *    -> the library never allocates device or pinned memory: the caller allocates
 *       workspaces once (e.g. from PyTorch's caching allocator, the counterpart of
 *       the memory pool of Sec. 4.1) and binds them; device-side errors are
 *       accumulated in a device error word instead of device asserts.
 *  - Sec. 4.2 (Product<T>): a data product carries the device, the stream its work
 *    was queued on and an event marking completion.
 *    -> pxcl_clusters carries device pointers, the stream and a hipEvent_t.
 *
 * The clustering itself is the work the paper's Figure 1 (Sec. 3) names as the
 * "ClusterProducer" that turns raw detector data into clusters (the GPU variant
 * goes from raw data straight on): per detector module (160 rows x 416 columns),
 * the 8-connected components of the fired pixels ("digis"); per component its id
 * = the smallest linear pixel index  module*66560 + col*160 + row, its charge = the
 * sum of the digis' ADC counts (uint32 arithmetic, reported as int32) and its size;
 * components with charge >= charge_cut are kept.  Every step is integer arithmetic
 * and the result is unique, so results are bit-exact.
 *
 * Threading: a context serves any number of threads.  An event (or batch) object
 * has one owner at a time and at most one piece of work in flight.
 * All functions return PXCL_OK (0) or a negative PXCL_E_* code unless stated.
 */
#ifndef PXCL_H
#define PXCL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- geometry and limits ------------------------------------------------ */
#define PXCL_ROWS 160u
#define PXCL_COLS 416u
#define PXCL_PIXELS_PER_MODULE 66560u        /* ROWS * COLS */
#define PXCL_MAX_MODULES 32263u              /* so every cluster id fits in int32 */
#define PXCL_MAX_BATCH 128u                  /* events per pxcl_acquire_batch */
#define PXCL_MAX_EVENT_DIGIS (1u << 28)      /* capacity limit of one event slot */

/* ---- status codes --------------------------------------------------------- */
#define PXCL_OK 0
#define PXCL_E_INVAL (-1)       /* bad argument (null pointer, zero size, bad config) */
#define PXCL_E_CAPACITY (-2)    /* n digis > the event slot's capacity, k > batch capacity */
#define PXCL_E_BUSY (-3)        /* the event/batch has work in flight; ctx has bound objects */
#define PXCL_E_NOT_READY (-4)   /* produce() before completion */
#define PXCL_E_DUP_PIXEL (-5)   /* async: the same pixel fired twice in one module */
#define PXCL_E_RANGE (-6)       /* async: module >= n_modules, row >= 160 or col >= 416 */
#define PXCL_E_ORDER (-7)       /* async: module ids decrease along the input */
#define PXCL_E_HIP (-8)         /* a HIP runtime call failed */
#define PXCL_E_INTERNAL (-10)   /* library bug: inconsistent device state (a list overflowed, a
                                   module entry out of range) or a missing status write-back */
#define PXCL_E_NOTFOUND (-11)   /* autotune cache file missing or without this key */
#define PXCL_E_HINT (-12)       /* async: a module has more digis than pxcl_digis.max_module_digis */

/* Asynchronous error bits (pxcl_clusters.err_bits).  When several are set the
 * status reports, in this order: RANGE, ORDER, HINT, DUP.  With RANGE or ORDER set
 * the DUP bit is not reliable (grouping by module is then undefined); with HINT set
 * the modules above the hint were not clustered. */
#define PXCL_ERRBIT_RANGE 1u
#define PXCL_ERRBIT_ORDER 2u
#define PXCL_ERRBIT_DUP 4u
#define PXCL_ERRBIT_INTERNAL 8u
#define PXCL_ERRBIT_HINT 16u

/* ---- types -------------------------------------------------------------------- */
typedef struct pxcl_ctx pxcl_ctx;
typedef struct pxcl_event pxcl_event;
typedef struct pxcl_batch pxcl_batch;

typedef struct {
    uint32_t n_modules;   /* 1 .. PXCL_MAX_MODULES */
    uint32_t charge_cut;  /* keep a cluster iff its charge >= charge_cut (unsigned compare) */
} pxcl_config;

#define PXCL_WHERE_HOST 0     /* pinned host memory (hipHostMalloc / torch pin_memory) */
#define PXCL_WHERE_DEVICE 1   /* device memory on the context's device */

/* Input digis: structure of arrays, grouped by non-decreasing module id, any order
 * within a module -- or, with PXCL_DIGIS_ANY_ORDER in flags, in any order at all
 * (the raw data of the paper's Figure 1 carries no grouping): the library then
 * groups them by module on the device with a counting sort (per-chunk module
 * histograms, a scan of the module totals, a scatter into a grouped copy in the
 * event workspace) before the clustering, every per-digi output still goes to the
 * digi's input position, and PXCL_E_ORDER cannot occur.  The result is the same as
 * for the grouped digis.  All four arrays hold n uint16 values and must stay valid and
 * unmodified until the done callback has fired.
 * max_module_digis: optional upper bound on the digis of any one module (0 =
 * unknown).  When it is at most the small-module kernel's capacity (workgroup size /
 * modules per workgroup * 8 digis), neither big-module kernel is launched; when it
 * is at most 16,384 the scratch-mode kernel is not launched.  A module above the
 * bound is then not clustered and the event fails with PXCL_E_HINT. */
typedef struct {
    const uint16_t* module;
    const uint16_t* row;
    const uint16_t* col;
    const uint16_t* adc;
    uint32_t n;
    int32_t where;        /* PXCL_WHERE_HOST or PXCL_WHERE_DEVICE */
    uint32_t max_module_digis;
    uint32_t flags;       /* PXCL_DIGIS_ANY_ORDER | PXCL_DIGIS_HITS | PXCL_DIGIS_DEFER_BIG, or 0 */
} pxcl_digis;
#define PXCL_DIGIS_ANY_ORDER 1u
/* Deferred big-module kernels (single-event pxcl_acquire only; PXCL_E_INVAL in a
 * batch): the launch holds no big-module kernels.  If the small-module kernel finds
 * modules above its capacity it lists them and the compaction leaves the event
 * unfinished; the completion thread then queues the big-module kernels and the
 * compaction on the event's stream (a second launch, recording the completion event
 * again) before the callback fires.  Events without such modules finish in the one
 * launch, sparing the two big-module launches, which wait for whole compute units.
 * The results are final only when the callback fires: work queued after the acquire
 * on the same stream is not ordered after the second launch, and pxcl_hits_enqueue
 * and pxcl_copy_to_host return PXCL_E_BUSY while the event is in flight.  With
 * PXCL_DIGIS_HITS the hits are complete with the event, as without this flag.  If the
 * second launch cannot be queued, what was queued of it drains first and the callback
 * then fires with PXCL_E_INTERNAL (the event's results are not valid). */
#define PXCL_DIGIS_DEFER_BIG 4u
/* Hits fused into the clustering (Figure 1's GPU chain goes from raw data to hits): the
 * clustering kernels add every kept digi's adc*col and adc*row to exact 64-bit sums of
 * its cluster, and the compaction writes each cluster's hit beside its record, so the
 * hits are complete when the event is (pxcl_hits_enqueue then queues no kernel, only
 * the completion on its stream).  Same values as the hits kernel. */
#define PXCL_DIGIS_HITS 2u

/* Completion callback.  Runs on the context's completion thread once the event's
 * (or batch's) device work and status write-back are complete; status = PXCL_OK or
 * an async error code.  It must not block: the context's other completions wait
 * while it runs.  It may produce and acquire again; it may not destroy the context
 * (PXCL_E_BUSY).  It fires exactly once per successful pxcl_acquire /
 * pxcl_acquire_batch and never when they return an error. */
typedef void (*pxcl_done_cb)(void* user, int32_t status);

/* Results of one event (device pointers into the event's workspace).  Valid until
 * the next acquire on the event or its unbind. */
typedef struct {
    int32_t status;            /* PXCL_OK or the async error code */
    uint32_t err_bits;         /* PXCL_ERRBIT_* */
    uint32_t n_clusters;       /* kept clusters */
    uint32_t n_digis;
    const int32_t* id;         /* [n_clusters] ascending cluster ids */
    const int32_t* charge;     /* [n_clusters] */
    const int32_t* size;       /* [n_clusters] */
    const int32_t* digi_cluster; /* [n_digis] id of the digi's cluster if kept, else -1 */
    void* stream;              /* hipStream_t the work was queued on */
    void* done_event;          /* hipEvent_t recorded after the work */
    int32_t device;
} pxcl_clusters;

/* ---- context ---------------------------------------------------------------- */
/* Create a context on `device`.  Queries the device, sets the default kernel
 * configuration and starts the context's completion thread (asleep while nothing
 * is in flight).  Allocates only small host metadata. */
int pxcl_ctx_create(const pxcl_config* cfg, int device, pxcl_ctx** out);
/* Stops the completion thread.  PXCL_E_BUSY while events or batches are still
 * bound, or when called from a completion callback. */
int pxcl_ctx_destroy(pxcl_ctx* ctx);

/* Clustering kernel shape: workgroup size wg in {64,128,256,512} and modules per
 * workgroup mpw in {1,2,4} with wg/mpw >= 64.  Affects later acquires only. */
int pxcl_set_kernel_config(pxcl_ctx* ctx, uint32_t wg, uint32_t mpw);
int pxcl_get_kernel_config(const pxcl_ctx* ctx, uint32_t* wg, uint32_t* mpw);

/* Per-kernel device timing: hipEvents recorded on the launch stream around each
 * kernel of every period-th launch of each event or batch object (period 0: off,
 * the default; 1: every launch).  Launches that replay a captured graph are never
 * timed: elapsed times of events recorded inside a captured graph are not
 * available.  Stats: for each of the 5 kernels (0 segmentation, 1 big-module
 * clustering in register and scratch mode, 2 small-module clustering, 3 compaction,
 * 4 hits) the summed milliseconds and the number of timed launches; a kernel a launch
 * did not run (segmentation of single-event launches, big-module kernels skipped by
 * the size hint) is not counted; a launch is counted once its event (or its hits) is
 * produced, or the event or batch object is used again or unbound. */
int pxcl_set_timing(pxcl_ctx* ctx, int period);
int pxcl_get_timing(pxcl_ctx* ctx, double* ms_sum /*[5]*/, uint64_t* launches /*[5]*/, int reset);

/* ---- event slots ------------------------------------------------------------ */
/* Device workspace bytes for an event slot of capacity max_digis (inputs staged for
 * host digis, outputs, temporaries); 0 if max_digis is 0 or too large. */
size_t pxcl_event_workspace_bytes(const pxcl_ctx* ctx, uint32_t max_digis);
/* Pinned host bytes for an event slot's status block. */
size_t pxcl_event_pinned_bytes(const pxcl_ctx* ctx);

/* Bind caller-owned memory to a new event object.  d_ws: device memory on the
 * context's device, 256-byte aligned, >= pxcl_event_workspace_bytes; h_pinned:
 * pinned host memory, 64-byte aligned, >= pxcl_event_pinned_bytes.  The library
 * borrows both until pxcl_event_unbind.  Clears the slot's control words with
 * hipMemsetAsync on `stream` (a hipStream_t; NULL = the null stream). */
int pxcl_event_bind(pxcl_ctx* ctx, void* d_ws, size_t ws_bytes, void* h_pinned,
                    size_t pinned_bytes, uint32_t max_digis, void* stream, pxcl_event** out);
/* PXCL_E_BUSY while work is in flight.  Waits for a completion callback of the
 * event that is still running on another thread; called from inside such a
 * callback it returns PXCL_E_BUSY instead. */
int pxcl_event_unbind(pxcl_event* ev);
uint32_t pxcl_event_capacity(const pxcl_event* ev);

/* Enqueue the clustering of one event on `stream` (hipStream_t): an async copy of
 * host digis into the slot (PXCL_WHERE_HOST), the device kernels (a single event
 * needs no segmentation kernel: the small-module kernel finds every module's digis
 * by search and checks the module ids itself), and a completion event that the
 * context's completion thread polls.  Returns without waiting for the device.  Synchronous errors
 * (PXCL_E_INVAL, PXCL_E_CAPACITY, PXCL_E_BUSY, PXCL_E_HIP) mean nothing was queued
 * and `cb` will not be called; otherwise `cb` (may be NULL) fires exactly once. */
int pxcl_acquire(pxcl_event* ev, const pxcl_digis* in, void* stream, pxcl_done_cb cb,
                 void* user);
/* PXCL_OK once complete, PXCL_E_NOT_READY while in flight, PXCL_E_INVAL if never
 * acquired.  Non-blocking. */
int pxcl_query(const pxcl_event* ev);
/* Non-blocking.  PXCL_E_NOT_READY before completion; otherwise fills *out and
 * returns the event's status (PXCL_OK or the async error). */
int pxcl_produce(pxcl_event* ev, pxcl_clusters* out);
/* Blocking wait for tests and simple callers: hipEventSynchronize on the event's
 * completion event, then a wait until the completion callback of the launch has
 * returned (skipped when called from inside a completion callback).  The contrast
 * to the callback style, never used on the asynchronous paths. */
int pxcl_wait(pxcl_event* ev);

/* A ready-made callback: `user` points to a pxcl_flag; the callback stores the
 * status and then increments `fired` (release order). */
typedef struct {
    volatile int32_t status;
    volatile uint32_t fired;
} pxcl_flag;
void pxcl_flag_cb(void* user, int32_t status);

/* ---- hits: a consumer of an event's clusters ----------------------------------- */
/* The paper's Figure 1 (Sec. 3) derives hits from clusters.  Here a hit is the
 * charge-weighted centroid of a kept cluster's pixels, in pixel units:
 * x = sum(adc*col) / charge, y = sum(adc*row) / charge, from exact 64-bit sums
 * divided in double precision and rounded to float (NaN for zero charge), one per
 * kept cluster in the clusters' order.
 * pxcl_hits_enqueue queues the hits of the event's last acquire on `stream`
 * (a kernel over the event's clusters; for an event acquired with PXCL_DIGIS_HITS the
 * hits were computed with the clusters and only the completion is queued)
 * (hipStream_t) as a consumer of its clusters in the way Sec. 4.2 describes: when
 * `stream` is not the stream the event's work went to and that work may still be
 * running, `stream` first waits for the event's completion event; on the same
 * stream the order of the stream suffices.  The event must have been acquired and
 * its input digis must stay valid until `cb` fires (exactly once, with the event's
 * status).  PXCL_E_BUSY if hits of the event are in flight; an acquire of the event
 * returns PXCL_E_BUSY while they are.  Non-blocking. */
typedef struct {
    int32_t status;            /* the event's status */
    uint32_t n_hits;           /* = the event's kept clusters */
    const float* x;            /* [n_hits] column centroid (device) */
    const float* y;            /* [n_hits] row centroid (device) */
    void* stream;              /* hipStream_t the hits were queued on */
    void* done_event;          /* hipEvent_t recorded after them */
    int32_t device;
} pxcl_hits;
int pxcl_hits_enqueue(pxcl_event* ev, void* stream, pxcl_done_cb cb, void* user);
/* PXCL_OK once the hits are complete, PXCL_E_NOT_READY while in flight,
 * PXCL_E_INVAL if none were queued.  Non-blocking. */
int pxcl_hits_query(const pxcl_event* ev);
/* Non-blocking.  PXCL_E_NOT_READY before completion; otherwise fills *out (device
 * pointers into the event's workspace, valid until its next acquire or unbind) and
 * returns the status. */
int pxcl_hits_produce(pxcl_event* ev, pxcl_hits* out);
/* Blocking wait for the hits (tests and simple callers), like pxcl_wait. */
int pxcl_hits_wait(pxcl_event* ev);

/* ---- transfer to the host on demand ----------------------------------------------- */
/* Sec. 4.3: device results go to the host only when a CPU consumer asks.
 * pxcl_copy_to_host queues asynchronous device-to-host copies of the event's kept
 * clusters (and, if digi_cluster is set, its per-digi ids; if x and y are set, its
 * hits, which must have been queued) into caller-owned pinned buffers, on `stream`,
 * waiting for the event (and the hits) across streams like pxcl_hits_enqueue.  The
 * cluster arrays must hold `capacity` >= the event's kept clusters once it is
 * complete, or >= its digis while it may be in flight (PXCL_E_CAPACITY otherwise).
 * When `cb` fires (exactly once, with the event's status) the buffers hold the data
 * and n_clusters and status are set.  PXCL_E_BUSY while a copy of the event is in
 * flight; an acquire of the event returns PXCL_E_BUSY while it is.  Non-blocking. */
typedef struct {
    int32_t* id;               /* pinned host [capacity] */
    int32_t* charge;           /* pinned host [capacity] */
    int32_t* size;             /* pinned host [capacity] */
    int32_t* digi_cluster;     /* pinned host [n_digis], or NULL */
    float* x;                  /* pinned host [capacity] hits, or NULL (with y) */
    float* y;
    uint32_t capacity;
    uint32_t n_clusters;       /* out, when the callback fires */
    int32_t status;            /* out, when the callback fires */
} pxcl_host_clusters;
int pxcl_copy_to_host(pxcl_event* ev, void* stream, pxcl_host_clusters* dst, pxcl_done_cb cb, void* user);
/* PXCL_OK once the copy is complete, PXCL_E_NOT_READY while in flight, PXCL_E_INVAL
 * if none was queued.  Non-blocking. */
int pxcl_copy_query(const pxcl_event* ev);

/* ---- batches: many events in one launch --------------------------------------- */
size_t pxcl_batch_workspace_bytes(const pxcl_ctx* ctx, uint32_t max_events);
size_t pxcl_batch_pinned_bytes(const pxcl_ctx* ctx, uint32_t max_events);
int pxcl_batch_bind(pxcl_ctx* ctx, void* d_ws, size_t ws_bytes, void* h_pinned,
                    size_t pinned_bytes, uint32_t max_events, void* stream, pxcl_batch** out);
int pxcl_batch_unbind(pxcl_batch* b);

#define PXCL_BATCH_GRAPH 1u   /* replay a captured hipGraph of the per-batch pipeline */
/* Deferred big-module kernels for a whole batch: as PXCL_DIGIS_DEFER_BIG for one event
 * (the second launch, big-module kernels and the compaction of the events the first
 * launch left unfinished, is queued by the completion thread before the callback, only
 * if some event lists a module for them).  The events' results are final at the
 * callback; their hits and copy calls return PXCL_E_BUSY until then. */
#define PXCL_BATCH_DEFER_BIG 2u

/* Enqueue k events (each bound to its own slot, none in flight) as one batch: one
 * set of persistent kernels processes every module of every event.  ins[i] are
 * event evs[i]'s digis.  `cb` fires once per batch with PXCL_OK if every event
 * succeeded, else the first event error; each event's own status and results come
 * from pxcl_produce(evs[i]).  Same synchronous-error rules as pxcl_acquire. */
int pxcl_acquire_batch(pxcl_batch* b, pxcl_event* const* evs, const pxcl_digis* ins,
                       uint32_t k, void* stream, pxcl_done_cb cb, void* user, uint32_t flags);
int pxcl_batch_query(const pxcl_batch* b);

/* ---- autotuning ---------------------------------------------------------------- */
/* Time every kernel configuration (wg x mpw) on the given batch (reps replays each,
 * blocking: a setup-time call), select the fastest, and, if cache_path is not NULL,
 * record it in that JSON file under a key of device architecture and shape bucket.
 * us_out (may be NULL) receives 12 mean times in microseconds, wg-major
 * (64,128,256,512) x mpw (1,2,4); invalid combinations report -1. */
int pxcl_autotune(pxcl_ctx* ctx, pxcl_batch* b, pxcl_event* const* evs, const pxcl_digis* ins,
                  uint32_t k, void* stream, uint32_t reps, const char* cache_path,
                  float* us_out);
/* Load a configuration recorded by pxcl_autotune for this device and shape bucket
 * (mean digis per event).  PXCL_E_NOTFOUND if absent. */
int pxcl_autotune_load(pxcl_ctx* ctx, const char* cache_path, uint32_t mean_digis);

/* ---- drivers: the asynchronous and the serving forms ------------------------------ */
typedef struct {
    double wall_s;               /* timed wall-clock seconds */
    uint64_t events;             /* events completed */
    uint64_t digis;              /* digis clustered */
    double lat_p50_us, lat_p99_us, lat_max_us;
    double blocked_us_per_event; /* host wall time inside acquire + produce (+ waits) */
    double cpu_tasks_per_s;      /* synthetic CPU tasks completed per second */
    uint64_t cpu_tasks;
    uint32_t errors;             /* events whose status was not PXCL_OK */
    uint32_t max_inflight;       /* largest number of events in flight at once */
    uint64_t peak_resident_bytes;/* largest sum of the workspace bytes of occupied slots */
    uint64_t batches;            /* device launches (pxcl_acquire_batch calls) */
    /* serving form only: median and 99th percentile of the time requests spend in each
     * stage, in microseconds: [0] arrival -> admission (a free slot), [1] admission ->
     * launch (batching), [2] launch -> completion callback (device and completion
     * thread), [3] callback -> produce returned (a CPU thread picking it up) */
    double stage_p50_us[4];
    double stage_p99_us[4];
    double cpu_tasks_per_s_idle; /* serving form: the same CPU threads' task rate with no requests */
    double offered_per_s;        /* serving form: requests / time of the last arrival (the rate drawn) */
} pxcl_run_stats;

/* Asynchronous form: n_threads host threads, each owning evs[t] and stream
 * streams[t], keep one event in flight each; while it is in flight the thread runs
 * synthetic CPU tasks of cpu_task_ns nanoseconds (0 = none) and picks the event's
 * produce as soon as its callback has fired.  Thread t processes pool entries
 * t, t+n_threads, ... (mod pool_size), events_per_thread of them.  flags:
 * PXCL_RUN_BLOCKING: the thread instead waits with hipStreamSynchronize (the
 * contrast); PXCL_RUN_HITS: every event's hits are queued right behind it on the
 * same stream and produced with it.
 * Verification mode: with d_results and result_offsets given (both NULL: off), event
 * i of thread t (request r = t + i * n_threads, pool entry r mod pool_size) has its
 * results copied to d_results + result_offsets[r] after its produce (int32 per-digi
 * ids [n], then ids, charges, sizes [n_clusters each] at +4n, +8n, +12n bytes), and
 * the thread waits for the copy before it reuses its event; that wait counts as
 * blocked time.  result_offsets holds n_threads * events_per_thread entries. */
#define PXCL_RUN_BLOCKING 1
#define PXCL_RUN_HITS 2
int pxcl_run_async(pxcl_ctx* ctx, pxcl_event* const* evs, void* const* streams,
                   uint32_t n_threads, const pxcl_digis* pool, uint32_t pool_size,
                   uint32_t events_per_thread, uint32_t cpu_task_ns, int flags,
                   pxcl_run_stats* out, void* d_results, const uint64_t* result_offsets);

/* Serving form: requests arrive as a Poisson process (rate_hz, seeded) and draw
 * their digis round-robin from `pool`.  At set-up the device arena
 * [d_arena, d_arena + arena_bytes) is carved into at most n_slots event slots of
 * min(budget_bytes, arena_bytes) bytes in total, bound once, in size classes (powers
 * of two from 16,384 digis up to the largest request) shared out in proportion to the
 * requests that need each class; requests are admitted in arrival order, each to a
 * free slot of its class or else of the smallest larger class with one, and a request
 * that finds none waits without holding back later requests that can be admitted
 * (they can only take slots it cannot use); admission neither allocates nor clears
 * memory.  Every tick
 * the admitted requests not yet launched go to the device as one batch on a free batch
 * object (continuous batching: batches on different streams overlap), at most
 * max_inflight of them on the device at once: while they run, arrivals accumulate, so
 * batches grow with the load instead of the latency.  n_cpu_threads
 * threads run synthetic CPU tasks (cpu_task_ns each) and the produce work, at a lower
 * priority than the dispatcher; with at least four CPUs in the process's affinity set
 * the dispatcher (the calling thread) keeps the last CPU to itself, the context's
 * completion thread the one before, and the CPU threads stay off both (both
 * affinities are restored on return).
 * Latency = arrival -> produce returned.  h_pinned must hold n_slots event status
 * blocks (pxcl_event_pinned_bytes each).
 * Verification mode: with d_results and result_offsets given, the produce step also
 * copies request r's results to d_results + result_offsets[r] (int32 per-digi ids
 * [n], then ids, charges, sizes [n_clusters each] at +4n, +8n, +12n bytes) and waits
 * for the copy before the workspace is released; that wait counts as blocked time. */
typedef struct {
    double rate_hz;
    uint32_t n_requests;
    uint64_t budget_bytes;
    uint32_t n_slots;            /* event slots at most (max requests resident at once) */
    uint32_t max_batch;          /* events per launch (<= each batch's capacity) */
    uint32_t n_cpu_threads;
    uint32_t cpu_task_ns;
    uint32_t flags;              /* PXCL_BATCH_GRAPH | PXCL_BATCH_DEFER_BIG */
    uint64_t seed;
    uint32_t max_inflight;       /* batches on the device at once (0 = n_batches) */
    uint32_t batch_delay_us;     /* 0: a batch starts as soon as fewer than max_inflight are on
                                    the device; else, while others run, it waits to be half
                                    full or for its oldest request to have waited this long */
} pxcl_serve_opts;
int pxcl_serve(pxcl_ctx* ctx, void* d_arena, size_t arena_bytes, void* h_pinned,
               size_t pinned_bytes, pxcl_batch* const* batches, void* const* streams,
               uint32_t n_batches, const pxcl_digis* pool, uint32_t pool_size,
               const pxcl_serve_opts* opts, pxcl_run_stats* out,
               int32_t* request_status /* [n_requests] or NULL */,
               uint32_t* request_nclusters /* [n_requests] or NULL */,
               void* d_results /* device, or NULL */,
               const uint64_t* result_offsets /* [n_requests] byte offsets, or NULL */);

/* ---- allocation-free clustering of one event ------------------------------------ */
/* For callers that cannot allocate device memory or bind a workspace: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  The same
 * kernels as pxcl_acquire cluster one event whose digis are in device memory, but
 * their scratch (control words, per-module table and lists, cluster records before
 * compaction) lives in a fixed device array of the library, one per GPU, held until
 * the process ends: PXCL_NOALLOC_SCRATCH_BYTES, sized for events of at most
 * PXCL_NOALLOC_MAX_DIGIS digis and PXCL_MAX_MODULES modules.  Nothing is allocated,
 * freed or bound by the call; the array's address on each device is looked up once,
 * by pxcl_ctx_create on that device.
 *
 * Stream-ordered, no callback: the work is queued on `stream` (hipStream_t) and the
 * results are complete when the stream reaches that point (synchronise, record an
 * event, or capture the call into a graph).  `in` must be device digis
 * (PXCL_WHERE_DEVICE), grouped by module as for pxcl_acquire; max_module_digis is
 * honoured the same way.  Outputs, caller-owned device memory:
 *   digi_cluster [n]  per-digi cluster id, -1 if cut;
 *   id, charge, size [n each]  kept clusters in ascending id in the first
 *       n_clusters entries (all n entries may be written: they also hold
 *       per-cluster temporaries of the largest modules);
 *   status [16 words, 4-byte aligned]  written at the end of the work: word 0 the
 *       call's launch tag (also returned in *tag), word 1 the PXCL_ERRBIT_* error bits
 *       of the event, word 2 the number of kept clusters.
 * A call with n = 0 writes only status.  Returns PXCL_E_CAPACITY if n exceeds
 * PXCL_NOALLOC_MAX_DIGIS (nothing queued), PXCL_E_INVAL for a null or host input or
 * a null output, PXCL_E_HIP if the device array could not be located or a launch
 * failed.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU (on
 * different streams, or from different threads without ordering) race and give
 * wrong results.  Calls in one stream, or otherwise ordered, are safe; after a
 * failed launch the next call clears the control words with a kernel first. */
#define PXCL_NOALLOC_MAX_DIGIS 262144u
#define PXCL_NOALLOC_SCRATCH_BYTES 15972352u
typedef struct {
    int32_t* digi_cluster;
    int32_t* id;
    int32_t* charge;
    int32_t* size;
    uint32_t* status;
} pxcl_noalloc_out;
int pxcl_cluster_noalloc(pxcl_ctx* ctx, const pxcl_digis* in, const pxcl_noalloc_out* out,
                         void* stream, uint32_t* tag);

/* ---- misc --------------------------------------------------------------------- */
const char* pxcl_strerror(int code);
/* Library version string. */
const char* pxcl_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PXCL_H */
