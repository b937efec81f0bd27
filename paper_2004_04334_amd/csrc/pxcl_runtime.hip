// Host runtime of the pixel-clustering library: the C ABI of include/pxcl.h.
//
// acquire() only validates, stages host inputs with async copies, launches the
// kernels on the caller's stream and records a completion event -- the split
// of a module's work into acquire/produce with a completion callback that releases
// the waiting task (paper Sec. 2 and Sec. 4.1).  The callback runs on the context's
// completion thread, which polls the completion events of the launches in flight:
// a host function queued into the stream (the mechanism of Sec. 4.1) costs the
// calling thread tens of microseconds per launch here and fires tens of
// microseconds after the work ends, while a query of an event is a read of its
// signal.  No device or pinned allocation happens after bind.
#include <hip/hip_runtime.h>
#include <pthread.h>
#include <sched.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <unistd.h>
#include <vector>

#include "../../include/pxcl.h"
#include "pxcl_internal.h"

namespace pxcl {
bool cluster_config_valid(u32 wg, u32 mpw);
u32 cluster_capacity(u32 wg, u32 mpw);
int occupancy_segment();
int occupancy_cluster(u32 wg, u32 mpw);
int occupancy_big();
int occupancy_compact();
hipError_t launch_segment(const LaunchArgs& a, u32 grid, hipStream_t s);
hipError_t launch_small(u32 wg, u32 mpw, const LaunchArgs& a, u32 grid, hipStream_t s);
hipError_t launch_big(const LaunchArgs& a, u32 grid, u32 grid_scratch, hipStream_t s);
int occupancy_scratch();
hipError_t launch_compact(const LaunchArgs& a, u32 grid, hipStream_t s);
u32 compact_waves_per_block(u32 waves, u32 blocks);
int occupancy_hits();
hipError_t launch_hits(const LaunchArgs& a, u32 grid, hipStream_t s);
hipError_t launch_fill(u32* p, u32 n, u32 v, hipStream_t s);
int occupancy_group();
u32 group_chunk();
u32 group_scatter_chunk();
hipError_t launch_group(const LaunchArgs& a, u32 grid, u32 grid_events, u32 grid_scatter, hipStream_t s);
}  // namespace pxcl

using namespace pxcl;

namespace {

enum : int { ST_IDLE = 0, ST_INFLIGHT = 1, ST_DONE = 2 };

// Launch tags for look-back status words: unique within the process and seeded
// per process so that stale words left in reused memory do not match.
std::atomic<u32> g_epoch{0};
u32 next_epoch() {
    static std::once_flag once;
    std::call_once(once, [] {
        u64 t = (u64)std::chrono::steady_clock::now().time_since_epoch().count();
        u64 x = t ^ ((u64)getpid() << 32) ^ 0x9E3779B97F4A7C15ull;
        x ^= x >> 33; x *= 0xff51afd7ed558ccdull; x ^= x >> 33;
        g_epoch.store(u32(x) | 1u);
    });
    u32 e;
    do { e = g_epoch.fetch_add(1u); } while (e == 0u);
    return e;
}

int status_from_bits(u32 bits) {
    if (bits & EB_RANGE) return PXCL_E_RANGE;
    if (bits & EB_ORDER) return PXCL_E_ORDER;
    if (bits & EB_HINT) return PXCL_E_HINT;
    if (bits & EB_DUP) return PXCL_E_DUP_PIXEL;
    if (bits & EB_INTERNAL) return PXCL_E_INTERNAL;
    return PXCL_OK;
}

// A launch whose completion event the completion thread polls.
enum : int { CK_EVENT = 0, CK_BATCH = 1, CK_HITS = 2, CK_COPY = 3 };
struct Pending {
    int kind;
    void* obj;          // pxcl_event* or pxcl_batch*
    hipEvent_t done;    // recorded after the launch's work
};

}  // namespace

struct pxcl_completer {
    std::mutex mu;
    std::condition_variable cv;
    std::vector<Pending> in;           // posted, not yet taken by the thread
    std::atomic<bool> has_in{false};
    bool stop = false, idle = false;
    std::thread th;
};

struct pxcl_ctx {
    int device = 0;
    u32 n_modules = 0, charge_cut = 0;
    u32 n_cu = 0;
    std::string arch;
    std::atomic<u32> wg{256}, mpw{1};
    int occ_a = 1, occ_l = 1, occ_c = 1, occ_h = 1, occ_x = 1, occ_g = 1;
    int occ_s[4][5] = {};               // small kernel per shape [log2(wg) - 6][mpw], queried once
    std::atomic<int> bound{0};
    std::atomic<int> timing{0};
    std::mutex tmu;
    double tsum[5] = {0, 0, 0, 0, 0};   // segment, big, small, compact, hits
    u64 tcnt[5] = {0, 0, 0, 0, 0};
    pxcl_completer comp;
};

struct pxcl_event {
    pxcl_ctx* ctx = nullptr;
    u8* ws = nullptr;
    size_t ws_bytes = 0;
    u32 cap = 0;
    u32* hs = nullptr;        // host view of the status block
    u32* hs_dev = nullptr;    // device view of the same pinned memory
    std::atomic<int> state{ST_IDLE};
    u32 epoch = 0, n = 0;
    int32_t status = PXCL_OK;
    u32 err_bits = 0, ncl = 0;
    hipStream_t stream = nullptr;
    hipEvent_t done_ev = nullptr;
    hipEvent_t tev[5] = {};
    bool timed = false;
    pxcl_done_cb cb = nullptr;
    void* user = nullptr;
    pxcl_batch* batch = nullptr;
    std::atomic<int> cb_pending{0};   // launches whose completion callback has not returned
    u32 launches = 0;                 // for sampling launches to time
    u32 timed_flags = 0;              // launch flags of the timed launch (kernels it ran)
    EventDesc desc{};                 // the event as the kernels saw it (for the hits)
    // a launch with the big-module kernels deferred (PXCL_DIGIS_DEFER_BIG): its
    // arguments and grids for the second launch, and whether that is still possible
    bool defer = false;
    bool defer_first = false;         // the first launch's completion is pending
    LaunchArgs defer_args{};
    u32 defer_grid_b = 1, defer_grid_x = 1, defer_grid_c = 1;
    u32 slot = 0;                     // launch parity of the last launch
    bool dirty = false;               // a launch failed to queue or reported an error: clear
                                      // the control words, grouping counts and hit sums first
    // hits of the last acquired event
    std::atomic<int> hstate{ST_IDLE};
    std::atomic<int> hits_pending{0};
    hipEvent_t hits_ev = nullptr;
    hipEvent_t hits_done = nullptr;   // the event the last hits completion waits for
    hipEvent_t hits_tev[2] = {};      // around the hits kernel of a timed launch
    bool hits_timed = false;
    u32 hits_launches = 0;
    hipStream_t hits_stream = nullptr;
    pxcl_done_cb hits_cb = nullptr;
    void* hits_user = nullptr;
    int32_t hits_status = PXCL_OK;
    u32 hits_n = 0;
    // copy to host of the last acquired event
    std::atomic<int> cstate{ST_IDLE};
    std::atomic<int> copy_pending{0};
    hipEvent_t copy_ev = nullptr;
    pxcl_host_clusters* copy_dst = nullptr;
    pxcl_done_cb copy_cb = nullptr;
    void* copy_user = nullptr;
};

struct pxcl_batch {
    pxcl_ctx* ctx = nullptr;
    u8* ws = nullptr;
    size_t ws_bytes = 0;
    u8* hp = nullptr;         // pinned staging of the header
    u32 max_events = 0;
    std::atomic<int> state{ST_IDLE};
    pxcl_event* evs[MAXB] = {};
    u32 k = 0;
    int32_t status = PXCL_OK;
    pxcl_done_cb cb = nullptr;
    void* user = nullptr;
    hipEvent_t done_ev = nullptr;
    hipStream_t cap_stream = nullptr;
    // captured pipelines, one per combination of the launch flags that change it
    // (LF_NO_BIG, LF_SEG_WIDE, LF_NO_SCRATCH, LF_GROUP, LF_NO_SEG, LF_DEFER), all for
    // the kernel shape g_wg x g_mpw
    static constexpr int N_GRAPHS = 64;
    hipGraphExec_t gexec[N_GRAPHS] = {};
    hipGraph_t graph[N_GRAPHS] = {};
    u32 g_wg = 0, g_mpw = 0;
    u32 launches = 0;
    u32 timed_flags = 0;
    hipEvent_t tev[5] = {};
    bool timed = false;       // the launch in flight records per-kernel events
    // deferred big-module kernels (PXCL_BATCH_DEFER_BIG): the second launch's
    // arguments and grids, and whether the first launch's completion is pending
    hipStream_t stream = nullptr;
    bool defer_first = false;
    LaunchArgs defer_args{};
    u32 defer_grid_b = 1, defer_grid_x = 1, defer_grid_c = 1;
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
namespace {

struct Grids {
    u32 a, b, s, c, x;   // segment, big, small, compact, scratch
    u32 g, ge, gs;       // grouping of digis in any order: count, table, scatter
};

// Wide segmentation chunks once a launch holds at least one of them per compute
// unit: the chip is still filled and the end-of-chunk atomics are four times fewer.
static u32 seg_flag(const pxcl_ctx* ctx, u64 digis) {
    return digis >= (u64)ctx->n_cu * seg_chunk(LF_SEG_WIDE) ? LF_SEG_WIDE : 0u;
}

// Grids of the kernels.  `digis` bounds the launch's digis and `present` its
// modules present (at most min(digis, modules) per event); with `full` (a captured
// graph replays with any input)
// every kernel gets what fits on the device at once.
Grids grids_for(const pxcl_ctx* ctx, u32 wg, u32 mpw, u64 digis, u64 present, u32 k, u32 flags, bool full,
                u64 any_digis = 0, u32 any_events = 0) {
    Grids g;
    const u64 ncu = ctx->n_cu;
    const u64 fa = ncu * (u64)ctx->occ_a;
    const u64 fb = ncu * (u64)ctx->occ_l;
    const u64 fs = ncu * (u64)ctx->occ_s[31 - __builtin_clz(wg) - 6][mpw];
    const u64 fc = ncu * (u64)ctx->occ_c;
    // modules above BIG_RCAP digis are rare outliers (one per stress event): the scratch
    // kernel's workgroups, each holding a whole compute unit's LDS, are capped at a
    // quarter of the chip, the rest loop
    const u64 fx = std::min<u64>(ncu * (u64)ctx->occ_x, std::max<u64>(ncu / 4, 1));
    const u64 fg = ncu * (u64)ctx->occ_g;
    if (full) {
        g.a = u32(fa); g.b = u32(fb); g.s = u32(fs); g.c = u32(fc); g.x = u32(fx);
        g.g = u32(fg); g.ge = u32(std::min<u64>(ncu, MAXB)); g.gs = u32(fg);
        return g;
    }
    const u64 gch = group_chunk();
    g.g = u32(std::max<u64>(1, std::min<u64>(fg, (any_digis + gch - 1) / gch + any_events)));
    const u64 gsc = group_scatter_chunk();
    g.gs = u32(std::max<u64>(1, std::min<u64>(fg, (any_digis + gsc - 1) / gsc + any_events)));
    g.ge = std::max<u32>(1u, any_events);
    const u32 dcap = cluster_capacity(wg, mpw);
    const u64 ch = seg_chunk(flags);
    g.a = u32(std::max<u64>(1, std::min<u64>(fa, (digis + ch - 1) / ch + k)));
    g.b = u32(std::max<u64>(1, std::min<u64>(fb, digis / (dcap + 1))));
    g.x = u32(std::max<u64>(1, std::min<u64>(fx, digis / (BIG_RCAP + 1))));
    g.s = u32(std::max<u64>(1, std::min<u64>(fs, (present + mpw - 1) / mpw)));
    // compaction: a wave per 64 modules, or several when that fills less than the device
    const u64 blocks = u64(k) * ((ctx->n_modules + 63) / 64);
    const u64 split = compact_waves_per_block(u32(std::min<u64>(fc * (C_WG / 64), 0xFFFFFFFFull)),
                                              u32(std::min<u64>(blocks, 0xFFFFFFFFull)));
    g.c = u32(std::max<u64>(1, std::min<u64>(fc, (blocks * split + C_WG / 64 - 1) / (C_WG / 64))));
    return g;
}

hipError_t launch_all(const LaunchArgs& a, const Grids& g, u32 wg, u32 mpw, hipStream_t s, hipEvent_t* tev) {
    hipError_t e;
    if (tev && (e = hipEventRecord(tev[0], s)) != hipSuccess) return e;
    if ((a.flags & LF_GROUP) && (e = launch_group(a, g.g, g.ge, g.gs, s)) != hipSuccess) return e;
    if (!(a.flags & (LF_FUSED | LF_NO_SEG)) && (e = launch_segment(a, g.a, s)) != hipSuccess) return e;
    if (tev && (e = hipEventRecord(tev[1], s)) != hipSuccess) return e;
    if ((e = launch_small(wg, mpw, a, g.s, s)) != hipSuccess) return e;   // lists the big modules
    if (tev && (e = hipEventRecord(tev[2], s)) != hipSuccess) return e;
    if (!(a.flags & LF_NO_BIG) && (e = launch_big(a, g.b, g.x, s)) != hipSuccess) return e;
    if (tev && (e = hipEventRecord(tev[3], s)) != hipSuccess) return e;
    if ((e = launch_compact(a, g.c, s)) != hipSuccess) return e;
    if (tev && (e = hipEventRecord(tev[4], s)) != hipSuccess) return e;
    return hipSuccess;
}

bool digis_ok(const pxcl_digis* in) {
    if (!in) return false;
    if (in->where != PXCL_WHERE_HOST && in->where != PXCL_WHERE_DEVICE) return false;
    if (in->n && (!in->module || !in->row || !in->col || !in->adc)) return false;
    if (in->flags & ~(PXCL_DIGIS_ANY_ORDER | PXCL_DIGIS_HITS | PXCL_DIGIS_DEFER_BIG)) return false;
    return true;
}

// The event as the kernels see it, its host inputs staged into the slot (one async
// copy per array: the caller's four arrays need not be adjacent).  The launch parity
// alternates; after a launch whose work was not all queued the control words are
// cleared first (a count that launch left would otherwise carry over).
hipError_t make_desc(pxcl_event* ev, const pxcl_digis* in, hipStream_t s, EventDesc* d) {
    const EvLayout L = ev_layout(ev->cap, ev->ctx->n_modules);
    if (ev->dirty) {
        hipError_t e = hipMemsetAsync(ev->ws + L.ctl, 0, CTL_WORDS * 4, s);
        if (e == hipSuccess) e = hipMemsetAsync(ev->ws + L.gcnt, 0, size_t(4) * ev->ctx->n_modules, s);
        if (e == hipSuccess) e = hipMemsetAsync(ev->ws + L.hsum, 0, size_t(16) * ev->cap, s);
        if (e != hipSuccess) return e;
        ev->dirty = false;
    }
    ev->slot ^= 1u;
    std::memset(d, 0, sizeof(*d));
    d->ws = ev->ws;
    d->hstat = ev->hs_dev;
    d->o_digi = reinterpret_cast<int32_t*>(ev->ws + L.digi);
    d->o_id = reinterpret_cast<int32_t*>(ev->ws + L.id);
    d->o_charge = reinterpret_cast<int32_t*>(ev->ws + L.charge);
    d->o_size = reinterpret_cast<int32_t*>(ev->ws + L.size);
    d->n = in->n;
    d->cap = ev->cap;
    d->epoch = ev->epoch;
    d->slot = ev->slot;
    // digis in any order: the kernels read them through r_* and cluster the grouped
    // copy the grouping kernels write to the workspace
    const bool any = (in->flags & PXCL_DIGIS_ANY_ORDER) != 0;
    if (in->flags & PXCL_DIGIS_HITS) d->flags |= EF_HITS;
    const u16** dst[4] = {&d->module, &d->row, &d->col, &d->adc};
    if (any) {
        d->flags |= EF_UNSORTED;
        u16* g = reinterpret_cast<u16*>(ev->ws + L.grp);
        for (int i = 0; i < 4; ++i) *dst[i] = g + size_t(i) * ev->cap;
        dst[0] = &d->r_module; dst[1] = &d->r_row; dst[2] = &d->r_col; dst[3] = &d->r_adc;
    }
    if (in->where == PXCL_WHERE_DEVICE) {
        *dst[0] = in->module; *dst[1] = in->row; *dst[2] = in->col; *dst[3] = in->adc;
        return hipSuccess;
    }
    u16* m = reinterpret_cast<u16*>(ev->ws + L.in_mod);
    u16* r = reinterpret_cast<u16*>(ev->ws + L.in_row);
    u16* c = reinterpret_cast<u16*>(ev->ws + L.in_col);
    u16* a = reinterpret_cast<u16*>(ev->ws + L.in_adc);
    *dst[0] = m; *dst[1] = r; *dst[2] = c; *dst[3] = a;
    const size_t b = size_t(in->n) * 2;
    if (!b) return hipSuccess;
    hipError_t e;
    if ((e = hipMemcpyAsync(m, in->module, b, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(r, in->row, b, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(c, in->col, b, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    return hipMemcpyAsync(a, in->adc, b, hipMemcpyHostToDevice, s);
}

void finish_event_from_host_status(pxcl_event* ev) {
    volatile u32* hs = ev->hs;
    const u32 tag = __atomic_load_n(&ev->hs[HS_EPOCH], __ATOMIC_ACQUIRE);
    u32 bits = hs[HS_ERR];
    if (tag != ev->epoch) bits |= EB_INTERNAL;       // status write-back missing
    if (bits & EB_DEFER) bits = (bits & ~EB_DEFER) | (bits == EB_DEFER ? EB_INTERNAL : 0u);   // not finished
    ev->err_bits = bits;
    const u32 ncl = hs[HS_NCL];
    ev->ncl = ncl < ev->n ? ncl : ev->n;              // never more clusters than digis
    ev->status = status_from_bits(bits);
    // after an error some staged sums of fused hits may not have been read back and
    // zeroed by the compaction: the next launch clears the slot's scratch first
    if (ev->status != PXCL_OK) ev->dirty = true;
}

// Set while a completion callback runs on this thread: a wait called from inside
// the callback must not wait for the callback itself.
thread_local int t_in_callback = 0;

// The second launch of an event whose big-module kernels were deferred: those
// kernels and the compaction, on the event's stream, then its completion event again.
bool relaunch_deferred(pxcl_event* ev) {
    const LaunchArgs& a = ev->defer_args;
    hipError_t e = launch_big(a, ev->defer_grid_b, ev->defer_grid_x, ev->stream);
    if (e == hipSuccess) e = launch_compact(a, ev->defer_grid_c, ev->stream);
    if (e == hipSuccess) e = hipEventRecord(ev->done_ev, ev->stream);
    if (e != hipSuccess) {
        // part of the second launch may be queued: let it drain before the event is
        // finished (with an error) and its slot can be launched again
        (void)hipGetLastError();
        (void)hipStreamSynchronize(ev->stream);
        (void)hipGetLastError();
    }
    return e == hipSuccess;
}

// false: the event goes on (its deferred second launch is queued, its completion
// event recorded again), true: it is complete and its callback has run.
bool event_complete(void* p) {
    pxcl_event* ev = static_cast<pxcl_event*>(p);
    if (ev->defer_first) {
        ev->defer_first = false;
        const u32 tag = __atomic_load_n(&ev->hs[HS_EPOCH], __ATOMIC_ACQUIRE);
        const u32 bits = static_cast<volatile u32*>(ev->hs)[HS_ERR];
        // modules above the small kernel's capacity and no input error: second launch
        if (tag == ev->epoch && bits == EB_DEFER && relaunch_deferred(ev)) return false;
    }
    finish_event_from_host_status(ev);
    pxcl_done_cb cb = ev->cb;
    void* user = ev->user;
    const int32_t st = ev->status;
    ev->state.store(ST_DONE, std::memory_order_release);   // the callback may produce and re-acquire
    if (cb) {
        ++t_in_callback;
        cb(user, st);
        --t_in_callback;
    }
    ev->cb_pending.fetch_sub(1, std::memory_order_acq_rel);
    return true;
}

// The second launch of a batch whose big-module kernels were deferred.
bool relaunch_deferred(pxcl_batch* b) {
    const LaunchArgs& a = b->defer_args;
    hipError_t e = launch_big(a, b->defer_grid_b, b->defer_grid_x, b->stream);
    if (e == hipSuccess) e = launch_compact(a, b->defer_grid_c, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->done_ev, b->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();            // as for one event: drain what was queued
        (void)hipStreamSynchronize(b->stream);
        (void)hipGetLastError();
    }
    return e == hipSuccess;
}

// false: the batch goes on (its deferred second launch is queued), true: complete.
bool batch_complete(void* p) {
    pxcl_batch* b = static_cast<pxcl_batch*>(p);
    if (b->defer_first) {
        b->defer_first = false;
        bool any = false;
        for (u32 i = 0; i < b->k && !any; ++i) {
            const pxcl_event* ev = b->evs[i];
            any = __atomic_load_n(&ev->hs[HS_EPOCH], __ATOMIC_ACQUIRE) == ev->epoch &&
                  (static_cast<volatile u32*>(ev->hs)[HS_ERR] & EB_DEFER) != 0;
        }
        if (any && relaunch_deferred(b)) return false;
    }
    int32_t bst = PXCL_OK;
    for (u32 i = 0; i < b->k; ++i) {
        pxcl_event* ev = b->evs[i];
        finish_event_from_host_status(ev);
        if (bst == PXCL_OK && ev->status != PXCL_OK) bst = ev->status;
    }
    b->status = bst;
    pxcl_done_cb cb = b->cb;
    void* user = b->user;
    const u32 k = b->k;
    pxcl_event* evs[MAXB];                         // the callback may launch the batch again
    for (u32 i = 0; i < k; ++i) evs[i] = b->evs[i];
    for (u32 i = 0; i < k; ++i) evs[i]->state.store(ST_DONE, std::memory_order_release);
    b->state.store(ST_DONE, std::memory_order_release);
    if (cb) {
        ++t_in_callback;
        cb(user, bst);
        --t_in_callback;
    }
    for (u32 i = 0; i < k; ++i) evs[i]->cb_pending.fetch_sub(1, std::memory_order_acq_rel);
    return true;
}

bool claim(std::atomic<int>& st) {
    int cur = st.load(std::memory_order_acquire);
    while (cur != ST_INFLIGHT) {
        if (st.compare_exchange_weak(cur, ST_INFLIGHT, std::memory_order_acq_rel)) return true;
    }
    return false;
}

}  // namespace

// ---------------------------------------------------------------------------
// completion thread
// ---------------------------------------------------------------------------
static void completer_loop(pxcl_completer* c, int device);

// Hand a launch to the completion thread; its completion step and callback run once
// `done` has completed.
static void completer_post(pxcl_ctx* ctx, int kind, void* obj, hipEvent_t done) {
    pxcl_completer& c = ctx->comp;
    bool wake;
    {
        std::lock_guard<std::mutex> g(c.mu);
        c.in.push_back(Pending{kind, obj, done});
        c.has_in.store(true, std::memory_order_release);
        wake = c.idle;
    }
    if (wake) c.cv.notify_one();
}

// ---------------------------------------------------------------------------
// scratch of the allocation-free entry point: one fixed event workspace per GPU
// (capacity PXCL_NOALLOC_MAX_DIGIS digis, PXCL_MAX_MODULES modules).  In host code
// `scratch` is only a stand-in for the symbol: its device address on each GPU comes
// from hipGetSymbolAddress, looked up once per device with that device current.
// ---------------------------------------------------------------------------
constexpr u32 NOALLOC_CAP = PXCL_NOALLOC_MAX_DIGIS;
// The entry point takes no input flags, so its kernels never reach the fused-hit sums
// at the end of the layout: the array ends where they would begin.
static_assert(ev_layout(NOALLOC_CAP, PXCL_MAX_MODULES).hsum == PXCL_NOALLOC_SCRATCH_BYTES,
              "PXCL_NOALLOC_SCRATCH_BYTES matches the workspace layout");
static __device__ __align__(256) u8 scratch[PXCL_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_DEVICES = 64;
struct NoAllocDevice {
    std::once_flag once;
    u8* ptr = nullptr;                  // device address of `scratch` on this device
    std::atomic<u32> slot{0};           // launch parity of the calls on this device
    std::atomic<bool> dirty{false};     // a launch failed: clear the control words first
};
NoAllocDevice g_noalloc[NOALLOC_DEVICES];

// Once per device, with `device` current: locate the array and clear its control
// words and module table (set-up time, so a blocking wait is allowed here).
void noalloc_setup(int device) {
    if (device < 0 || device >= NOALLOC_DEVICES) return;
    NoAllocDevice& d = g_noalloc[device];
    std::call_once(d.once, [&d] {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return;                           // the entry point then reports PXCL_E_HIP
        }
        u8* base = static_cast<u8*>(p);
        const EvLayout L = ev_layout(NOALLOC_CAP, PXCL_MAX_MODULES);
        hipError_t e = launch_fill(reinterpret_cast<u32*>(base + L.ctl), CTL_WORDS, 0u, nullptr);
        if (e == hipSuccess) e = launch_fill(reinterpret_cast<u32*>(base + L.mtab), 4u * PXCL_MAX_MODULES, 0u, nullptr);
        if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return;
        }
        d.ptr = base;
    });
}
}  // namespace

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
extern "C" int pxcl_ctx_create(const pxcl_config* cfg, int device, pxcl_ctx** out) {
    if (!cfg || !out || cfg->n_modules == 0 || cfg->n_modules > PXCL_MAX_MODULES) return PXCL_E_INVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PXCL_E_INVAL;
    int prev = 0;
    hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess) return PXCL_E_HIP;
    pxcl_ctx* c = new pxcl_ctx();
    c->device = device;
    c->n_modules = cfg->n_modules;
    c->charge_cut = cfg->charge_cut;
    int ncu = 0;
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);
    c->n_cu = ncu > 0 ? u32(ncu) : 1u;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        std::string a(prop.gcnArchName);
        c->arch = a.substr(0, a.find(':'));
    }
    c->occ_a = occupancy_segment();
    for (u32 w = 64; w <= 512; w *= 2)
        for (u32 m = 1; m <= 4; m *= 2)
            if (cluster_config_valid(w, m)) c->occ_s[31 - __builtin_clz(w) - 6][m] = occupancy_cluster(w, m);
    c->occ_l = occupancy_big();
    c->occ_x = occupancy_scratch();
    c->occ_c = occupancy_compact();
    c->occ_h = occupancy_hits();
    c->occ_g = occupancy_group();
    noalloc_setup(device);
    hipSetDevice(prev);
    try {
        c->comp.th = std::thread(completer_loop, &c->comp, device);
    } catch (...) {
        delete c;
        return PXCL_E_INTERNAL;
    }
    *out = c;
    return PXCL_OK;
}

extern "C" int pxcl_ctx_destroy(pxcl_ctx* ctx) {
    if (!ctx) return PXCL_E_INVAL;
    if (ctx->bound.load() != 0) return PXCL_E_BUSY;   // nothing bound, so nothing in flight
    if (t_in_callback) return PXCL_E_BUSY;            // the callback runs on the thread to stop
    {
        std::lock_guard<std::mutex> g(ctx->comp.mu);
        ctx->comp.stop = true;
    }
    ctx->comp.cv.notify_one();
    if (ctx->comp.th.joinable()) ctx->comp.th.join();
    delete ctx;
    return PXCL_OK;
}

extern "C" int pxcl_set_kernel_config(pxcl_ctx* ctx, uint32_t wg, uint32_t mpw) {
    if (!ctx || !cluster_config_valid(wg, mpw)) return PXCL_E_INVAL;
    ctx->wg.store(wg);
    ctx->mpw.store(mpw);
    return PXCL_OK;
}

extern "C" int pxcl_get_kernel_config(const pxcl_ctx* ctx, uint32_t* wg, uint32_t* mpw) {
    if (!ctx || !wg || !mpw) return PXCL_E_INVAL;
    *wg = ctx->wg.load();
    *mpw = ctx->mpw.load();
    return PXCL_OK;
}

extern "C" int pxcl_set_timing(pxcl_ctx* ctx, int period) {
    if (!ctx || period < 0) return PXCL_E_INVAL;
    ctx->timing.store(period);
    return PXCL_OK;
}

extern "C" int pxcl_get_timing(pxcl_ctx* ctx, double* ms_sum, uint64_t* launches, int reset) {
    if (!ctx) return PXCL_E_INVAL;
    std::lock_guard<std::mutex> g(ctx->tmu);
    for (int i = 0; i < 5; ++i) {
        if (ms_sum) ms_sum[i] = ctx->tsum[i];
        if (launches) launches[i] = ctx->tcnt[i];
        if (reset) { ctx->tsum[i] = 0; ctx->tcnt[i] = 0; }
    }
    return PXCL_OK;
}

// ---------------------------------------------------------------------------
// events
// ---------------------------------------------------------------------------
extern "C" size_t pxcl_event_workspace_bytes(const pxcl_ctx* ctx, uint32_t max_digis) {
    if (!ctx || max_digis == 0 || max_digis > PXCL_MAX_EVENT_DIGIS) return 0;
    return ev_layout(max_digis, ctx->n_modules).total;
}

extern "C" size_t pxcl_event_pinned_bytes(const pxcl_ctx* ctx) { return ctx ? HS_BYTES : 0; }

extern "C" int pxcl_event_bind(pxcl_ctx* ctx, void* d_ws, size_t ws_bytes, void* h_pinned, size_t pinned_bytes,
                               uint32_t max_digis, void* stream, pxcl_event** out) {
    if (!ctx || !d_ws || !h_pinned || !out) return PXCL_E_INVAL;
    if (max_digis == 0 || max_digis > PXCL_MAX_EVENT_DIGIS) return PXCL_E_INVAL;
    if ((reinterpret_cast<uintptr_t>(d_ws) & 255u) || (reinterpret_cast<uintptr_t>(h_pinned) & 63u))
        return PXCL_E_INVAL;
    const EvLayout L = ev_layout(max_digis, ctx->n_modules);
    if (ws_bytes < L.total || pinned_bytes < HS_BYTES) return PXCL_E_CAPACITY;
    void* hdev = nullptr;
    if (hipHostGetDevicePointer(&hdev, h_pinned, 0) != hipSuccess || !hdev) {
        (void)hipGetLastError();
        return PXCL_E_INVAL;   // not pinned host memory
    }
    pxcl_event* ev = new pxcl_event();
    ev->ctx = ctx;
    ev->ws = static_cast<u8*>(d_ws);
    ev->ws_bytes = ws_bytes;
    ev->cap = max_digis;
    ev->hs = static_cast<u32*>(h_pinned);
    ev->hs_dev = static_cast<u32*>(hdev);
    std::memset(h_pinned, 0, HS_BYTES);
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipEventCreateWithFlags(&ev->done_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev->hits_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev->copy_ev, hipEventDisableTiming);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipEventCreate(&ev->hits_tev[i]);
    for (int i = 0; i < 5 && e == hipSuccess; ++i) e = hipEventCreate(&ev->tev[i]);
    if (e == hipSuccess) e = hipMemsetAsync(ev->ws + L.ctl, 0, CTL_WORDS * 4, s);
    if (e == hipSuccess) e = hipMemsetAsync(ev->ws + L.mtab, 0, size_t(16) * ctx->n_modules, s);
    if (e == hipSuccess) e = hipMemsetAsync(ev->ws + L.gcnt, 0, size_t(4) * ctx->n_modules, s);
    if (e == hipSuccess) e = hipMemsetAsync(ev->ws + L.hsum, 0, size_t(16) * max_digis, s);
    hipSetDevice(prev);
    if (e != hipSuccess) {
        if (ev->done_ev) hipEventDestroy(ev->done_ev);
        if (ev->hits_ev) hipEventDestroy(ev->hits_ev);
        if (ev->copy_ev) hipEventDestroy(ev->copy_ev);
        for (int i = 0; i < 2; ++i) if (ev->hits_tev[i]) hipEventDestroy(ev->hits_tev[i]);
        for (int i = 0; i < 5; ++i) if (ev->tev[i]) hipEventDestroy(ev->tev[i]);
        delete ev;
        return PXCL_E_HIP;
    }
    ctx->bound.fetch_add(1);
    *out = ev;
    return PXCL_OK;
}

extern "C" int pxcl_event_unbind(pxcl_event* ev) {
    if (!ev) return PXCL_E_INVAL;
    if (ev->state.load(std::memory_order_acquire) == ST_INFLIGHT) return PXCL_E_BUSY;
    if (ev->hstate.load(std::memory_order_acquire) == ST_INFLIGHT) return PXCL_E_BUSY;
    if (ev->cstate.load(std::memory_order_acquire) == ST_INFLIGHT) return PXCL_E_BUSY;
    auto pending = [ev]() {
        return ev->cb_pending.load(std::memory_order_acquire) > 0 ||
               ev->hits_pending.load(std::memory_order_acquire) > 0 ||
               ev->copy_pending.load(std::memory_order_acquire) > 0;
    };
    if (pending()) {
        if (t_in_callback) return PXCL_E_BUSY;                    // a callback of it is still running
        while (pending()) std::this_thread::yield();
    }
    hipEventDestroy(ev->done_ev);
    hipEventDestroy(ev->hits_ev);
    hipEventDestroy(ev->copy_ev);
    for (int i = 0; i < 2; ++i) hipEventDestroy(ev->hits_tev[i]);
    for (int i = 0; i < 5; ++i) hipEventDestroy(ev->tev[i]);
    ev->ctx->bound.fetch_sub(1);
    delete ev;
    return PXCL_OK;
}

extern "C" uint32_t pxcl_event_capacity(const pxcl_event* ev) { return ev ? ev->cap : 0; }

extern "C" int pxcl_acquire(pxcl_event* ev, const pxcl_digis* in, void* stream, pxcl_done_cb cb, void* user) {
    if (!ev || !digis_ok(in)) return PXCL_E_INVAL;
    if (in->n > ev->cap) return PXCL_E_CAPACITY;
    if (ev->hstate.load(std::memory_order_acquire) == ST_INFLIGHT) return PXCL_E_BUSY;   // hits read the slot
    if (ev->cstate.load(std::memory_order_acquire) == ST_INFLIGHT) return PXCL_E_BUSY;   // so does a copy
    if (!claim(ev->state)) return PXCL_E_BUSY;
    ev->hstate.store(ST_IDLE, std::memory_order_release);
    pxcl_ctx* ctx = ev->ctx;
    hipStream_t s = static_cast<hipStream_t>(stream);
    ev->epoch = next_epoch();
    ev->n = in->n;
    ev->cb = cb;
    ev->user = user;
    ev->stream = s;
    ev->batch = nullptr;
    ev->status = PXCL_OK;
    __atomic_store_n(&ev->hs[HS_EPOCH], 0u, __ATOMIC_RELEASE);
    const u32 wg = ctx->wg.load(), mpw = ctx->mpw.load();
    const int period = ctx->timing.load();
    const bool timed = period > 0 && (ev->launches++ % u32(period)) == 0;
    int prev = 0;
    hipGetDevice(&prev);
    if (prev != ctx->device) hipSetDevice(ctx->device);
    LaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.hdr = nullptr;
    a.ctr = reinterpret_cast<u32*>(ev->ws + ev_layout(ev->cap, ctx->n_modules).ctl) + CTL_CTR;
    a.n_modules = ctx->n_modules;
    a.charge_cut = ctx->charge_cut;
    a.dcap = cluster_capacity(wg, mpw);
    if (in->max_module_digis && in->max_module_digis <= a.dcap) a.flags |= LF_NO_BIG;
    if (in->max_module_digis && in->max_module_digis <= BIG_RCAP) a.flags |= LF_NO_SCRATCH;
    const bool any = (in->flags & PXCL_DIGIS_ANY_ORDER) != 0;
    // one event grouped by module: ranges by search, no segmentation kernel; in any
    // order: the grouping kernels build the module table instead
    a.flags |= any ? (LF_GROUP | LF_NO_SEG) : LF_FUSED;
    // deferred big-module kernels: only if the small kernel lists a module for them
    // does the completion thread queue them (and the compaction) in a second launch
    ev->defer = (in->flags & PXCL_DIGIS_DEFER_BIG) != 0;
    if (ev->defer) a.flags |= LF_NO_BIG | LF_NO_SCRATCH | LF_DEFER;
    hipError_t e = make_desc(ev, in, s, &a.single);
    ev->desc = a.single;
    const Grids g = grids_for(ctx, wg, mpw, in->n, in->n ? ctx->n_modules : 0u, 1, a.flags, false,
                              any ? in->n : 0u, any ? 1u : 0u);
    ev->defer_first = ev->defer;
    if (ev->defer) {
        ev->defer_args = a;
        ev->defer_args.flags &= ~(LF_NO_BIG | LF_NO_SCRATCH | LF_DEFER);
        ev->defer_grid_b = g.b;
        ev->defer_grid_x = g.x;
        ev->defer_grid_c = g.c;
    }
    if (e == hipSuccess) e = launch_all(a, g, wg, mpw, s, timed ? ev->tev : nullptr);
    if (e == hipSuccess) e = hipEventRecord(ev->done_ev, s);
    if (e == hipSuccess) {
        ev->cb_pending.fetch_add(1, std::memory_order_acq_rel);
        completer_post(ctx, CK_EVENT, ev, ev->done_ev);
    }
    if (e != hipSuccess) {
        // part of the launch may be queued: let it drain before the slot is released
        // (its kernels write the workspace; the next launch clears the control words)
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s);
        (void)hipGetLastError();
        ev->dirty = true;
        ev->state.store(ST_IDLE, std::memory_order_release);
        if (prev != ctx->device) hipSetDevice(prev);
        return PXCL_E_HIP;
    }
    if (prev != ctx->device) hipSetDevice(prev);
    ev->timed = timed;
    ev->timed_flags = a.flags;
    return PXCL_OK;
}

extern "C" int pxcl_query(const pxcl_event* ev) {
    if (!ev) return PXCL_E_INVAL;
    const int st = ev->state.load(std::memory_order_acquire);
    if (st == ST_DONE) return PXCL_OK;
    if (st == ST_INFLIGHT) return PXCL_E_NOT_READY;
    return PXCL_E_INVAL;
}

// flags: the launch's LF_* (a kernel not launched is not counted).  Launch order
// segment, small, big, compact; sums in the order segment, big, small, compact.
static void add_timing(pxcl_ctx* ctx, hipEvent_t* tev, u32 flags) {
    float ms[4];
    for (int i = 0; i < 4; ++i)
        if (hipEventElapsedTime(&ms[i], tev[i], tev[i + 1]) != hipSuccess) { (void)hipGetLastError(); return; }
    static const int slot[4] = {0, 2, 1, 3};
    std::lock_guard<std::mutex> g(ctx->tmu);
    for (int i = 0; i < 4; ++i) {
        if ((slot[i] == 1 && (flags & LF_NO_BIG)) || (slot[i] == 0 && (flags & LF_FUSED))) continue;
        if (slot[i] == 0 && (flags & LF_NO_SEG) && !(flags & LF_GROUP)) continue;
        ctx->tsum[slot[i]] += ms[i];
        ctx->tcnt[slot[i]] += 1;
    }
}

static void collect_timing(pxcl_event* ev) {
    if (!ev->timed) return;
    ev->timed = false;
    add_timing(ev->ctx, ev->tev, ev->timed_flags);
}

extern "C" int pxcl_produce(pxcl_event* ev, pxcl_clusters* out) {
    if (!ev || !out) return PXCL_E_INVAL;
    const int st = ev->state.load(std::memory_order_acquire);
    if (st == ST_INFLIGHT) return PXCL_E_NOT_READY;
    if (st != ST_DONE) return PXCL_E_INVAL;
    collect_timing(ev);
    const EvLayout L = ev_layout(ev->cap, ev->ctx->n_modules);
    out->status = ev->status;
    out->err_bits = ev->err_bits;
    out->n_clusters = ev->ncl;
    out->n_digis = ev->n;
    out->id = reinterpret_cast<const int32_t*>(ev->ws + L.id);
    out->charge = reinterpret_cast<const int32_t*>(ev->ws + L.charge);
    out->size = reinterpret_cast<const int32_t*>(ev->ws + L.size);
    out->digi_cluster = reinterpret_cast<const int32_t*>(ev->ws + L.digi);
    out->stream = ev->stream;
    out->done_event = ev->batch ? ev->batch->done_ev : ev->done_ev;
    out->device = ev->ctx->device;
    return ev->status;
}

extern "C" int pxcl_wait(pxcl_event* ev) {
    if (!ev) return PXCL_E_INVAL;
    int st = ev->state.load(std::memory_order_acquire);
    if (st == ST_IDLE) return PXCL_E_INVAL;
    if (st == ST_INFLIGHT) {
        hipEvent_t de = ev->batch ? ev->batch->done_ev : ev->done_ev;
        if (hipEventSynchronize(de) != hipSuccess) return PXCL_E_HIP;
        while (ev->state.load(std::memory_order_acquire) != ST_DONE) std::this_thread::yield();
    }
    // the completion callback has returned too (unless this is that callback)
    if (!t_in_callback)
        while (ev->cb_pending.load(std::memory_order_acquire) > 0) std::this_thread::yield();
    return PXCL_OK;
}

extern "C" void pxcl_flag_cb(void* user, int32_t status) {
    pxcl_flag* f = static_cast<pxcl_flag*>(user);
    if (!f) return;
    f->status = status;
    __atomic_fetch_add(&f->fired, 1u, __ATOMIC_RELEASE);
}

// ---------------------------------------------------------------------------
// allocation-free clustering of one event: pxcl_acquire's kernels over the device's
// fixed scratch array, with the caller's outputs; stream-ordered, no callback
// ---------------------------------------------------------------------------
extern "C" int pxcl_cluster_noalloc(pxcl_ctx* ctx, const pxcl_digis* in, const pxcl_noalloc_out* out,
                                    void* stream, uint32_t* tag) {
    if (!ctx || !digis_ok(in) || !out || !out->status) return PXCL_E_INVAL;
    if (in->where != PXCL_WHERE_DEVICE || in->flags) return PXCL_E_INVAL;
    if (in->n && (!out->digi_cluster || !out->id || !out->charge || !out->size)) return PXCL_E_INVAL;
    if (in->n > NOALLOC_CAP) return PXCL_E_CAPACITY;
    if (ctx->device < 0 || ctx->device >= NOALLOC_DEVICES) return PXCL_E_HIP;
    NoAllocDevice& d = g_noalloc[ctx->device];
    u8* ws = d.ptr;
    if (!ws) return PXCL_E_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const u32 wg = ctx->wg.load(), mpw = ctx->mpw.load();
    const EvLayout L = ev_layout(NOALLOC_CAP, ctx->n_modules);
    LaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.ctr = reinterpret_cast<u32*>(ws + L.ctl) + CTL_CTR;
    a.n_modules = ctx->n_modules;
    a.charge_cut = ctx->charge_cut;
    a.dcap = cluster_capacity(wg, mpw);
    if (in->max_module_digis && in->max_module_digis <= a.dcap) a.flags |= LF_NO_BIG;
    if (in->max_module_digis && in->max_module_digis <= BIG_RCAP) a.flags |= LF_NO_SCRATCH;
    a.flags |= LF_FUSED;
    EventDesc& E = a.single;
    E.module = in->module; E.row = in->row; E.col = in->col; E.adc = in->adc;
    E.ws = ws;
    E.hstat = out->status;
    E.o_digi = out->digi_cluster;
    E.o_id = out->id;
    E.o_charge = out->charge;
    E.o_size = out->size;
    E.n = in->n;
    E.cap = NOALLOC_CAP;
    E.epoch = next_epoch();
    E.slot = d.slot.fetch_add(1u, std::memory_order_relaxed) & 1u;
    int prev = 0;
    hipGetDevice(&prev);
    if (prev != ctx->device) hipSetDevice(ctx->device);
    hipError_t e = hipSuccess;
    if (d.dirty.exchange(false)) e = launch_fill(reinterpret_cast<u32*>(ws + L.ctl), CTL_WORDS, 0u, s);
    const Grids g = grids_for(ctx, wg, mpw, in->n, in->n ? ctx->n_modules : 0u, 1, a.flags, false);
    if (e == hipSuccess) e = launch_all(a, g, wg, mpw, s, nullptr);
    if (prev != ctx->device) hipSetDevice(prev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        d.dirty.store(true);
        return PXCL_E_HIP;
    }
    if (tag) *tag = E.epoch;
    return PXCL_OK;
}

// ---------------------------------------------------------------------------
// hits: a consumer of an event's clusters
// ---------------------------------------------------------------------------
namespace {
void hits_complete(void* p) {
    pxcl_event* ev = static_cast<pxcl_event*>(p);
    // the event's work completed before the hits (stream order or the wait on its
    // completion event), so its status block is final, whether or not the event's
    // own callback has run yet
    volatile u32* hs = ev->hs;
    const u32 tag = __atomic_load_n(&ev->hs[HS_EPOCH], __ATOMIC_ACQUIRE);
    u32 bits = hs[HS_ERR];
    if (tag != ev->epoch) bits |= EB_INTERNAL;
    const u32 ncl = hs[HS_NCL];
    ev->hits_n = ncl < ev->n ? ncl : ev->n;
    ev->hits_status = status_from_bits(bits);
    pxcl_done_cb cb = ev->hits_cb;
    void* user = ev->hits_user;
    const int32_t st = ev->hits_status;
    ev->hstate.store(ST_DONE, std::memory_order_release);
    if (cb) {
        ++t_in_callback;
        cb(user, st);
        --t_in_callback;
    }
    ev->hits_pending.fetch_sub(1, std::memory_order_acq_rel);
}
}  // namespace

// add the hits kernel time of the last timed hits launch (complete by now)
static void collect_hits_timing(pxcl_event* ev) {
    if (!ev->hits_timed) return;
    ev->hits_timed = false;
    float ms = 0;
    if (hipEventElapsedTime(&ms, ev->hits_tev[0], ev->hits_tev[1]) != hipSuccess) { (void)hipGetLastError(); return; }
    std::lock_guard<std::mutex> g(ev->ctx->tmu);
    ev->ctx->tsum[4] += ms;
    ev->ctx->tcnt[4] += 1;
}

extern "C" int pxcl_hits_enqueue(pxcl_event* ev, void* stream, pxcl_done_cb cb, void* user) {
    if (!ev) return PXCL_E_INVAL;
    const int st = ev->state.load(std::memory_order_acquire);
    if (st == ST_IDLE) return PXCL_E_INVAL;                     // no event acquired
    if (st == ST_INFLIGHT && ev->defer) return PXCL_E_BUSY;      // its results are final only at the callback
    if (!claim(ev->hstate)) return PXCL_E_BUSY;
    pxcl_ctx* ctx = ev->ctx;
    collect_hits_timing(ev);                                    // the previous hits are complete
    const int period = ctx->timing.load();
    const bool timed = period > 0 && (ev->hits_launches++ % u32(period)) == 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int prev = 0;
    hipGetDevice(&prev);
    if (prev != ctx->device) hipSetDevice(ctx->device);
    hipError_t e = hipSuccess;
    // a consumer on another stream waits for the clusters if they may not be ready
    if (st == ST_INFLIGHT && s != ev->stream)
        e = hipStreamWaitEvent(s, ev->batch ? ev->batch->done_ev : ev->done_ev, 0);
    ev->hits_cb = cb;
    ev->hits_user = user;
    ev->hits_stream = s;
    ev->hits_status = PXCL_OK;
    ev->hits_n = 0;
    const bool fused = (ev->desc.flags & EF_HITS) != 0;   // computed with the clusters
    if (!fused) {
        LaunchArgs a;
        std::memset(&a, 0, sizeof(a));
        a.single = ev->desc;
        a.n_modules = ctx->n_modules;
        a.charge_cut = ctx->charge_cut;
        const u32 grid = u32(std::max<u64>(1, std::min<u64>((u64)ctx->n_cu * ctx->occ_h, ctx->n_modules)));
        if (e == hipSuccess && timed) e = hipEventRecord(ev->hits_tev[0], s);
        if (e == hipSuccess) e = launch_hits(a, grid, s);
        if (e == hipSuccess && timed) e = hipEventRecord(ev->hits_tev[1], s);
    }
    // fused hits asked for on the event's own stream are complete with the event: its
    // completion event serves, no event is recorded
    ev->hits_done = (fused && s == ev->stream) ? (ev->batch ? ev->batch->done_ev : ev->done_ev) : ev->hits_ev;
    if (e == hipSuccess && ev->hits_done == ev->hits_ev) e = hipEventRecord(ev->hits_ev, s);
    if (e == hipSuccess) {
        ev->hits_pending.fetch_add(1, std::memory_order_acq_rel);
        completer_post(ctx, CK_HITS, ev, ev->hits_done);
    }
    if (prev != ctx->device) hipSetDevice(prev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ev->hstate.store(ST_IDLE, std::memory_order_release);
        return PXCL_E_HIP;
    }
    ev->hits_timed = timed && !fused;
    return PXCL_OK;
}

extern "C" int pxcl_hits_query(const pxcl_event* ev) {
    if (!ev) return PXCL_E_INVAL;
    const int st = ev->hstate.load(std::memory_order_acquire);
    if (st == ST_DONE) return PXCL_OK;
    if (st == ST_INFLIGHT) return PXCL_E_NOT_READY;
    return PXCL_E_INVAL;
}

extern "C" int pxcl_hits_produce(pxcl_event* ev, pxcl_hits* out) {
    if (!ev || !out) return PXCL_E_INVAL;
    const int st = ev->hstate.load(std::memory_order_acquire);
    if (st == ST_INFLIGHT) return PXCL_E_NOT_READY;
    if (st != ST_DONE) return PXCL_E_INVAL;
    collect_hits_timing(ev);
    const EvLayout L = ev_layout(ev->cap, ev->ctx->n_modules);
    out->status = ev->hits_status;
    out->n_hits = ev->hits_status == PXCL_OK ? ev->hits_n : 0u;
    out->x = reinterpret_cast<const float*>(ev->ws + L.hit_x);
    out->y = reinterpret_cast<const float*>(ev->ws + L.hit_y);
    out->stream = ev->hits_stream;
    out->done_event = ev->hits_done;
    out->device = ev->ctx->device;
    return ev->hits_status;
}

// ---------------------------------------------------------------------------
// copy to host on demand
// ---------------------------------------------------------------------------
namespace {
void copy_complete(void* p) {
    pxcl_event* ev = static_cast<pxcl_event*>(p);
    volatile u32* hs = ev->hs;
    const u32 tag = __atomic_load_n(&ev->hs[HS_EPOCH], __ATOMIC_ACQUIRE);
    u32 bits = hs[HS_ERR];
    if (tag != ev->epoch) bits |= EB_INTERNAL;
    const u32 ncl = hs[HS_NCL];
    pxcl_host_clusters* d = ev->copy_dst;
    d->status = status_from_bits(bits);
    d->n_clusters = d->status == PXCL_OK ? (ncl < ev->n ? ncl : ev->n) : 0u;
    pxcl_done_cb cb = ev->copy_cb;
    void* user = ev->copy_user;
    const int32_t st = d->status;
    ev->cstate.store(ST_DONE, std::memory_order_release);
    if (cb) {
        ++t_in_callback;
        cb(user, st);
        --t_in_callback;
    }
    ev->copy_pending.fetch_sub(1, std::memory_order_acq_rel);
}
}  // namespace

// The completion thread: takes posted launches, queries their completion events
// and runs the completion step of each one that has completed (an event that
// reports an error counts as completed: the status block then shows the missing
// write-back).  It sleeps while nothing is in flight and yields between passes.
static void completer_loop(pxcl_completer* c, int device) {
    hipSetDevice(device);
    std::vector<Pending> mine;
    for (;;) {
        if (mine.empty() || c->has_in.load(std::memory_order_acquire)) {
            std::unique_lock<std::mutex> lk(c->mu);
            if (mine.empty() && c->in.empty()) {
                if (c->stop) return;
                c->idle = true;
                c->cv.wait(lk, [c] { return c->stop || !c->in.empty(); });
                c->idle = false;
                if (c->in.empty()) return;
            }
            mine.insert(mine.end(), c->in.begin(), c->in.end());
            c->in.clear();
            c->has_in.store(false, std::memory_order_relaxed);
        }
        bool any = false;
        for (size_t i = 0; i < mine.size();) {
            const hipError_t q = hipEventQuery(mine[i].done);
            if (q == hipErrorNotReady) { ++i; continue; }
            if (q != hipSuccess) (void)hipGetLastError();
            // hits and copies read an event's results: their completion follows the
            // event's own (whose work has finished too, by stream order or the wait
            // on its completion event, so it is processed in this pass or the next)
            if ((mine[i].kind == CK_HITS || mine[i].kind == CK_COPY) &&
                static_cast<pxcl_event*>(mine[i].obj)->state.load(std::memory_order_acquire) == ST_INFLIGHT) {
                ++i;
                continue;
            }
            const Pending p = mine[i];
            mine[i] = mine.back();
            mine.pop_back();
            switch (p.kind) {
                case CK_EVENT:
                    if (!event_complete(p.obj)) mine.push_back(p);   // its second launch
                    break;
                case CK_BATCH:
                    if (!batch_complete(p.obj)) mine.push_back(p);   // its second launch
                    break;
                case CK_HITS: hits_complete(p.obj); break;
                default: copy_complete(p.obj); break;
            }
            any = true;
        }
        if (!any) std::this_thread::yield();
    }
}

extern "C" int pxcl_copy_to_host(pxcl_event* ev, void* stream, pxcl_host_clusters* dst, pxcl_done_cb cb,
                                 void* user) {
    if (!ev || !dst || !dst->id || !dst->charge || !dst->size) return PXCL_E_INVAL;
    const int st = ev->state.load(std::memory_order_acquire);
    if (st == ST_IDLE) return PXCL_E_INVAL;
    if (st == ST_INFLIGHT && ev->defer) return PXCL_E_BUSY;     // its results are final only at the callback
    const bool want_hits = dst->x || dst->y;
    const int hst = ev->hstate.load(std::memory_order_acquire);
    if (want_hits && (!dst->x || !dst->y || hst == ST_IDLE)) return PXCL_E_INVAL;   // no hits queued
    // clusters to copy: exact once the event is complete, else the bound n
    const u32 ncl = (st == ST_DONE) ? ev->ncl : ev->n;
    if (dst->capacity < ncl) return PXCL_E_CAPACITY;
    if (!claim(ev->cstate)) return PXCL_E_BUSY;
    pxcl_ctx* ctx = ev->ctx;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int prev = 0;
    hipGetDevice(&prev);
    if (prev != ctx->device) hipSetDevice(ctx->device);
    hipError_t e = hipSuccess;
    if (st == ST_INFLIGHT && s != ev->stream)
        e = hipStreamWaitEvent(s, ev->batch ? ev->batch->done_ev : ev->done_ev, 0);
    if (e == hipSuccess && want_hits && hst == ST_INFLIGHT && s != ev->hits_stream)
        e = hipStreamWaitEvent(s, ev->hits_done, 0);
    ev->copy_dst = dst;
    ev->copy_cb = cb;
    ev->copy_user = user;
    dst->n_clusters = 0;
    dst->status = PXCL_E_NOT_READY;
    const EvLayout L = ev_layout(ev->cap, ctx->n_modules);
    auto d2h = [&](void* to, size_t off, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(to, ev->ws + off, bytes, hipMemcpyDeviceToHost, s);
    };
    d2h(dst->id, L.id, size_t(ncl) * 4);
    d2h(dst->charge, L.charge, size_t(ncl) * 4);
    d2h(dst->size, L.size, size_t(ncl) * 4);
    if (dst->digi_cluster) d2h(dst->digi_cluster, L.digi, size_t(ev->n) * 4);
    if (want_hits) {
        d2h(dst->x, L.hit_x, size_t(ncl) * 4);
        d2h(dst->y, L.hit_y, size_t(ncl) * 4);
    }
    if (e == hipSuccess) e = hipEventRecord(ev->copy_ev, s);
    if (e == hipSuccess) {
        ev->copy_pending.fetch_add(1, std::memory_order_acq_rel);
        completer_post(ctx, CK_COPY, ev, ev->copy_ev);
    }
    if (prev != ctx->device) hipSetDevice(prev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ev->cstate.store(ST_IDLE, std::memory_order_release);
        return PXCL_E_HIP;
    }
    return PXCL_OK;
}

extern "C" int pxcl_copy_query(const pxcl_event* ev) {
    if (!ev) return PXCL_E_INVAL;
    const int st = ev->cstate.load(std::memory_order_acquire);
    if (st == ST_DONE) return PXCL_OK;
    if (st == ST_INFLIGHT) return PXCL_E_NOT_READY;
    return PXCL_E_INVAL;
}

extern "C" int pxcl_hits_wait(pxcl_event* ev) {
    if (!ev) return PXCL_E_INVAL;
    const int st = ev->hstate.load(std::memory_order_acquire);
    if (st == ST_IDLE) return PXCL_E_INVAL;
    if (st == ST_INFLIGHT) {
        if (hipEventSynchronize(ev->hits_done) != hipSuccess) return PXCL_E_HIP;
        while (ev->hstate.load(std::memory_order_acquire) != ST_DONE) std::this_thread::yield();
    }
    if (!t_in_callback)
        while (ev->hits_pending.load(std::memory_order_acquire) > 0) std::this_thread::yield();
    return PXCL_OK;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
extern "C" size_t pxcl_batch_workspace_bytes(const pxcl_ctx* ctx, uint32_t max_events) {
    if (!ctx || max_events == 0 || max_events > MAXB) return 0;
    return batch_ws_bytes(max_events);
}

extern "C" size_t pxcl_batch_pinned_bytes(const pxcl_ctx* ctx, uint32_t max_events) {
    if (!ctx || max_events == 0 || max_events > MAXB) return 0;
    return al256(header_bytes(max_events));
}

extern "C" int pxcl_batch_bind(pxcl_ctx* ctx, void* d_ws, size_t ws_bytes, void* h_pinned, size_t pinned_bytes,
                               uint32_t max_events, void* stream, pxcl_batch** out) {
    if (!ctx || !d_ws || !h_pinned || !out || max_events == 0 || max_events > MAXB) return PXCL_E_INVAL;
    if ((reinterpret_cast<uintptr_t>(d_ws) & 255u) || (reinterpret_cast<uintptr_t>(h_pinned) & 63u))
        return PXCL_E_INVAL;
    if (ws_bytes < batch_ws_bytes(max_events) || pinned_bytes < header_bytes(max_events)) return PXCL_E_CAPACITY;
    pxcl_batch* b = new pxcl_batch();
    b->ctx = ctx;
    b->ws = static_cast<u8*>(d_ws);
    b->ws_bytes = ws_bytes;
    b->hp = static_cast<u8*>(h_pinned);
    b->max_events = max_events;
    std::memset(h_pinned, 0, header_bytes(max_events));
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(ctx->device);
    hipError_t e = hipEventCreateWithFlags(&b->done_ev, hipEventDisableTiming);
    for (int i = 0; i < 5 && e == hipSuccess; ++i) e = hipEventCreate(&b->tev[i]);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMemsetAsync(b->ws, 0, BW_HDR, static_cast<hipStream_t>(stream));
    hipSetDevice(prev);
    if (e != hipSuccess) {
        if (b->done_ev) hipEventDestroy(b->done_ev);
        for (int i = 0; i < 5; ++i) if (b->tev[i]) hipEventDestroy(b->tev[i]);
        if (b->cap_stream) hipStreamDestroy(b->cap_stream);
        delete b;
        return PXCL_E_HIP;
    }
    ctx->bound.fetch_add(1);
    *out = b;
    return PXCL_OK;
}

static void drop_graphs(pxcl_batch* b) {
    for (int i = 0; i < pxcl_batch::N_GRAPHS; ++i) {
        if (b->gexec[i]) hipGraphExecDestroy(b->gexec[i]);
        if (b->graph[i]) hipGraphDestroy(b->graph[i]);
        b->gexec[i] = nullptr;
        b->graph[i] = nullptr;
    }
}

static u32 graph_slot(u32 flags) {
    return ((flags & LF_NO_BIG) ? 1u : 0u) | ((flags & LF_SEG_WIDE) ? 2u : 0u) | ((flags & LF_NO_SCRATCH) ? 4u : 0u) |
           ((flags & LF_GROUP) ? 8u : 0u) | ((flags & LF_NO_SEG) ? 16u : 0u) | ((flags & LF_DEFER) ? 32u : 0u);
}

extern "C" int pxcl_batch_unbind(pxcl_batch* b) {
    if (!b) return PXCL_E_INVAL;
    if (b->state.load(std::memory_order_acquire) == ST_INFLIGHT) return PXCL_E_BUSY;
    if (b->timed) { b->timed = false; add_timing(b->ctx, b->tev, b->timed_flags); }
    drop_graphs(b);
    hipEventDestroy(b->done_ev);
    for (int i = 0; i < 5; ++i) hipEventDestroy(b->tev[i]);
    hipStreamDestroy(b->cap_stream);
    b->ctx->bound.fetch_sub(1);
    delete b;
    return PXCL_OK;
}

static LaunchArgs batch_args(pxcl_batch* b, u32 wg, u32 mpw) {
    LaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.hdr = reinterpret_cast<const u32*>(b->ws + BW_HDR);
    a.ctr = reinterpret_cast<u32*>(b->ws + BW_CTR);
    a.n_modules = b->ctx->n_modules;
    a.charge_cut = b->ctx->charge_cut;
    a.dcap = cluster_capacity(wg, mpw);
    return a;
}

// Capture the per-batch pipeline (header copy + kernels, full grids) once per kernel
// configuration and flag combination, so that launches whose flags alternate reuse
// their graphs; replays read k and the event descriptors from the header.
static hipError_t ensure_graph(pxcl_batch* b, u32 wg, u32 mpw, u32 flags, hipGraphExec_t* out) {
    if (b->g_wg != wg || b->g_mpw != mpw) {
        drop_graphs(b);
        b->g_wg = wg;
        b->g_mpw = mpw;
    }
    const u32 gs = graph_slot(flags);
    *out = b->gexec[gs];
    if (*out) return hipSuccess;
    pxcl_ctx* ctx = b->ctx;
    LaunchArgs a = batch_args(b, wg, mpw);
    a.flags = flags;
    const Grids g = grids_for(ctx, wg, mpw, 0, 0, 0, flags, true);
    hipStream_t cs = b->cap_stream;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t e2 = hipMemcpyAsync(b->ws + BW_HDR, b->hp, header_bytes(b->max_events), hipMemcpyHostToDevice, cs);
    if (e2 == hipSuccess) e2 = launch_all(a, g, wg, mpw, cs, nullptr);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    if (e2 != hipSuccess) { if (graph) hipGraphDestroy(graph); return e2; }
    if (e != hipSuccess) return e;
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) { hipGraphDestroy(graph); return e; }
    b->graph[gs] = graph;
    b->gexec[gs] = *out = exec;
    return hipSuccess;
}

extern "C" int pxcl_acquire_batch(pxcl_batch* b, pxcl_event* const* evs, const pxcl_digis* ins, uint32_t k,
                                  void* stream, pxcl_done_cb cb, void* user, uint32_t flags) {
    if (!b || !evs || !ins || k == 0) return PXCL_E_INVAL;
    if (k > b->max_events) return PXCL_E_CAPACITY;
    for (u32 i = 0; i < k; ++i) {
        if (!evs[i] || evs[i]->ctx != b->ctx || !digis_ok(&ins[i])) return PXCL_E_INVAL;
        if (ins[i].flags & PXCL_DIGIS_DEFER_BIG) return PXCL_E_INVAL;   // single-event launches only
        if (ins[i].n > evs[i]->cap) return PXCL_E_CAPACITY;
        if (evs[i]->hstate.load(std::memory_order_acquire) == ST_INFLIGHT) return PXCL_E_BUSY;
        if (evs[i]->cstate.load(std::memory_order_acquire) == ST_INFLIGHT) return PXCL_E_BUSY;
        for (u32 j = 0; j < i; ++j)
            if (evs[j] == evs[i]) return PXCL_E_INVAL;
    }
    if (!claim(b->state)) return PXCL_E_BUSY;
    u32 got = 0;
    for (; got < k; ++got)
        if (!claim(evs[got]->state)) break;
    if (got < k) {
        for (u32 i = 0; i < got; ++i) evs[i]->state.store(ST_IDLE, std::memory_order_release);
        b->state.store(ST_IDLE, std::memory_order_release);
        return PXCL_E_BUSY;
    }
    pxcl_ctx* ctx = b->ctx;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int prev = 0;
    hipGetDevice(&prev);
    if (prev != ctx->device) hipSetDevice(ctx->device);
    const u32 wg = ctx->wg.load(), mpw = ctx->mpw.load();
    if (b->timed) { b->timed = false; add_timing(ctx, b->tev, b->timed_flags); }   // the previous launch is complete
    // graph replays are never timed (elapsed times of events recorded inside a captured
    // graph are not available); plain launches are sampled every `period` launches
    const int period = ctx->timing.load();
    const bool timed = !(flags & PXCL_BATCH_GRAPH) && period > 0 && (b->launches++ % u32(period)) == 0;
    b->k = k;
    b->cb = cb;
    b->user = user;
    b->status = PXCL_OK;
    *reinterpret_cast<u32*>(b->hp) = k;
    EventDesc* hd = reinterpret_cast<EventDesc*>(b->hp + HDR_EV_OFFSET);
    hipError_t e = hipSuccess;
    u64 digis = 0, present = 0, sorted_digis = 0, any_digis = 0;
    u32 any_events = 0;
    const u32 dcap = cluster_capacity(wg, mpw);
    u32 lflags = LF_NO_BIG | LF_NO_SCRATCH;     // unless an event may hold a big module
    for (u32 i = 0; i < k && e == hipSuccess; ++i) {
        pxcl_event* ev = evs[i];
        b->evs[i] = ev;
        if (!ins[i].max_module_digis || ins[i].max_module_digis > dcap) lflags &= ~LF_NO_BIG;
        if (!ins[i].max_module_digis || ins[i].max_module_digis > BIG_RCAP) lflags &= ~LF_NO_SCRATCH;
        ev->epoch = next_epoch();
        ev->n = ins[i].n;
        ev->cb = nullptr;
        ev->user = nullptr;
        ev->stream = s;
        ev->batch = b;
        ev->timed = false;
        ev->defer = (flags & PXCL_BATCH_DEFER_BIG) != 0;       // results final at the callback
        ev->defer_first = false;
        ev->status = PXCL_OK;
        __atomic_store_n(&ev->hs[HS_EPOCH], 0u, __ATOMIC_RELEASE);
        ev->hstate.store(ST_IDLE, std::memory_order_release);
        e = make_desc(ev, &ins[i], s, &hd[i]);
        ev->desc = hd[i];
        digis += ins[i].n;
        present += std::min<u64>(ins[i].n, (u64)ctx->n_modules);
        if (ins[i].flags & PXCL_DIGIS_ANY_ORDER) {
            any_digis += ins[i].n;
            ++any_events;
        } else {
            sorted_digis += ins[i].n;
        }
    }
    if (any_events) lflags |= LF_GROUP;
    if (any_events == k) lflags |= LF_NO_SEG;
    // a captured graph replays with any input: its segmentation always takes wide
    // chunks (correct for any size), so batches of varying size share one graph
    lflags |= (flags & PXCL_BATCH_GRAPH) ? LF_SEG_WIDE : seg_flag(ctx, sorted_digis);
    // deferred big-module kernels: a second launch (big-module kernels, compaction of
    // the events the first one left) only if some event lists a module for them
    b->defer_first = (flags & PXCL_BATCH_DEFER_BIG) != 0;
    if (b->defer_first) lflags |= LF_NO_BIG | LF_NO_SCRATCH | LF_DEFER;
    b->stream = s;
    if (e == hipSuccess) {
        const bool graph = (flags & PXCL_BATCH_GRAPH) != 0;
        const Grids g = graph ? grids_for(ctx, wg, mpw, 0, 0, 0, lflags, true)
                              : grids_for(ctx, wg, mpw, digis, present, k, lflags, false, any_digis, any_events);
        if (b->defer_first) {
            b->defer_args = batch_args(b, wg, mpw);
            b->defer_args.flags = (lflags & ~(LF_NO_BIG | LF_NO_SCRATCH | LF_DEFER)) | LF_SECOND;
            b->defer_grid_b = g.b;
            b->defer_grid_x = g.x;
            b->defer_grid_c = g.c;
        }
        if (graph) {
            hipGraphExec_t exec = nullptr;
            e = ensure_graph(b, wg, mpw, lflags, &exec);
            if (e == hipSuccess) e = hipGraphLaunch(exec, s);
        } else {
            LaunchArgs a = batch_args(b, wg, mpw);
            a.flags = lflags;
            e = hipMemcpyAsync(b->ws + BW_HDR, b->hp, header_bytes(k), hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = launch_all(a, g, wg, mpw, s, timed ? b->tev : nullptr);
        }
    }
    if (e == hipSuccess) e = hipEventRecord(b->done_ev, s);
    if (e == hipSuccess) {
        for (u32 i = 0; i < k; ++i) evs[i]->cb_pending.fetch_add(1, std::memory_order_acq_rel);
        completer_post(ctx, CK_BATCH, b, b->done_ev);
    }
    if (e != hipSuccess) {
        // part of the launch may be queued: let it drain before the batch and its
        // events are released (the segmentation kernel of the next launch resets the
        // batch's ticket counter; the events' control words are cleared then too)
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s);
        (void)hipGetLastError();
        for (u32 i = 0; i < k; ++i) {
            evs[i]->dirty = true;
            evs[i]->state.store(ST_IDLE, std::memory_order_release);
        }
        b->state.store(ST_IDLE, std::memory_order_release);
        if (prev != ctx->device) hipSetDevice(prev);
        return PXCL_E_HIP;
    }
    if (prev != ctx->device) hipSetDevice(prev);
    b->timed = timed;
    b->timed_flags = lflags;
    return PXCL_OK;
}

extern "C" int pxcl_batch_query(const pxcl_batch* b) {
    if (!b) return PXCL_E_INVAL;
    const int st = b->state.load(std::memory_order_acquire);
    if (st == ST_DONE) return PXCL_OK;
    if (st == ST_INFLIGHT) return PXCL_E_NOT_READY;
    return PXCL_E_INVAL;
}

// ---------------------------------------------------------------------------
// misc
// ---------------------------------------------------------------------------
extern "C" const char* pxcl_strerror(int code) {
    switch (code) {
        case PXCL_OK: return "ok";
        case PXCL_E_INVAL: return "invalid argument";
        case PXCL_E_CAPACITY: return "capacity exceeded";
        case PXCL_E_BUSY: return "work in flight";
        case PXCL_E_NOT_READY: return "not ready";
        case PXCL_E_DUP_PIXEL: return "pixel fired twice in a module";
        case PXCL_E_RANGE: return "module, row or column out of range";
        case PXCL_E_ORDER: return "digis not grouped by ascending module";
        case PXCL_E_HIP: return "HIP runtime error";
        case PXCL_E_INTERNAL: return "internal error (inconsistent device state or missing status write-back)";
        case PXCL_E_NOTFOUND: return "not found";
        case PXCL_E_HINT: return "a module has more digis than the size hint";
        default: return "unknown error";
    }
}

extern "C" const char* pxcl_version(void) { return "pxcl 0.1 gfx950"; }

// internal accessors for the drivers and the autotuner
namespace pxcl {
u32 event_n(const pxcl_event* ev) { return ev->n; }
hipEvent_t batch_done_event(const pxcl_batch* b) { return b->done_ev; }
const std::string& ctx_arch(const pxcl_ctx* c) { return c->arch; }
int ctx_device(const pxcl_ctx* c) { return c->device; }
// Restrict the context's completion thread to `cpus` (a cpu_set_t), or to every CPU of
// the process's affinity set with nullptr.
void ctx_place_completer(pxcl_ctx* c, const void* cpus) {
    cpu_set_t all;
    if (!cpus) {
        CPU_ZERO(&all);
        if (sched_getaffinity(0, sizeof(all), &all) != 0) return;
        cpus = &all;
    }
    if (c->comp.th.joinable())
        (void)pthread_setaffinity_np(c->comp.th.native_handle(), sizeof(cpu_set_t), static_cast<const cpu_set_t*>(cpus));
}
}  // namespace pxcl


