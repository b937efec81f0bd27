// Drivers around the acquire/produce boundary: the asynchronous form (host threads
// keep doing CPU work while their event is on the device), the serving form
// (Poisson arrivals, admission under a device-memory budget, continuous batching)
// and the autotuner of the clustering kernel's shape.
//
// The asynchronous form is the External Worker pattern of the paper (Sec. 2): the
// thread that called acquire() does not wait; the completion callback releases the
// produce() step, which a thread picks up between other tasks.  The serving form's
// memory handling follows Sec. 4.1: workspaces are carved out of one arena that the
// caller allocated once (the role of the caching allocator), sized per event rather
// than for the largest possible event.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <fstream>
#include <map>
#include <mutex>
#include <random>
#include <sstream>
#include <string>
#include <pthread.h>
#include <sched.h>
#include <sys/prctl.h>
#include <sys/resource.h>
#include <sys/syscall.h>
#include <unistd.h>
#include <thread>
#include <vector>

#include "../../include/pxcl.h"
#include "pxcl_internal.h"

namespace pxcl {
bool cluster_config_valid(u32 wg, u32 mpw);
const std::string& ctx_arch(const pxcl_ctx* c);
int ctx_device(const pxcl_ctx* c);
void ctx_place_completer(pxcl_ctx* c, const void* cpus);
}  // namespace pxcl

using namespace pxcl;
using clk = std::chrono::steady_clock;

namespace {

inline double us_since(clk::time_point t0, clk::time_point t1) {
    return std::chrono::duration<double, std::micro>(t1 - t0).count();
}

// Synthetic CPU task: an integer hash loop that runs for `ns` nanoseconds.
u64 cpu_task(u32 ns, u64 seed) {
    const auto t0 = clk::now();
    u64 x = seed | 1u;
    for (;;) {
        for (int i = 0; i < 256; ++i) {
            x ^= x >> 31; x *= 0x7fb5d329728ea185ull; x ^= x >> 27; x *= 0x81dadef4bc2dd44dull;
        }
        if (std::chrono::duration_cast<std::chrono::nanoseconds>(clk::now() - t0).count() >= (long long)ns) break;
    }
    return x;
}

double percentile(std::vector<double>& v, double p) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = p * double(v.size() - 1);
    const size_t lo = size_t(std::floor(pos)), hi = std::min(v.size() - 1, lo + 1);
    const double f = pos - double(lo);
    return v[lo] * (1.0 - f) + v[hi] * f;
}

std::atomic<u64> g_sink{0};   // keeps the CPU tasks' results alive

// CPU worker threads of the serving form run at a lower priority (nice 10) than the
// dispatcher and the completion thread: with as many busy workers as cores, those two
// would otherwise wait for whole scheduler time slices (milliseconds).  Raising a
// thread's niceness needs no privileges.
void lower_priority() { (void)setpriority(PRIO_PROCESS, id_t(syscall(SYS_gettid)), 10); }

// Cores of the serving form: with at least four CPUs in the process's affinity set,
// the dispatcher (the calling thread) keeps the last one to itself, the context's
// completion thread the one before, and the CPU threads stay off both, so that the
// dispatcher, the completion thread and the runtime's own threads never wait behind
// busy CPU threads for a time slice; the CPU threads share the other cores (with as
// many threads as cores the synthetic work is bound by the cores anyway).
struct CorePlan {
    bool on = false;
    cpu_set_t all, workers, dispatcher, completer;
};
CorePlan plan_cores() {
    CorePlan p;
    CPU_ZERO(&p.all);
    if (sched_getaffinity(0, sizeof(p.all), &p.all) != 0) return p;
    std::vector<int> cpus;
    for (int c = 0; c < CPU_SETSIZE; ++c)
        if (CPU_ISSET(c, &p.all)) cpus.push_back(c);
    if (cpus.size() < 4) return p;
    CPU_ZERO(&p.workers);
    CPU_ZERO(&p.dispatcher);
    CPU_ZERO(&p.completer);
    for (size_t i = 0; i + 2 < cpus.size(); ++i) CPU_SET(cpus[i], &p.workers);
    CPU_SET(cpus.back(), &p.dispatcher);
    CPU_SET(cpus[cpus.size() - 2], &p.completer);
    p.on = true;
    return p;
}
void place_worker(const CorePlan& p) {
    if (p.on) (void)pthread_setaffinity_np(pthread_self(), sizeof(cpu_set_t), &p.workers);
    lower_priority();
}

}  // namespace

// ---------------------------------------------------------------------------
// asynchronous form
// ---------------------------------------------------------------------------
extern "C" int pxcl_run_async(pxcl_ctx* ctx, pxcl_event* const* evs, void* const* streams, uint32_t n_threads,
                              const pxcl_digis* pool, uint32_t pool_size, uint32_t events_per_thread,
                              uint32_t cpu_task_ns, int flags, pxcl_run_stats* out, void* d_results,
                              const uint64_t* result_offsets) {
    const bool blocking = (flags & PXCL_RUN_BLOCKING) != 0, with_hits = (flags & PXCL_RUN_HITS) != 0;
    if (!ctx || !evs || !streams || !pool || !out || n_threads == 0 || pool_size == 0) return PXCL_E_INVAL;
    std::vector<std::vector<double>> lat(n_threads);
    std::vector<double> blocked(n_threads, 0.0);
    std::vector<u64> tasks(n_threads, 0), digis(n_threads, 0);
    std::vector<u32> errors(n_threads, 0);
    std::atomic<int> rc{PXCL_OK};
    std::atomic<u32> ready{0};
    std::atomic<bool> go{false};
    std::atomic<u32> inflight{0}, max_inflight{0};
    const int dev = ctx_device(ctx);

    auto worker = [&](u32 t) {
        hipSetDevice(dev);
        lat[t].reserve(events_per_thread);
        ready.fetch_add(1);
        while (!go.load(std::memory_order_acquire)) std::this_thread::yield();
        for (u32 i = 0; i < events_per_thread && rc.load() == PXCL_OK; ++i) {
            const pxcl_digis& in = pool[(t + u64(i) * n_threads) % pool_size];
            pxcl_flag flag, hflag;
            flag.status = 0;
            flag.fired = 0;
            hflag.status = 0;
            hflag.fired = 0;
            const auto t0 = clk::now();
            int r = pxcl_acquire(evs[t], &in, streams[t], pxcl_flag_cb, &flag);
            if (r == PXCL_OK && with_hits) r = pxcl_hits_enqueue(evs[t], streams[t], pxcl_flag_cb, &hflag);
            const auto t1 = clk::now();
            blocked[t] += us_since(t0, t1);
            if (r != PXCL_OK) { rc.store(r); break; }
            // the hits' callback comes after the event's (stream order)
            pxcl_flag& last = with_hits ? hflag : flag;
            const u32 now_in = inflight.fetch_add(1) + 1;
            u32 m = max_inflight.load();
            while (now_in > m && !max_inflight.compare_exchange_weak(m, now_in)) {}
            if (blocking) {
                const auto w0 = clk::now();
                hipStreamSynchronize(static_cast<hipStream_t>(streams[t]));
                while (__atomic_load_n(&last.fired, __ATOMIC_ACQUIRE) == 0) std::this_thread::yield();
                blocked[t] += us_since(w0, clk::now());
            } else {
                while (__atomic_load_n(&last.fired, __ATOMIC_ACQUIRE) == 0) {
                    if (cpu_task_ns) {
                        g_sink.fetch_add(cpu_task(cpu_task_ns, tasks[t] + t), std::memory_order_relaxed);
                        ++tasks[t];
                    } else {
                        std::this_thread::yield();
                    }
                }
            }
            inflight.fetch_sub(1);
            pxcl_clusters res;
            const auto p0 = clk::now();
            r = pxcl_produce(evs[t], &res);
            if (r == PXCL_OK && with_hits) {
                pxcl_hits hits;
                r = pxcl_hits_produce(evs[t], &hits);
            }
            const auto p1 = clk::now();
            blocked[t] += us_since(p0, p1);
            if (d_results && result_offsets && r == PXCL_OK) {   // verification mode: copy out, then reuse
                u8* dst = static_cast<u8*>(d_results) + result_offsets[t + u64(i) * n_threads];
                const size_t nb = size_t(res.n_digis) * 4, cb = size_t(res.n_clusters) * 4;
                hipStream_t rs = static_cast<hipStream_t>(res.stream);
                hipError_t ce = hipSuccess;
                if (nb) ce = hipMemcpyAsync(dst, res.digi_cluster, nb, hipMemcpyDeviceToDevice, rs);
                if (cb && ce == hipSuccess) ce = hipMemcpyAsync(dst + nb, res.id, cb, hipMemcpyDeviceToDevice, rs);
                if (cb && ce == hipSuccess) ce = hipMemcpyAsync(dst + 2 * nb, res.charge, cb, hipMemcpyDeviceToDevice, rs);
                if (cb && ce == hipSuccess) ce = hipMemcpyAsync(dst + 3 * nb, res.size, cb, hipMemcpyDeviceToDevice, rs);
                if (ce == hipSuccess) ce = hipStreamSynchronize(rs);
                if (ce != hipSuccess) { rc.store(PXCL_E_HIP); break; }
                blocked[t] += us_since(p1, clk::now());
            }
            if (r != PXCL_OK) ++errors[t];
            digis[t] += in.n;
            lat[t].push_back(us_since(t0, p1));
        }
    };
    std::vector<std::thread> th;
    for (u32 t = 0; t < n_threads; ++t) th.emplace_back(worker, t);
    while (ready.load() < n_threads) std::this_thread::yield();
    const auto w0 = clk::now();
    go.store(true, std::memory_order_release);
    for (auto& x : th) x.join();
    const auto w1 = clk::now();

    std::memset(out, 0, sizeof(*out));
    std::vector<double> all;
    double bl = 0;
    for (u32 t = 0; t < n_threads; ++t) {
        all.insert(all.end(), lat[t].begin(), lat[t].end());
        bl += blocked[t];
        out->cpu_tasks += tasks[t];
        out->digis += digis[t];
        out->errors += errors[t];
    }
    out->wall_s = us_since(w0, w1) * 1e-6;
    out->events = all.size();
    out->lat_p50_us = percentile(all, 0.50);
    out->lat_p99_us = percentile(all, 0.99);
    out->lat_max_us = all.empty() ? 0 : all.back();
    out->blocked_us_per_event = all.empty() ? 0 : bl / double(all.size());
    out->cpu_tasks_per_s = out->wall_s > 0 ? double(out->cpu_tasks) / out->wall_s : 0;
    out->max_inflight = max_inflight.load();
    out->batches = all.size();
    return rc.load();
}

// ---------------------------------------------------------------------------
// serving form
// ---------------------------------------------------------------------------
namespace {

struct Request {
    double arrival_us;
    double admit_us, launch_us, done_us, produce_us;   // stage ends
    u32 pool_idx;
    u32 cls;      // size class
    u32 slot;     // event slot while admitted
};

// Event slots for the serving form, bound once in size classes: class c holds events
// of up to cap[c] digis (powers of two from 16,384 up to the largest request).  The
// slots of a class take a share of the slot count and of the memory budget in
// proportion to how many requests need that class, at least one each.  Admission then
// takes a free slot of the request's class (or of a larger one): no allocation, binding
// or clearing happens per request.
struct SlotPool {
    std::vector<u32> cap;                     // per class: capacity in digis
    std::vector<size_t> bytes;                // per class: workspace bytes
    std::vector<std::vector<u32>> free;       // per class: free slot indices
    std::vector<u32> slot_cls;                // per slot: its class
    std::vector<pxcl_event*> ev;              // per slot
    size_t in_use = 0, peak = 0;
    u32 class_of(u32 n) const {
        for (u32 c = 0; c < cap.size(); ++c)
            if (n <= cap[c]) return c;
        return u32(cap.size()) - 1;
    }
};

struct ServeState;


struct BatchCtx {
    ServeState* S;
    u32 bi;
    u32 k;
    u32 req[MAXB];
};

// Hand-overs between the serving threads take no lock: a CPU thread (lower priority,
// more threads than its cores) preempted while holding a lock would stall the
// dispatcher or the completion thread for a time slice (milliseconds).  Every request
// passes each queue once, so each is an array of n_requests places filled in order.
struct ServeState {
    u32* produce_q = nullptr;           // requests whose batch completed (one producer:
    u32 produce_fill = 0;               // the completion thread, which alone uses fill)
    std::atomic<u32> produce_tail{0};   // places published
    std::atomic<u32> produce_head{0};   // places taken by the CPU threads
    std::atomic<u32> done{0};
    std::atomic<u32> batch_free_mask{0};
    Request* req = nullptr;
    clk::time_point t0;
    std::atomic<int> dispatch_wake{0};  // a batch completed: the dispatcher may launch
};

void serve_batch_done(void* user, int32_t) {
    BatchCtx* bc = static_cast<BatchCtx*>(user);
    ServeState* S = bc->S;
    S->dispatch_wake.store(1, std::memory_order_release);
    const double now = us_since(S->t0, clk::now());
    for (u32 i = 0; i < bc->k; ++i) {
        S->req[bc->req[i]].done_us = now;
        S->produce_q[S->produce_fill++] = bc->req[i];
    }
    S->produce_tail.store(S->produce_fill, std::memory_order_release);
    S->batch_free_mask.fetch_or(1u << bc->bi, std::memory_order_acq_rel);
}

}  // namespace

extern "C" int pxcl_serve(pxcl_ctx* ctx, void* d_arena, size_t arena_bytes, void* h_pinned, size_t pinned_bytes,
                          pxcl_batch* const* batches, void* const* streams, uint32_t n_batches,
                          const pxcl_digis* pool, uint32_t pool_size, const pxcl_serve_opts* o, pxcl_run_stats* out,
                          int32_t* request_status, uint32_t* request_nclusters, void* d_results,
                          const uint64_t* result_offsets) {
    if (!ctx || !d_arena || !h_pinned || !batches || !streams || !pool || !o || !out) return PXCL_E_INVAL;
    if (n_batches == 0 || n_batches > 32 || pool_size == 0 || o->n_slots == 0 || o->max_batch == 0 ||
        o->max_batch > MAXB || o->n_requests == 0 || !(o->rate_hz > 0))
        return PXCL_E_INVAL;
    if (pinned_bytes < size_t(o->n_slots) * pxcl_event_pinned_bytes(ctx)) return PXCL_E_CAPACITY;
    const int dev = ctx_device(ctx);
    hipSetDevice(dev);
    u32 max_n = 0;
    for (u32 i = 0; i < pool_size; ++i) max_n = std::max(max_n, pool[i].n);
    const size_t min_ws = pxcl_event_workspace_bytes(ctx, std::max<u32>(max_n, 1));
    if (min_ws == 0 || min_ws > arena_bytes || min_ws > o->budget_bytes) return PXCL_E_CAPACITY;

    SlotPool P;
    for (u32 c = 16384;; c *= 2) {
        P.cap.push_back(std::min(c, std::max<u32>(max_n, 1)));
        if (c >= max_n) break;
    }
    const u32 ncls = u32(P.cap.size());
    for (u32 c = 0; c < ncls; ++c) P.bytes.push_back(al256(pxcl_event_workspace_bytes(ctx, P.cap[c])));
    std::vector<double> need(ncls, 0.0);
    for (u32 i = 0; i < o->n_requests; ++i) need[P.class_of(std::max<u32>(pool[i % pool_size].n, 1))] += 1.0;
    const size_t budget = std::min<size_t>(o->budget_bytes, arena_bytes);
    std::vector<u32> count(ncls, 0);
    size_t total = 0;
    u32 nslots = 0;
    for (u32 c = 0; c < ncls; ++c)
        if (need[c] > 0) {
            count[c] = std::max<u32>(1, u32(double(o->n_slots) * need[c] / double(o->n_requests)));
            total += count[c] * P.bytes[c];
            nslots += count[c];
        }
    while ((total > budget || nslots > o->n_slots) ) {   // shrink the class with the most bytes
        u32 w = ncls;
        for (u32 c = 0; c < ncls; ++c)
            if (count[c] > 1 && (w == ncls || count[c] * P.bytes[c] > count[w] * P.bytes[w])) w = c;
        if (w == ncls) break;
        --count[w];
        total -= P.bytes[w];
        --nslots;
    }
    if (total > budget || nslots > o->n_slots) return PXCL_E_CAPACITY;
    const size_t hsb = pxcl_event_pinned_bytes(ctx);
    hipStream_t s0 = static_cast<hipStream_t>(streams[0]);
    int rc = PXCL_OK;
    P.free.resize(ncls);
    size_t off = 0;
    for (u32 c = 0; c < ncls && rc == PXCL_OK; ++c)
        for (u32 j = 0; j < count[c] && rc == PXCL_OK; ++j) {
            const u32 i = u32(P.ev.size());
            pxcl_event* e = nullptr;
            rc = pxcl_event_bind(ctx, static_cast<u8*>(d_arena) + off, P.bytes[c], static_cast<u8*>(h_pinned) + i * hsb,
                                 hsb, P.cap[c], s0, &e);
            if (rc != PXCL_OK) break;
            P.ev.push_back(e);
            P.slot_cls.push_back(c);
            P.free[c].push_back(i);
            off += P.bytes[c];
        }
    if (rc == PXCL_OK && hipStreamSynchronize(s0) != hipSuccess) rc = PXCL_E_HIP;
    if (rc != PXCL_OK) {
        for (auto* e : P.ev) pxcl_event_unbind(e);
        return rc;
    }
    std::vector<pxcl_event*>& slot_ev = P.ev;

    // arrivals
    std::vector<Request> req(o->n_requests);
    {
        std::mt19937_64 rng(o->seed);
        std::exponential_distribution<double> gap(o->rate_hz * 1e-6);
        double t = 0;
        for (u32 i = 0; i < o->n_requests; ++i) {
            t += gap(rng);
            req[i].arrival_us = t;
            req[i].pool_idx = i % pool_size;
            req[i].cls = P.class_of(std::max<u32>(pool[req[i].pool_idx].n, 1));
        }
    }

    const CorePlan cores = plan_cores();
    // the CPU threads' task rate with no requests (the reference for the rate while serving)
    double idle_rate = 0.0;
    if (o->cpu_task_ns) {
        const u32 nt = std::max<u32>(1, o->n_cpu_threads);
        std::atomic<u64> n_idle{0};
        std::vector<std::thread> it;
        const auto i0 = clk::now();
        for (u32 t = 0; t < nt; ++t)
            it.emplace_back([&, t] {
                place_worker(cores);
                u64 k = 0;
                while (us_since(i0, clk::now()) < 50000.0) {
                    g_sink.fetch_add(cpu_task(o->cpu_task_ns, k + t), std::memory_order_relaxed);
                    ++k;
                }
                n_idle.fetch_add(k);
            });
        for (auto& x : it) x.join();
        idle_rate = double(n_idle.load()) / (us_since(i0, clk::now()) * 1e-6);
    }

    ServeState S;
    std::vector<u32> produce_q(o->n_requests);
    S.produce_q = produce_q.data();
    S.req = req.data();
    // slots released by the CPU threads: a thread claims a place, then writes slot + 1
    // there; the dispatcher, which alone owns the free lists, takes them in order
    std::vector<std::atomic<u32>> released(o->n_requests);
    for (auto& x : released) x.store(0u, std::memory_order_relaxed);
    std::atomic<u32> released_tail{0};
    u32 released_head = 0;
    S.batch_free_mask.store((n_batches >= 32 ? 0xFFFFFFFFu : ((1u << n_batches) - 1u)));
    std::vector<BatchCtx> bctx(n_batches);
    for (u32 b = 0; b < n_batches; ++b) { bctx[b].S = &S; bctx[b].bi = b; bctx[b].k = 0; }
    std::vector<double> lat(o->n_requests, 0.0);
    std::atomic<u64> blocked_ns{0}, tasks{0}, batches_launched{0};
    std::atomic<u32> errors{0}, inflight{0}, max_inflight{0};
    std::atomic<bool> stop{false};
    std::atomic<int> err_rc{PXCL_OK};
    // the arrival clock starts once the CPU threads exist (they read it only for
    // requests, which come after it starts, through the completion thread's hand-over)
    clk::time_point t0;

    // CPU threads: produce first, else a synthetic task
    auto cpu_worker = [&](u32 t) {
        hipSetDevice(dev);
        place_worker(cores);
        u64 local_tasks = 0;
        for (;;) {
            u32 r = 0xFFFFFFFFu;
            for (u32 h = S.produce_head.load(std::memory_order_acquire);
                 h < S.produce_tail.load(std::memory_order_acquire);) {
                if (S.produce_head.compare_exchange_weak(h, h + 1, std::memory_order_acq_rel)) {
                    r = S.produce_q[h];
                    break;
                }
            }
            if (r == 0xFFFFFFFFu) {
                if (stop.load()) break;
                if (!o->cpu_task_ns) std::this_thread::sleep_for(std::chrono::microseconds(20));
            }
            if (r != 0xFFFFFFFFu) {
                Request& q = req[r];
                pxcl_clusters res;
                const auto p0 = clk::now();
                const int st = pxcl_produce(slot_ev[q.slot], &res);
                const auto p1 = clk::now();
                blocked_ns.fetch_add(u64(std::chrono::duration_cast<std::chrono::nanoseconds>(p1 - p0).count()));
                q.produce_us = us_since(t0, p1);
                lat[r] = q.produce_us - q.arrival_us;
                if (d_results && result_offsets) {   // verification mode: copy out, then release
                    u8* dst = static_cast<u8*>(d_results) + result_offsets[r];
                    const size_t nb = size_t(res.n_digis) * 4, cb = size_t(res.n_clusters) * 4;
                    hipStream_t rs = static_cast<hipStream_t>(res.stream);
                    const auto c0 = clk::now();
                    hipError_t ce = hipSuccess;
                    if (nb) ce = hipMemcpyAsync(dst, res.digi_cluster, nb, hipMemcpyDeviceToDevice, rs);
                    if (cb && ce == hipSuccess) ce = hipMemcpyAsync(dst + nb, res.id, cb, hipMemcpyDeviceToDevice, rs);
                    if (cb && ce == hipSuccess) ce = hipMemcpyAsync(dst + 2 * nb, res.charge, cb, hipMemcpyDeviceToDevice, rs);
                    if (cb && ce == hipSuccess) ce = hipMemcpyAsync(dst + 3 * nb, res.size, cb, hipMemcpyDeviceToDevice, rs);
                    if (ce == hipSuccess) ce = hipStreamSynchronize(rs);
                    if (ce != hipSuccess) err_rc.store(PXCL_E_HIP);
                    blocked_ns.fetch_add(u64(std::chrono::duration_cast<std::chrono::nanoseconds>(clk::now() - c0).count()));
                }
                if (st != PXCL_OK) errors.fetch_add(1);
                if (request_status) request_status[r] = st;
                if (request_nclusters) request_nclusters[r] = res.n_clusters;
                released[released_tail.fetch_add(1, std::memory_order_acq_rel)].store(q.slot + 1u,
                                                                                   std::memory_order_release);
                inflight.fetch_sub(1);
                S.done.fetch_add(1, std::memory_order_acq_rel);
            } else if (o->cpu_task_ns) {
                g_sink.fetch_add(cpu_task(o->cpu_task_ns, local_tasks + t), std::memory_order_relaxed);
                ++local_tasks;
            }
        }
        tasks.fetch_add(local_tasks);
    };
    const u32 ncpu = std::max<u32>(1, o->n_cpu_threads);
    std::vector<std::thread> th;
    for (u32 t = 0; t < ncpu; ++t) th.emplace_back(cpu_worker, t);
    t0 = clk::now();
    S.t0 = t0;

    // dispatcher: arrivals -> admission -> batches.  Its waits are short sleeps; the
    // thread's timer slack is cut to 1 us meanwhile (the default 50 us would be the
    // granularity of every wait), and restored at the end.
    const int old_slack = prctl(PR_GET_TIMERSLACK, 0, 0, 0, 0);
    prctl(PR_SET_TIMERSLACK, 1000UL, 0, 0, 0);
    if (cores.on) {
        (void)sched_setaffinity(0, sizeof(cpu_set_t), &cores.dispatcher);
        ctx_place_completer(ctx, &cores.completer);
    }
    std::deque<u32> arrived, admitted;
    u32 next_arrival = 0;
    std::vector<pxcl_event*> bev(MAXB);
    std::vector<pxcl_digis> bin(MAXB);
    while (S.done.load(std::memory_order_acquire) < o->n_requests && err_rc.load() == PXCL_OK) {
        const double now = us_since(t0, clk::now());
        while (next_arrival < o->n_requests && req[next_arrival].arrival_us <= now) arrived.push_back(next_arrival++);
        for (u32 v; released_head < o->n_requests &&
                    (v = released[released_head].load(std::memory_order_acquire)) != 0u; ++released_head) {
            P.free[P.slot_cls[v - 1u]].push_back(v - 1u);      // a slot free again
            P.in_use -= P.bytes[P.slot_cls[v - 1u]];
        }
        if (!arrived.empty()) {
            // In arrival order, a request takes a free slot of its class or else of the
            // smallest larger class that has one.  One that finds none waits without
            // holding back those behind it: every class it can use is empty, so a later
            // request admitted now takes nothing it waits for, and a later one of its
            // class or above waits too (blocked_from).
            const u32 ncls_ = u32(P.free.size());
            u32 blocked_from = ncls_;
            for (size_t i = 0, n = arrived.size(); i < n; ++i) {
                const u32 ri = arrived.front();
                arrived.pop_front();
                Request& q = req[ri];
                u32 c = q.cls;
                if (c < blocked_from)
                    while (c < ncls_ && P.free[c].empty()) ++c;
                if (c >= blocked_from || c >= ncls_) {
                    blocked_from = std::min(blocked_from, q.cls);
                    arrived.push_back(ri);               // keeps its place among those waiting
                    continue;
                }
                q.slot = P.free[c].back();
                P.free[c].pop_back();
                q.admit_us = now;
                P.in_use += P.bytes[c];
                P.peak = std::max(P.peak, P.in_use);
                admitted.push_back(ri);
            }
        }
        u32 mask = S.batch_free_mask.load(std::memory_order_acquire);
        // At most max_inflight batches on the device: while they run, arrivals
        // accumulate, so batches grow with the load.  With a batching delay, a batch
        // also waits, while others run, to be half full or for its oldest request to
        // have waited that long; with nothing in flight it starts at once.
        const u32 all = n_batches >= 32 ? 0xFFFFFFFFu : ((1u << n_batches) - 1u);
        const u32 busy = u32(__builtin_popcount(all & ~mask));
        const u32 limit = o->max_inflight ? std::min(o->max_inflight, n_batches) : n_batches;
        const bool ready = !admitted.empty() && busy < limit &&
                           (busy == 0 || !o->batch_delay_us || admitted.size() >= std::max<u32>(1, o->max_batch / 2) ||
                            now - req[admitted.front()].arrival_us >= double(o->batch_delay_us));
        if (ready && mask) {
            const u32 b = __builtin_ctz(mask);
            S.batch_free_mask.fetch_and(~(1u << b), std::memory_order_acq_rel);
            BatchCtx& bc = bctx[b];
            u32 k = 0;
            hipStream_t s = static_cast<hipStream_t>(streams[b]);
            const auto a0 = clk::now();
            while (!admitted.empty() && k < o->max_batch) {
                const u32 r = admitted.front();
                admitted.pop_front();
                Request& q = req[r];
                bev[k] = slot_ev[q.slot];
                bin[k] = pool[q.pool_idx];
                bc.req[k] = r;
                ++k;
            }
            bc.k = k;
            const double lnow = us_since(t0, a0);
            for (u32 i = 0; i < k; ++i) req[bc.req[i]].launch_us = lnow;
            const int r = pxcl_acquire_batch(batches[b], bev.data(), bin.data(), k, s, serve_batch_done, &bc,
                                             o->flags);
            blocked_ns.fetch_add(u64(std::chrono::duration_cast<std::chrono::nanoseconds>(clk::now() - a0).count()));
            if (r != PXCL_OK) { err_rc.store(r); break; }
            batches_launched.fetch_add(1);
            const u32 now_in = inflight.fetch_add(k) + k;
            u32 m = max_inflight.load();
            while (now_in > m && !max_inflight.compare_exchange_weak(m, now_in)) {}
        } else {
            // nothing to launch: sleep until the next arrival or a batch completion,
            // checking every 5 us at most
            const double next = next_arrival < o->n_requests ? req[next_arrival].arrival_us : now + 5.0;
            const double wait = std::min(5.0, std::max(0.0, next - now));
            if (!S.dispatch_wake.exchange(0, std::memory_order_acq_rel) && wait > 0.5)
                std::this_thread::sleep_for(std::chrono::nanoseconds(u64(wait * 1000.0)));
        }
    }
    // the requests are served: the run ends here, not when the CPU threads (which may be
    // waiting for a time slice) have noticed the stop
    const auto t1 = clk::now();
    if (old_slack > 0) prctl(PR_SET_TIMERSLACK, u64(old_slack), 0, 0, 0);
    if (cores.on) {
        (void)sched_setaffinity(0, sizeof(cpu_set_t), &cores.all);
        ctx_place_completer(ctx, nullptr);
    }
    stop.store(true);
    for (auto& x : th) x.join();
    const auto t_join = clk::now();
    for (u32 b = 0; b < n_batches; ++b) hipStreamSynchronize(static_cast<hipStream_t>(streams[b]));
    for (auto* e : slot_ev) pxcl_event_unbind(e);

    std::memset(out, 0, sizeof(*out));
    std::vector<double> l(lat);
    u64 dg = 0;
    for (u32 i = 0; i < o->n_requests; ++i) dg += pool[req[i].pool_idx].n;
    out->wall_s = us_since(t0, t1) * 1e-6;
    out->events = o->n_requests;
    out->digis = dg;
    out->lat_p50_us = percentile(l, 0.50);
    out->lat_p99_us = percentile(l, 0.99);
    out->lat_max_us = l.empty() ? 0 : l.back();
    out->blocked_us_per_event = double(blocked_ns.load()) * 1e-3 / double(o->n_requests);
    out->cpu_tasks = tasks.load();
    const double cpu_s = us_since(t0, t_join) * 1e-6;      // the CPU threads ran until they stopped
    out->cpu_tasks_per_s = cpu_s > 0 ? double(out->cpu_tasks) / cpu_s : 0;
    out->errors = errors.load();
    out->max_inflight = max_inflight.load();
    out->peak_resident_bytes = P.peak;
    out->batches = batches_launched.load();
    std::vector<double> st(o->n_requests);
    for (int k = 0; k < 4; ++k) {
        for (u32 i = 0; i < o->n_requests; ++i) {
            const Request& q = req[i];
            const double a[5] = {q.arrival_us, q.admit_us, q.launch_us, q.done_us, q.produce_us};
            st[i] = a[k + 1] - a[k];
        }
        out->stage_p50_us[k] = percentile(st, 0.50);
        out->stage_p99_us[k] = percentile(st, 0.99);
    }
    out->cpu_tasks_per_s_idle = idle_rate;
    const double last_arrival_us = o->n_requests ? req[o->n_requests - 1].arrival_us : 0.0;
    out->offered_per_s = last_arrival_us > 0 ? double(o->n_requests) / (last_arrival_us * 1e-6) : 0.0;
    return err_rc.load();
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
namespace {
const u32 kWG[4] = {64, 128, 256, 512};
const u32 kMPW[3] = {1, 2, 4};

std::string cache_key(pxcl_ctx* ctx, u32 mean_digis) {
    u32 bucket = 0;
    while ((2u << bucket) <= mean_digis && bucket < 31) ++bucket;
    return ctx_arch(ctx) + "|" + std::to_string(bucket);
}

// The cache is a flat JSON object {"<arch>|<log2 bucket>": [wg, mpw], ...}.
std::map<std::string, std::pair<u32, u32>> read_cache(const char* path) {
    std::map<std::string, std::pair<u32, u32>> m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t p = 0;
    for (;;) {
        const size_t q0 = s.find('"', p);
        if (q0 == std::string::npos) break;
        const size_t q1 = s.find('"', q0 + 1);
        const size_t b0 = s.find('[', q1);
        const size_t b1 = s.find(']', b0);
        if (q1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos) break;
        unsigned wg = 0, mpw = 0;
        if (std::sscanf(s.substr(b0 + 1, b1 - b0 - 1).c_str(), "%u , %u", &wg, &mpw) == 2)
            m[s.substr(q0 + 1, q1 - q0 - 1)] = {wg, mpw};
        p = b1 + 1;
    }
    return m;
}
}  // namespace

extern "C" int pxcl_autotune(pxcl_ctx* ctx, pxcl_batch* b, pxcl_event* const* evs, const pxcl_digis* ins, uint32_t k,
                             void* stream, uint32_t reps, const char* cache_path, float* us_out) {
    if (!ctx || !b || !evs || !ins || k == 0 || reps == 0) return PXCL_E_INVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipSetDevice(ctx_device(ctx));
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return PXCL_E_HIP;
    u32 best_wg = 0, best_mpw = 0;
    float best = 0;
    int rc = PXCL_OK;
    u64 digis = 0;
    for (u32 i = 0; i < k; ++i) digis += ins[i].n;
    for (u32 a = 0; a < 4 && rc == PXCL_OK; ++a)
        for (u32 c = 0; c < 3 && rc == PXCL_OK; ++c) {
            const u32 wg = kWG[a], mpw = kMPW[c];
            float* slot = us_out ? &us_out[a * 3 + c] : nullptr;
            if (!cluster_config_valid(wg, mpw)) { if (slot) *slot = -1.f; continue; }
            pxcl_set_kernel_config(ctx, wg, mpw);
            double tot = 0;
            for (u32 r = 0; r <= reps && rc == PXCL_OK; ++r) {   // r == 0 warms up
                hipEventRecord(e0, s);
                rc = pxcl_acquire_batch(b, evs, ins, k, s, nullptr, nullptr, 0);
                hipEventRecord(e1, s);
                if (rc != PXCL_OK) break;
                hipEventSynchronize(e1);
                while (pxcl_batch_query(b) == PXCL_E_NOT_READY) std::this_thread::yield();
                float ms = 0;
                hipEventElapsedTime(&ms, e0, e1);
                if (r) tot += ms;
            }
            const float us = float(tot * 1e3 / reps);
            if (slot) *slot = us;
            if (best_wg == 0 || us < best) { best = us; best_wg = wg; best_mpw = mpw; }
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc != PXCL_OK) return rc;
    pxcl_set_kernel_config(ctx, best_wg, best_mpw);
    if (cache_path) {
        auto m = read_cache(cache_path);
        m[cache_key(ctx, u32(digis / k))] = {best_wg, best_mpw};
        std::ofstream f(cache_path);
        if (!f) return PXCL_E_INVAL;
        f << "{\n";
        size_t i = 0;
        for (auto& kv : m)
            f << "  \"" << kv.first << "\": [" << kv.second.first << ", " << kv.second.second << "]"
              << (++i < m.size() ? ",\n" : "\n");
        f << "}\n";
    }
    return PXCL_OK;
}

extern "C" int pxcl_autotune_load(pxcl_ctx* ctx, const char* cache_path, uint32_t mean_digis) {
    if (!ctx || !cache_path) return PXCL_E_INVAL;
    auto m = read_cache(cache_path);
    auto it = m.find(cache_key(ctx, mean_digis));
    if (it == m.end()) return PXCL_E_NOTFOUND;
    return pxcl_set_kernel_config(ctx, it->second.first, it->second.second);
}
