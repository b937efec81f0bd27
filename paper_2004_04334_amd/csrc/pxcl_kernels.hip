// Device kernels of the pixel-clustering path (gfx950 / CDNA4, wave64).
//
// One launch processes k >= 1 events through four kernels:
//
//   segment  streams the module ids, scatters the first digi of every module
//            present into a per-module table, checks module range and order; the
//            workgroup that finishes an event's last chunk turns the table into
//            the event's ordered list of modules ("items") and splits it into
//            small and big items.
//   big      one big module per 512-thread workgroup (digis held in registers
//            up to 16,384 per module, beyond that re-read from memory).
//   small    one small module per group of threads (a single wave, or a whole
//            workgroup): fired-pixel bitmap in LDS, vertical runs, union-find over
//            runs, charge/size per cluster, charge cut; the module's kept clusters
//            go in ascending id to a staging area at the module's first digi, and
//            every digi gets its cluster id.  Groups take modules with an atomic
//            ticket and prefetch the next module while working on the current one.
//   compact  per event, the offset of each module's clusters (a sum over the
//            kept counts of the modules before it) and a copy of the staged
//            records to their final position; status write-back to the host.
//
// The clustering: 8-connected components of fired pixels within a module; cluster
// id = smallest linear index module*66560 + col*160 + row; charge = sum of ADC
// (uint32); keep iff charge >= cut.  This is the "ClusterProducer" step of the
// paper's Figure 1 (Sec. 3).  Errors go to a device error word, never to device
// asserts, which would synchronise (Sec. 4.1).
//
// Memory ordering.  Workgroup barriers here order LDS only (global loads and stores
// stay in flight across them).  Data that another workgroup of the same kernel reads
// is written with device-scope atomic stores and published by a device-scope atomic
// counter after the writer has waited for its stores to complete; everything else
// crosses a kernel boundary.  No device-scope release/acquire fence is used: on
// gfx950 those write back and invalidate the L2.
#include <hip/hip_runtime.h>

#include "pxcl_internal.h"

namespace pxcl {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ u32 ld_wg(const u32* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void st_wg(u32* p, u32 v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ u32 ld_ag(const u32* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_ag(u32* p, u32 v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 ld_ag64(const u64* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_ag64(u64* p, u64 v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_sys(u32* p, u32 v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
// Wait until every memory operation this thread issued has completed.
__device__ __forceinline__ void wait_all_mem() { __builtin_amdgcn_s_waitcnt(0); }

// Barrier over a group of G threads that orders LDS accesses only.  A group of 64
// is one wave: LDS requests of a wave are served in order, so only the compiler
// must be kept from moving accesses across the point.
template <u32 G>
__device__ __forceinline__ void gsync() {
    if constexpr (G == 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    }
}
__device__ __forceinline__ void lds_barrier() { gsync<128>(); }

__device__ __forceinline__ u32 num_events(const LaunchArgs& a) { return a.hdr ? a.hdr[0] : 1u; }
__device__ __forceinline__ EventDesc get_event(const LaunchArgs& a, u32 e) {
    return a.hdr ? reinterpret_cast<const EventDesc*>(reinterpret_cast<const u8*>(a.hdr) + HDR_EV_OFFSET)[e]
                 : a.single;
}
template <typename T>
__device__ __forceinline__ T* ws_ptr(const EventDesc& E, size_t off) {
    return reinterpret_cast<T*>(E.ws + off);
}

// Inclusive scan across the 64 lanes of a wave.
__device__ __forceinline__ u32 wave_incl_scan(u32 v) {
    const u32 lane = threadIdx.x & 63u;
#pragma unroll
    for (u32 d = 1; d < 64; d <<= 1) {
        const u32 y = __shfl_up(v, d, 64);
        if (lane >= d) v += y;
    }
    return v;
}

// Exclusive scan over a group of G threads (whole waves).  With G > 64 every thread
// of the workgroup must call it (it holds two LDS barriers); `wsum` has G/64 words
// private to the group.
template <u32 G>
__device__ __forceinline__ u32 group_excl_scan(u32 v, u32 lt, u32* wsum, u32& total) {
    const u32 inc = wave_incl_scan(v);
    if constexpr (G == 64) {
        total = __shfl(inc, 63, 64);
        return inc - v;
    } else {
        const u32 w = lt >> 6;
        if ((lt & 63u) == 63u) wsum[w] = inc;
        gsync<G>();
        u32 off = 0, tot = 0;
#pragma unroll
        for (u32 i = 0; i < G / 64; ++i) {
            const u32 s = wsum[i];
            off += (i < w) ? s : 0u;
            tot += s;
        }
        gsync<G>();
        total = tot;
        return off + inc - v;
    }
}

// Largest i in [0, k) with pref[i] <= t, given pref[0] <= t < pref[k].
__device__ __forceinline__ u32 find_slot(const u32* pref, u32 k, u32 t) {
    u32 lo = 0, hi = k;
    while (hi - lo > 1) {
        const u32 mid = (lo + hi) >> 1;
        if (pref[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// Prefix over the events of a launch of max(ceil(count / div), at_least), where
// count is the event's digis (which = 0) or one of its control words (which =
// CTL_*; 0 for an empty event).  pref[k] = total.  Every thread of the workgroup
// calls it; any k <= MAXB with any BS.
template <u32 BS>
__device__ __forceinline__ u32 event_prefix(const LaunchArgs& a, u32 k, u32* pref, u32* wsum, u32 which, u32 div, u32 at_least) {
    u32 carry = 0;
    for (u32 base = 0; base < k; base += BS) {
        const u32 e = base + threadIdx.x;
        u32 v = 0;
        if (e < k) {
            const EventDesc E = get_event(a, e);
            u32 cnt = 0;
            if (E.n) cnt = which ? ld_ag(ws_ptr<u32>(E, ev_layout(E.cap, a.n_modules).ctl) + which) : E.n;
            v = max((cnt + div - 1) / div, at_least);
        }
        u32 tot;
        const u32 ex = group_excl_scan<BS>(v, threadIdx.x, wsum, tot);
        if (e < k) pref[e] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) pref[k] = carry;
    lds_barrier();
    return pref[k];
}

// ---------------------------------------------------------------------------
// bitmap helpers (column-major: 5 words per column; bit b of word w is row
// (w % 5)*32 + b of column w / 5)
// ---------------------------------------------------------------------------
__device__ __forceinline__ u32 fired(const u32* bm, u32 lin) { return (bm[lin >> 5] >> (lin & 31u)) & 1u; }

// Bits of word w that start a vertical run (fired, with the pixel above not fired).
__device__ __forceinline__ u32 run_starts(const u32* bm, u32 w) {
    const u32 b = bm[w];
    const u32 carry = (w % WPC) ? (bm[w - 1] >> 31) : 0u;
    return b & ~((b << 1) | carry);
}

// Index of the vertical run containing fired pixel lin: run starts before word w
// plus run starts in w at or below bit b, minus one.
__device__ __forceinline__ u32 run_of(const u32* bm, const u16* rpre, u32 lin) {
    const u32 w = lin >> 5, b = lin & 31u;
    const u32 mask = (2u << b) - 1u;       // bits 0..b (b = 31 wraps to all ones)
    return u32(rpre[w]) + __popc(run_starts(bm, w) & mask) - 1u;
}

// Union-find over runs in LDS: parent[x] <= x always; union hooks the larger root
// under the smaller with atomicMin; find halves paths with plain stores, which only
// ever point a node to one of its ancestors.  Both loops strictly decrease their
// index, so they terminate; the caps are a second guard.
__device__ __forceinline__ u32 uf_find(u32* par, u32 x) {
    for (u32 it = 0; it < 2 * MAX_RUNS; ++it) {
        const u32 p = ld_wg(&par[x]);
        if (p == x) return x;
        const u32 g = ld_wg(&par[p]);
        if (g == p) return p;
        st_wg(&par[x], g);
        x = g;
    }
    return x;
}

__device__ __forceinline__ void uf_unite(u32* par, u32 a, u32 b) {
    for (u32 it = 0; it < 2 * MAX_RUNS; ++it) {
        a = uf_find(par, a);
        b = uf_find(par, b);
        if (a == b) return;
        if (a < b) { const u32 t = a; a = b; b = t; }
        const u32 old = __hip_atomic_fetch_min(&par[a], b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == a) return;
        a = old;
    }
}

// Links of fired pixel lin (row, col, run r) to the next column.  Pixel (row, col)
// touches (row-1..row+1, col+1).  If (row, col+1) is fired its run contains the other
// two when they are fired; a pixel whose upper neighbour (row-1, col) is fired leaves
// (row-1, col+1) and (row, col+1) to that neighbour.
__device__ __forceinline__ void link_right(u32* par, const u32* bm, const u16* rpre, u32 lin, u32 row, u32 col,
                                           u32 r) {
    if (col + 1 >= COLS) return;
    const bool up = row > 0 && fired(bm, lin - 1);
    if (fired(bm, lin + ROWS)) {
        if (!up) uf_unite(par, r, run_of(bm, rpre, lin + ROWS));
        return;
    }
    if (row + 1 < ROWS && fired(bm, lin + ROWS + 1)) uf_unite(par, r, run_of(bm, rpre, lin + ROWS + 1));
    if (!up && row > 0 && fired(bm, lin + ROWS - 1)) uf_unite(par, r, run_of(bm, rpre, lin + ROWS - 1));
}

// ---------------------------------------------------------------------------
// segment
// ---------------------------------------------------------------------------
// Turn the event's per-module table into the ordered item list and the two class
// lists.  Run by one whole workgroup of A_WG threads.
__device__ __forceinline__ void index_event(const LaunchArgs& a, const EventDesc& E, const EvLayout& L, u32* wsum) {
    const u32 tid = threadIdx.x;
    const u32 M = a.n_modules, n = E.n;
    const u64* seg = ws_ptr<const u64>(E, L.seg);
    u32* item_start = ws_ptr<u32>(E, L.item_start);
    u32* item_mod = ws_ptr<u32>(E, L.item_mod);
    u32* ctl = ws_ptr<u32>(E, L.ctl);
    u32 items = 0;
    for (u32 base = 0; base < M; base += A_WG) {
        const u32 m = base + tid;
        u64 v = 0;
        if (m < M) v = ld_ag64(&seg[m]);
        const bool act = m < M && u32(v >> 32) == E.epoch;
        u32 tot;
        const u32 ex = group_excl_scan<A_WG>(act ? 1u : 0u, tid, wsum, tot);
        if (act) {
            st_ag(&item_start[items + ex], min(u32(v), n));
            st_ag(&item_mod[items + ex], m);
        }
        items += tot;
    }
    if (tid == 0) {
        st_ag(&item_start[items], n);
        st_ag(&ctl[CTL_ITEMS], items);
    }
    wait_all_mem();
    lds_barrier();
    u32* small = ws_ptr<u32>(E, L.small);
    u32* big = ws_ptr<u32>(E, L.big);
    u32 ns = 0, nb = 0;
    for (u32 base = 0; base < items; base += A_WG) {
        const u32 i = base + tid;
        u32 cls = 0;   // 1 small, 2 big
        if (i < items) {
            const u32 s0 = ld_ag(&item_start[i]), s1 = ld_ag(&item_start[i + 1]);
            if (s1 > s0) cls = (s1 - s0 <= a.dcap) ? 1u : 2u;   // starts out of order: no item
        }
        u32 tot;
        const u32 ex = group_excl_scan<A_WG>((cls == 1 ? 1u : 0u) | (cls == 2 ? 1u << 16 : 0u), tid, wsum, tot);
        if (cls == 1) small[ns + (ex & 0xFFFFu)] = i;
        if (cls == 2) big[nb + (ex >> 16)] = i;
        ns += tot & 0xFFFFu;
        nb += tot >> 16;
    }
    if (tid == 0) {
        ctl[CTL_SMALL] = ns;
        ctl[CTL_BIG] = nb;
        st_ag(&ctl[CTL_SEGDONE], 0u);
    }
}

__global__ __launch_bounds__(A_WG) void k_segment(LaunchArgs a) {
    __shared__ u32 s_pref[MAXB + 1];
    __shared__ u32 s_wsum[A_WG / 64];
    __shared__ u32 s_err, s_last;
    const u32 tid = threadIdx.x;
    const u32 k = num_events(a);
    const u32 total = event_prefix<A_WG>(a, k, s_pref, s_wsum, 0, A_CH, 0);

    for (u32 t = blockIdx.x; t < total; t += gridDim.x) {
        if (tid == 0) s_err = 0;
        const u32 e = find_slot(s_pref, k, t);
        const u32 c = t - s_pref[e];
        const EventDesc E = get_event(a, e);
        const EvLayout L = ev_layout(E.cap, a.n_modules);
        u64* seg = ws_ptr<u64>(E, L.seg);
        const u32 n = E.n;
        const u32 i0 = c * A_CH + tid * A_PER;
        u32 m[A_PER];
#pragma unroll
        for (u32 j = 0; j < A_PER; ++j) m[j] = E.module[min(i0 + j, n - 1)];
        const u32 prev = E.module[i0 > 0 ? min(i0 - 1, n - 1) : 0];
        lds_barrier();                           // s_err cleared
        u32 err = 0;
        const u64 tag = u64(E.epoch) << 32;
#pragma unroll
        for (u32 j = 0; j < A_PER; ++j) {
            const u32 i = i0 + j;
            if (i < n) {
                const u32 pm = (j == 0) ? prev : m[j - 1];
                if (i > 0 && m[j] < pm) err |= EB_ORDER;
                if (m[j] >= a.n_modules) err |= EB_RANGE;
                else if (i == 0 || m[j] != pm) st_ag64(&seg[m[j]], tag | i);
            }
        }
        if (err) atomicOr(&s_err, err);
        wait_all_mem();                          // this thread's table entries are visible
        lds_barrier();
        const u32 chunks = (n + A_CH - 1) / A_CH;
        if (tid == 0) {
            u32* ctl = ws_ptr<u32>(E, L.ctl);
            if (s_err) atomicOr(&ctl[CTL_ERR], s_err);
            s_last = (atomicAdd(&ctl[CTL_SEGDONE], 1u) == chunks - 1) ? 1u : 0u;
        }
        lds_barrier();
        if (s_last) index_event(a, E, L, s_wsum);
        lds_barrier();
    }
}

// ---------------------------------------------------------------------------
// clustering of one module with its digis in registers (K per thread, group of G)
// ---------------------------------------------------------------------------
constexpr u32 NOPIX = 0xFFFFFFFFu;

template <u32 G, u32 K>
struct RegModuleSmem {
    static constexpr u32 RCAP = G * K, KBW = RCAP / 32;
    u32 bm[WORDS];     // fired-pixel bitmap (clear between modules)
    u64 acc[RCAP];     // union-find parents (as u32, first half), then charge | size << 44
    u32 kb[KBW];       // kept-root bits over run index
    u16 rpre[WORDS];   // run starts before each word
    u16 kpre[KBW];     // kept roots before each kb word
    u32 wsum[G / 64];
};

// A module as a group sees it.
struct Item {
    u32 e, it, st, n, mod;
    bool ok;
};

constexpr u32 BADPIX = 0xFFFFFFFEu;          // a digi whose row or column is out of range

// Linear pixel index (or NOPIX / BADPIX) and ADC of the module's digis j = lt + q*G.
template <u32 G, u32 K>
__device__ __forceinline__ void load_digis(const EventDesc& E, const Item& I, u32 lt, u32* LIN, u32* A) {
    u32 R[K], C[K];
#pragma unroll
    for (u32 q = 0; q < K; ++q) {
        const u32 j = lt + q * G;
        const u32 i = I.st + (j < I.n ? j : 0u);     // always inside the module
        R[q] = E.row[i];
        C[q] = E.col[i];
        A[q] = E.adc[i];
    }
#pragma unroll
    for (u32 q = 0; q < K; ++q) {
        const u32 j = lt + q * G;
        LIN[q] = j >= I.n ? NOPIX : (R[q] < ROWS && C[q] < COLS) ? C[q] * ROWS + R[q] : BADPIX;
    }
}

// Cluster module I (n <= G*K) whose digis are in LIN/AR (load_digis; AR holds the
// ADC in its low 16 bits, the digi's run and then its root go in the high 16 bits).
// Every thread of the group calls it; with G > 64 all groups of the workgroup call
// it together.  `mid(stage)` runs after phases 1, 3, 5 and 8 (the next module's
// prefetch).
template <u32 G, u32 K, typename Mid>
__device__ __forceinline__ void cluster_regs(const LaunchArgs& a, const EventDesc& E, const EvLayout& L,
                                             const Item& I, RegModuleSmem<G, K>& gp, u32 lt, u32* LIN, u32* AR,
                                             Mid mid) {
    static_assert(G * K <= 65536, "run indices are kept in 16 bits");
    constexpr u32 KBW = G * K / 32, WPT = (WORDS + G - 1) / G;
    u32* par = reinterpret_cast<u32*>(gp.acc);
    const bool act = I.ok;
    u32 err = 0;
    // P1: insert the module's digis into the bitmap
#pragma unroll
    for (u32 q = 0; q < K; ++q) {
        AR[q] &= 0xFFFFu;
        if (!act) LIN[q] = NOPIX;
        if (LIN[q] == BADPIX) {
            err |= EB_RANGE;
            LIN[q] = NOPIX;
        }
        if (LIN[q] != NOPIX) {
            const u32 lin = LIN[q];
            const u32 bit = 1u << (lin & 31u);
            if (atomicOr(&gp.bm[lin >> 5], bit) & bit) err |= EB_DUP;
        }
    }
    mid(0);
    gsync<G>();
    // P2: run starts per word, prefix over words; parents
    u32 nruns = 0;
    {
        u32 sw[WPT];
        u32 cnt = 0;
        const u32 w0 = lt * WPT;
#pragma unroll
        for (u32 i = 0; i < WPT; ++i) {
            const u32 w = w0 + i;
            sw[i] = (act && w < WORDS) ? __popc(run_starts(gp.bm, w)) : 0u;
            cnt += sw[i];
        }
        const u32 ex = group_excl_scan<G>(cnt, lt, gp.wsum, nruns);
        u32 run = ex;
#pragma unroll
        for (u32 i = 0; i < WPT; ++i) {
            const u32 w = w0 + i;
            if (act && w < WORDS) gp.rpre[w] = u16(run);
            run += sw[i];
        }
    }
    if (act)
        for (u32 r = lt; r < nruns; r += G) par[r] = r;
    gsync<G>();
    // P3: unions with the next column
#pragma unroll
    for (u32 q = 0; q < K; ++q) {
        const u32 lin = LIN[q];
        if (lin != NOPIX) {
            const u32 col = lin / ROWS, row = lin - col * ROWS;
            const u32 r = run_of(gp.bm, gp.rpre, lin);
            AR[q] |= r << 16;
            link_right(par, gp.bm, gp.rpre, lin, row, col, r);
        }
    }
    mid(1);
    gsync<G>();
    // P4: roots; the digi that starts its root's run speaks for the cluster
    u32 starts = 0;
#pragma unroll
    for (u32 q = 0; q < K; ++q) {
        const u32 lin = LIN[q];
        if (lin != NOPIX) {
            const u32 run = AR[q] >> 16;
            const u32 root = uf_find(par, run);
            if (root == run && !((lin % ROWS) > 0 && fired(gp.bm, lin - 1))) starts |= 1u << q;
            AR[q] = (AR[q] & 0xFFFFu) | (root << 16);
        }
    }
    gsync<G>();
    if (act) {
        for (u32 r = lt; r < nruns; r += G) gp.acc[r] = 0ull;
        for (u32 w = lt; w < KBW; w += G) gp.kb[w] = 0u;
    }
    gsync<G>();
    // P5: charge and size per root
#pragma unroll
    for (u32 q = 0; q < K; ++q)
        if (LIN[q] != NOPIX) atomicAdd(&gp.acc[AR[q] >> 16], (1ull << 44) | u64(AR[q] & 0xFFFFu));
    mid(2);
    gsync<G>();
    // P6: charge cut, one bit per kept root
#pragma unroll
    for (u32 q = 0; q < K; ++q)
        if (starts & (1u << q)) {
            const u32 r = AR[q] >> 16;
            if (u32(gp.acc[r]) >= a.charge_cut) atomicOr(&gp.kb[r >> 5], 1u << (r & 31u));
        }
    gsync<G>();
    // P7: kept roots before each kb word
    u32 Kc;
    {
        const u32 c = (act && lt < KBW) ? __popc(gp.kb[lt]) : 0u;
        const u32 ex = group_excl_scan<G>(c, lt, gp.wsum, Kc);
        if (act && lt < KBW) gp.kpre[lt] = u16(ex);
    }
    gsync<G>();
    // P8: kept clusters -> staging records at [st + position in the module]
    if (act) {
        int32_t* tid_ = ws_ptr<int32_t>(E, L.tid);
        int32_t* tch = ws_ptr<int32_t>(E, L.tcharge);
        int32_t* tsz = ws_ptr<int32_t>(E, L.tsize);
        const u32 idbase = I.mod * PIX;
#pragma unroll
        for (u32 q = 0; q < K; ++q)
            if (starts & (1u << q)) {
                const u32 r = AR[q] >> 16;
                const u64 v = gp.acc[r];
                const u32 charge = u32(v), size = u32(v >> 44);
                u32 id = NOPIX;
                if (charge >= a.charge_cut) {
                    const u32 pos = gp.kpre[r >> 5] + __popc(gp.kb[r >> 5] & ((1u << (r & 31u)) - 1u));
                    id = idbase + LIN[q];
                    tid_[I.st + pos] = int32_t(id);
                    tch[I.st + pos] = int32_t(charge);
                    tsz[I.st + pos] = int32_t(size);
                }
                gp.acc[r] = u64(id);
            }
        if (lt == 0) ws_ptr<u32>(E, L.item_kept)[I.it] = Kc;
    }
    mid(3);
    gsync<G>();
    // P9: per-digi cluster id; clear the bitmap words used
    if (act) {
        int32_t* od = ws_ptr<int32_t>(E, L.digi);
#pragma unroll
        for (u32 q = 0; q < K; ++q) {
            const u32 j = lt + q * G;
            if (j < I.n) od[I.st + j] = (LIN[q] != NOPIX) ? int32_t(u32(gp.acc[AR[q] >> 16])) : -1;
        }
#pragma unroll
        for (u32 q = 0; q < K; ++q)
            if (LIN[q] != NOPIX) gp.bm[LIN[q] >> 5] = 0u;
        if (err) atomicOr(ws_ptr<u32>(E, L.ctl) + CTL_ERR, err);
    }
    gsync<G>();
}

// ---------------------------------------------------------------------------
// small: groups of G = WG/MPW threads, one module each, modules by ticket
// ---------------------------------------------------------------------------
template <u32 WG, u32 MPW, u32 K>
struct SmallSmem {
    static constexpr u32 G = WG / MPW;
    RegModuleSmem<G, K> grp[MPW];
    u32 pref[MAXB + 1];
    u32 wsum[WG / 64];
    u32 tick[2];
};

// Resolve position t of the concatenated small lists into a module.  Items that
// fail the consistency checks are reported by the caller.
template <u32 G, u32 K>
__device__ __forceinline__ Item small_item(const LaunchArgs& a, const u32* pref, u32 k, u32 total, u32 t,
                                           EventDesc& E) {
    Item I{0, 0, 0, 0, 0, false};
    if (t >= total) return I;
    I.e = find_slot(pref, k, t);
    E = get_event(a, I.e);
    const EvLayout L = ev_layout(E.cap, a.n_modules);
    I.it = ws_ptr<const u32>(E, L.small)[t - pref[I.e]];
    const u32* item_start = ws_ptr<const u32>(E, L.item_start);
    I.st = item_start[I.it];
    const u32 en = item_start[I.it + 1];
    I.mod = ws_ptr<const u32>(E, L.item_mod)[I.it];
    I.n = en - I.st;
    I.ok = en > I.st && en <= E.n && I.n <= G * K && I.mod < a.n_modules;
    return I;
}

template <u32 WG, u32 MPW, u32 K>
__global__ __launch_bounds__(WG) void k_small(LaunchArgs a) {
    using S = SmallSmem<WG, MPW, K>;
    constexpr u32 G = S::G;
    constexpr bool WAVE = (G == 64);          // groups of one wave run independently
    constexpr u32 STEP = WAVE ? 1u : MPW;     // modules per ticket
    __shared__ S s;
    const u32 tid = threadIdx.x, g = tid / G, lt = tid % G;
    const u32 gofs = WAVE ? 0u : g;
    RegModuleSmem<G, K>& gp = s.grp[g];
    for (u32 w = lt; w < WORDS; w += G) gp.bm[w] = 0u;
    const u32 k = num_events(a);
    const u32 total = event_prefix<WG>(a, k, s.pref, s.wsum, CTL_SMALL, 1, 0);

    // first ticket: a wave draws with lane 0 and broadcasts with readfirstlane; a
    // lockstep workgroup draws MPW modules with thread 0 and broadcasts through LDS
    u32 base;
    if constexpr (WAVE) {
        u32 v = 0;
        if (lt == 0) v = atomicAdd(&a.ctr[S_TICK], 1u);
        base = __builtin_amdgcn_readfirstlane(v);
    } else {
        if (tid == 0) s.tick[0] = atomicAdd(&a.ctr[S_TICK], STEP);
        lds_barrier();
        base = s.tick[0];
    }
    EventDesc E{};
    Item I = small_item<G, K>(a, s.pref, k, total, base + gofs, E);
    u32 LIN[K], A[K];
    if (I.ok) load_digis<G, K>(E, I, lt, LIN, A);

    while (base < total) {
        u32 nbase = total, nv = 0;
        EventDesc En{};
        Item In{0, 0, 0, 0, 0, false};
        u32 NLIN[K], NA[K];
        auto mid = [&](int stage) {
            if (stage == 0) {                      // draw the next ticket
                if constexpr (WAVE) {
                    if (lt == 0) nv = atomicAdd(&a.ctr[S_TICK], 1u);
                } else {
                    if (tid == 0) nv = atomicAdd(&a.ctr[S_TICK], STEP);
                }
            } else if (stage == 1) {               // publish it
                if constexpr (WAVE) nbase = __builtin_amdgcn_readfirstlane(nv);
                else if (tid == 0) s.tick[1] = nv;
            } else if (stage == 2) {               // resolve it
                if constexpr (!WAVE) nbase = s.tick[1];
                In = small_item<G, K>(a, s.pref, k, total, nbase + gofs, En);
            } else {                               // load its digis
                if (In.ok) load_digis<G, K>(En, In, lt, NLIN, NA);
            }
        };
        if (base + gofs < total && !I.ok && lt == 0)
            atomicOr(ws_ptr<u32>(E, ev_layout(E.cap, a.n_modules).ctl) + CTL_ERR, EB_INTERNAL);
        if (!WAVE || I.ok) {
            const EvLayout L = ev_layout(E.cap, a.n_modules);
            cluster_regs<G, K>(a, E, L, I, gp, lt, LIN, A, mid);
        } else {
            mid(0);
            mid(1);
            mid(2);
            mid(3);
        }
        base = nbase;
        E = En;
        I = In;
#pragma unroll
        for (u32 q = 0; q < K; ++q) { LIN[q] = NLIN[q]; A[q] = NA[q]; }
    }
}

// ---------------------------------------------------------------------------
// big: one module per 512-thread workgroup
// ---------------------------------------------------------------------------
// Scratch mode (more than BIG_RCAP digis): up to MAX_RUNS parents in LDS; digis are
// re-read from memory in every phase; per-digi roots and root charges go to global
// scratch that only the same thread reads back (the module's slice of the event's
// final charge/size arrays, which the compaction kernel overwrites later).
struct BigScratchSmem {
    u32 bm[WORDS];
    u32 par[MAX_RUNS];
    u32 kb[MAX_RUNS / 32];
    u16 rpre[WORDS];
    u16 kpre[MAX_RUNS / 32];
    u32 wsum[B_WG / 64];
};
union BigSmem {
    RegModuleSmem<B_WG, K_BIG> reg;
    BigScratchSmem scr;
};

constexpr u32 UNR = 4;                        // digis per thread fetched at once
constexpr u32 SPAN = UNR * B_WG;

__device__ __forceinline__ u32 clampj(u32 j, u32 n) { return j < n ? j : 0u; }

__device__ __forceinline__ void cluster_scratch(const LaunchArgs& a, const EventDesc& E, const EvLayout& L, const Item& I,
                                BigScratchSmem& s) {
    constexpr u32 WPT = (WORDS + B_WG - 1) / B_WG;
    constexpr u32 KW = MAX_RUNS / 32, KPT = (KW + B_WG - 1) / B_WG;
    const u32 tid = threadIdx.x, n = I.n, st = I.st;
    u32* groot = ws_ptr<u32>(E, L.charge) + st;
    u32* gchg = ws_ptr<u32>(E, L.size) + st;
    int32_t* od = ws_ptr<int32_t>(E, L.digi) + st;
    u32 err = 0;
    // UNR digis' linear index (NOPIX when absent or out of range), loads first
    auto fetch = [&](u32 base, u32* lin) {
        u32 r[UNR], c[UNR];
#pragma unroll
        for (u32 u = 0; u < UNR; ++u) {
            const u32 i = st + clampj(base + u * B_WG + tid, n);
            r[u] = E.row[i];
            c[u] = E.col[i];
        }
#pragma unroll
        for (u32 u = 0; u < UNR; ++u) {
            const u32 j = base + u * B_WG + tid;
            lin[u] = (j < n && r[u] < ROWS && c[u] < COLS) ? c[u] * ROWS + r[u] : NOPIX;
            if (j < n && lin[u] == NOPIX) err |= EB_RANGE;
        }
    };
    auto is_root_start = [&](u32 lin, u32 root) {
        return !((lin % ROWS) > 0 && fired(s.bm, lin - 1)) && run_of(s.bm, s.rpre, lin) == root;
    };
    for (u32 base = 0; base < n; base += SPAN) {               // P1: bitmap
        u32 lin[UNR];
        fetch(base, lin);
#pragma unroll
        for (u32 u = 0; u < UNR; ++u)
            if (lin[u] != NOPIX) {
                const u32 bit = 1u << (lin[u] & 31u);
                if (atomicOr(&s.bm[lin[u] >> 5], bit) & bit) err |= EB_DUP;
            }
    }
    lds_barrier();
    u32 nruns;
    {                                                           // P2: runs
        u32 sw[WPT], cnt = 0;
#pragma unroll
        for (u32 i = 0; i < WPT; ++i) {
            const u32 w = tid * WPT + i;
            sw[i] = w < WORDS ? __popc(run_starts(s.bm, w)) : 0u;
            cnt += sw[i];
        }
        u32 run = group_excl_scan<B_WG>(cnt, tid, s.wsum, nruns);
#pragma unroll
        for (u32 i = 0; i < WPT; ++i) {
            const u32 w = tid * WPT + i;
            if (w < WORDS) s.rpre[w] = u16(run);
            run += sw[i];
        }
    }
    for (u32 r = tid; r < nruns; r += B_WG) s.par[r] = r;
    for (u32 w = tid; w < KW; w += B_WG) s.kb[w] = 0u;
    lds_barrier();
    for (u32 base = 0; base < n; base += SPAN) {               // P3: unions
        u32 lin[UNR];
        fetch(base, lin);
#pragma unroll
        for (u32 u = 0; u < UNR; ++u)
            if (lin[u] != NOPIX) {
                const u32 col = lin[u] / ROWS, row = lin[u] - col * ROWS;
                link_right(s.par, s.bm, s.rpre, lin[u], row, col, run_of(s.bm, s.rpre, lin[u]));
            }
    }
    lds_barrier();
    for (u32 base = 0; base < n; base += SPAN) {               // P4: roots to scratch
        u32 lin[UNR];
        fetch(base, lin);
#pragma unroll
        for (u32 u = 0; u < UNR; ++u)
            if (lin[u] != NOPIX) groot[base + u * B_WG + tid] = uf_find(s.par, run_of(s.bm, s.rpre, lin[u]));
    }
    lds_barrier();
    for (u32 r = tid; r < nruns; r += B_WG) s.par[r] = 0u;     // parents -> charge sums
    lds_barrier();
    for (u32 base = 0; base < n; base += SPAN) {               // P5: charge
        u32 lin[UNR], rt[UNR], ad[UNR];
        fetch(base, lin);
#pragma unroll
        for (u32 u = 0; u < UNR; ++u) {
            const u32 jj = clampj(base + u * B_WG + tid, n);
            rt[u] = groot[jj];
            ad[u] = E.adc[st + jj];
        }
#pragma unroll
        for (u32 u = 0; u < UNR; ++u)
            if (lin[u] != NOPIX) atomicAdd(&s.par[rt[u]], ad[u]);
    }
    lds_barrier();
    for (u32 base = 0; base < n; base += SPAN) {               // P6: cut at the root-start digi
        u32 lin[UNR], rt[UNR];
        fetch(base, lin);
#pragma unroll
        for (u32 u = 0; u < UNR; ++u) rt[u] = groot[clampj(base + u * B_WG + tid, n)];
#pragma unroll
        for (u32 u = 0; u < UNR; ++u)
            if (lin[u] != NOPIX && is_root_start(lin[u], rt[u])) {
                const u32 charge = s.par[rt[u]];
                gchg[base + u * B_WG + tid] = charge;
                if (charge >= a.charge_cut) atomicOr(&s.kb[rt[u] >> 5], 1u << (rt[u] & 31u));
            }
    }
    lds_barrier();
    {                                                           // P7: kept roots before each word
        u32 sw[KPT], cnt = 0;
#pragma unroll
        for (u32 i = 0; i < KPT; ++i) {
            const u32 w = tid * KPT + i;
            sw[i] = w < KW ? __popc(s.kb[w]) : 0u;
            cnt += sw[i];
        }
        u32 Kc;
        u32 run = group_excl_scan<B_WG>(cnt, tid, s.wsum, Kc);
#pragma unroll
        for (u32 i = 0; i < KPT; ++i) {
            const u32 w = tid * KPT + i;
            if (w < KW) s.kpre[w] = u16(run);
            run += sw[i];
        }
        if (tid == 0) ws_ptr<u32>(E, L.item_kept)[I.it] = Kc;
    }
    for (u32 r = tid; r < nruns; r += B_WG) s.par[r] = 0u;     // charge sums -> sizes
    lds_barrier();
    for (u32 base = 0; base < n; base += SPAN) {               // P8: sizes
        u32 lin[UNR], rt[UNR];
        fetch(base, lin);
#pragma unroll
        for (u32 u = 0; u < UNR; ++u) rt[u] = groot[clampj(base + u * B_WG + tid, n)];
#pragma unroll
        for (u32 u = 0; u < UNR; ++u)
            if (lin[u] != NOPIX) atomicAdd(&s.par[rt[u]], 1u);
    }
    lds_barrier();
    {                                                           // P9: records; root slot -> id
        int32_t* tid_ = ws_ptr<int32_t>(E, L.tid);
        int32_t* tch = ws_ptr<int32_t>(E, L.tcharge);
        int32_t* tsz = ws_ptr<int32_t>(E, L.tsize);
        for (u32 base = 0; base < n; base += SPAN) {
            u32 lin[UNR], rt[UNR], ch[UNR];
            fetch(base, lin);
#pragma unroll
            for (u32 u = 0; u < UNR; ++u) {
                const u32 jj = clampj(base + u * B_WG + tid, n);
                rt[u] = groot[jj];
                ch[u] = gchg[jj];
            }
#pragma unroll
            for (u32 u = 0; u < UNR; ++u)
                if (lin[u] != NOPIX && is_root_start(lin[u], rt[u])) {
                    const u32 r = rt[u];
                    const u32 size = s.par[r];
                    u32 id = NOPIX;
                    if (ch[u] >= a.charge_cut) {
                        const u32 pos = s.kpre[r >> 5] + __popc(s.kb[r >> 5] & ((1u << (r & 31u)) - 1u));
                        id = I.mod * PIX + lin[u];
                        tid_[st + pos] = int32_t(id);
                        tch[st + pos] = int32_t(ch[u]);
                        tsz[st + pos] = int32_t(size);
                    }
                    s.par[r] = id;
                }
        }
    }
    lds_barrier();
    for (u32 base = 0; base < n; base += SPAN) {               // P10: per-digi ids
        u32 lin[UNR], rt[UNR];
        fetch(base, lin);
#pragma unroll
        for (u32 u = 0; u < UNR; ++u) rt[u] = groot[clampj(base + u * B_WG + tid, n)];
#pragma unroll
        for (u32 u = 0; u < UNR; ++u) {
            const u32 j = base + u * B_WG + tid;
            if (j < n) od[j] = lin[u] != NOPIX ? int32_t(s.par[rt[u]]) : -1;
        }
    }
    if (err) atomicOr(ws_ptr<u32>(E, L.ctl) + CTL_ERR, err);
    for (u32 w = tid; w < WORDS; w += B_WG) s.bm[w] = 0u;
    lds_barrier();
}

__global__ __launch_bounds__(B_WG) void k_big(LaunchArgs a) {
    __shared__ BigSmem s;
    __shared__ u32 s_pref[MAXB + 1];
    __shared__ u32 s_wsum[B_WG / 64];
    const u32 tid = threadIdx.x;
    for (u32 w = tid; w < WORDS; w += B_WG) s.reg.bm[w] = 0u;   // bm leads both layouts
    const u32 k = num_events(a);
    const u32 total = event_prefix<B_WG>(a, k, s_pref, s_wsum, CTL_BIG, 1, 0);
    for (u32 t = blockIdx.x; t < total; t += gridDim.x) {
        Item I{0, 0, 0, 0, 0, false};
        I.e = find_slot(s_pref, k, t);
        const EventDesc E = get_event(a, I.e);
        const EvLayout L = ev_layout(E.cap, a.n_modules);
        I.it = ws_ptr<const u32>(E, L.big)[t - s_pref[I.e]];
        const u32* item_start = ws_ptr<const u32>(E, L.item_start);
        I.st = item_start[I.it];
        const u32 en = item_start[I.it + 1];
        I.mod = ws_ptr<const u32>(E, L.item_mod)[I.it];
        I.n = en - I.st;
        I.ok = en > I.st && en <= E.n && I.mod < a.n_modules;
        if (!I.ok) {
            if (tid == 0) atomicOr(ws_ptr<u32>(E, L.ctl) + CTL_ERR, EB_INTERNAL);
            continue;
        }
        if (I.n <= BIG_RCAP) {
            u32 LIN[K_BIG], A[K_BIG];
            load_digis<B_WG, K_BIG>(E, I, tid, LIN, A);
            cluster_regs<B_WG, K_BIG>(a, E, L, I, s.reg, tid, LIN, A, [](int) {});
        } else {
            cluster_scratch(a, E, L, I, s.scr);
        }
    }
}

// ---------------------------------------------------------------------------
// compact: per event, chunks of C_ITEMS modules; a chunk's offset is the sum of the
// kept counts of all earlier modules; one wave copies one module's records
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(C_WG) void k_compact(LaunchArgs a) {
    __shared__ u32 s_pref[MAXB + 1];
    __shared__ u32 s_wsum[C_WG / 64];
    __shared__ u32 s_off[C_ITEMS + 1];
    __shared__ u32 s_red[C_WG / 64];
    const u32 tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    const u32 k = num_events(a);
    if (blockIdx.x == 0 && tid == 0) st_ag(&a.ctr[S_TICK], 0u);   // the small kernel has finished
    const u32 total = event_prefix<C_WG>(a, k, s_pref, s_wsum, CTL_ITEMS, C_ITEMS, 1);
    for (u32 t = blockIdx.x; t < total; t += gridDim.x) {
        const u32 e = find_slot(s_pref, k, t);
        const u32 c = t - s_pref[e];
        const EventDesc E = get_event(a, e);
        const EvLayout L = ev_layout(E.cap, a.n_modules);
        u32* ctl = ws_ptr<u32>(E, L.ctl);
        const u32 items = E.n ? ctl[CTL_ITEMS] : 0u;
        const u32* kept = ws_ptr<const u32>(E, L.item_kept);
        const u32 i0 = c * C_ITEMS, i1 = min(i0 + C_ITEMS, items);
        u32 part = 0;                                      // kept clusters of items [0, i0)
        for (u32 i = tid; i < i0; i += C_WG) part += kept[i];
        const u32 wtot = __shfl(wave_incl_scan(part), 63, 64);
        if (lane == 0) s_red[wv] = wtot;
        const u32 v = (tid < C_ITEMS && i0 + tid < i1) ? kept[i0 + tid] : 0u;
        const u32 inc = wave_incl_scan(v);                 // offsets inside the chunk (wave 0)
        lds_barrier();
        u32 before = 0;
#pragma unroll
        for (u32 w = 0; w < C_WG / 64; ++w) before += s_red[w];
        if (tid < C_ITEMS) s_off[tid] = before + inc - v;
        if (tid == C_ITEMS - 1) s_off[C_ITEMS] = before + inc;
        lds_barrier();
        const u32* item_start = ws_ptr<const u32>(E, L.item_start);
        const int32_t* tid_ = ws_ptr<const int32_t>(E, L.tid);
        const int32_t* tch = ws_ptr<const int32_t>(E, L.tcharge);
        const int32_t* tsz = ws_ptr<const int32_t>(E, L.tsize);
        int32_t* oid = ws_ptr<int32_t>(E, L.id);
        int32_t* och = ws_ptr<int32_t>(E, L.charge);
        int32_t* osz = ws_ptr<int32_t>(E, L.size);
        for (u32 x = i0 + wv; x < i1; x += C_WG / 64) {
            const u32 off = s_off[x - i0], cnt = s_off[x - i0 + 1] - off;
            const u32 src = item_start[x];
            if (off + cnt > E.n || src + cnt > E.n) continue;   // inconsistent input (flagged)
            for (u32 j = lane; j < cnt; j += 64) {
                const int32_t a0 = tid_[src + j], a1 = tch[src + j], a2 = tsz[src + j];
                oid[off + j] = a0;
                och[off + j] = a1;
                osz[off + j] = a2;
            }
        }
        if (i1 >= items && tid == 0) {                     // the event's last chunk: status
            const u32 ncl = items ? s_off[i1 - i0] : 0u;
            const u32 err = ctl[CTL_ERR];
            ctl[CTL_ERR] = 0u;
            ctl[CTL_NCL] = ncl;
            u32* hs = E.hstat;
            st_sys(&hs[HS_ERR], err);
            st_sys(&hs[HS_NCL], ncl);
            st_sys(&hs[HS_ITEMS], items);
            st_sys(&hs[HS_BIG], E.n ? ctl[CTL_BIG] : 0u);
            st_sys(&hs[HS_EPOCH], E.epoch);
        }
        lds_barrier();
    }
}

// ---------------------------------------------------------------------------
// host-side launch helpers
// ---------------------------------------------------------------------------
typedef void (*SmallKernel)(LaunchArgs);

static SmallKernel small_kernel(u32 wg, u32 mpw) {
    switch (wg * 8 + mpw) {
        case 64 * 8 + 1: return k_small<64, 1, K_SMALL>;
        case 128 * 8 + 1: return k_small<128, 1, K_SMALL>;
        case 128 * 8 + 2: return k_small<128, 2, K_SMALL>;
        case 256 * 8 + 1: return k_small<256, 1, K_SMALL>;
        case 256 * 8 + 2: return k_small<256, 2, K_SMALL>;
        case 256 * 8 + 4: return k_small<256, 4, K_SMALL>;
        case 512 * 8 + 1: return k_small<512, 1, K_SMALL>;
        case 512 * 8 + 2: return k_small<512, 2, K_SMALL>;
        case 512 * 8 + 4: return k_small<512, 4, K_SMALL>;
        default: return nullptr;
    }
}

bool cluster_config_valid(u32 wg, u32 mpw) { return small_kernel(wg, mpw) != nullptr; }
u32 cluster_capacity(u32 wg, u32 mpw) { return (wg / mpw) * K_SMALL; }

static int occ(const void* fn, int bs) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, bs, 0) != hipSuccess || n < 1) n = 1;
    return n;
}

int occupancy_segment() { return occ(reinterpret_cast<const void*>(k_segment), A_WG); }
int occupancy_cluster(u32 wg, u32 mpw) {
    SmallKernel f = small_kernel(wg, mpw);
    return f ? occ(reinterpret_cast<const void*>(f), int(wg)) : 0;
}
int occupancy_big() { return occ(reinterpret_cast<const void*>(k_big), B_WG); }
int occupancy_compact() { return occ(reinterpret_cast<const void*>(k_compact), C_WG); }

hipError_t launch_segment(const LaunchArgs& a, u32 grid, hipStream_t s) {
    hipLaunchKernelGGL(k_segment, dim3(grid), dim3(A_WG), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_small(u32 wg, u32 mpw, const LaunchArgs& a, u32 grid, hipStream_t s) {
    SmallKernel f = small_kernel(wg, mpw);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(grid), dim3(wg), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_big(const LaunchArgs& a, u32 grid, hipStream_t s) {
    hipLaunchKernelGGL(k_big, dim3(grid), dim3(B_WG), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_compact(const LaunchArgs& a, u32 grid, hipStream_t s) {
    hipLaunchKernelGGL(k_compact, dim3(grid), dim3(C_WG), 0, s, a);
    return hipGetLastError();
}

}  // namespace pxcl
