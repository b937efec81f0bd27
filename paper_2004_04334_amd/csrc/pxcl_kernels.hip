// Device kernels of the pixel-clustering path (gfx950 / CDNA4, wave64).
//
// One launch processes k >= 1 events through four persistent kernels that pull
// work with atomic tickets:
//
//   segment   digis -> ordered list of the modules present ("items"), validation.
//   cluster   one module per group of threads: fired-pixel bitmap in LDS, vertical
//             runs, union-find over runs, charge/size per cluster, charge cut, the
//             module's kept clusters in ascending id (written to a per-module
//             staging area) and the per-digi cluster id.
//   large     the same for modules too big for the cluster kernel's LDS budget,
//             one 1024-thread workgroup per module.
//   compact   exclusive scan of kept-cluster counts over each event's modules
//             (single pass, decoupled look-back) and a copy of the staged records
//             to their final ascending-id position; status write-back.
//
// The clustering definition: 8-connected components of fired pixels within a module;
// cluster id = smallest linear index module*66560 + col*160 + row; charge = sum of
// ADC (uint32); keep iff charge >= cut.  This is the "ClusterProducer" work of the
// paper's Figure 1 (Sec. 3).  Errors go to a device error word, never to device
// asserts, which would synchronise (Sec. 4.1).
#include <hip/hip_runtime.h>

#include "pxcl_internal.h"

namespace pxcl {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
constexpr u32 SPIN_LIMIT = 1u << 24;          // bounded waits: ~1 s, then an internal error
constexpr u32 LB_A = 1u << 30, LB_P = 2u << 30, LB_VAL = (1u << 30) - 1;

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
        u32 y = __shfl_up(v, d, 64);
        if (lane >= d) v += y;
    }
    return v;
}

// Exclusive scan over a group of G threads (G a multiple of 64) made of whole waves.
// Every thread of the workgroup must call it (it contains workgroup barriers when
// G > 64).  `wsum` holds G/64 words of LDS private to the group.
template <u32 G>
__device__ __forceinline__ u32 group_excl_scan(u32 v, u32 lt, u32* wsum, u32& total) {
    const u32 inc = wave_incl_scan(v);
    if constexpr (G == 64) {
        total = __shfl(inc, 63, 64);
        return inc - v;
    } else {
        const u32 w = lt >> 6;
        if ((lt & 63u) == 63u) wsum[w] = inc;
        __syncthreads();
        u32 off = 0, tot = 0;
#pragma unroll
        for (u32 i = 0; i < G / 64; ++i) {
            const u32 s = wsum[i];
            off += (i < w) ? s : 0u;
            tot += s;
        }
        __syncthreads();
        total = tot;
        return off + inc - v;
    }
}

// Workgroup-wide exclusive scan (blockDim.x == BS).
template <u32 BS>
__device__ __forceinline__ u32 block_excl_scan(u32 v, u32* wsum, u32& total) {
    return group_excl_scan<BS>(v, threadIdx.x, wsum, total);
}

// Single-pass chained scan with decoupled look-back (Merrill & Garland): publish the
// local aggregate, walk back over predecessors until an inclusive prefix is found,
// publish the inclusive prefix.  Status word: epoch in the high 32 bits, then a
// 2-bit flag (A = aggregate, P = inclusive prefix) and a 30-bit value.  Waits are
// bounded; on expiry the internal-error bit is raised and the scan goes on.
__device__ u32 lookback(u64* st, u32 idx, u32 agg, u32 epoch, u32& err) {
    const u64 tag = u64(epoch) << 32;
    if (idx == 0) {
        st_ag64(&st[0], tag | LB_P | (agg & LB_VAL));
        return 0;
    }
    st_ag64(&st[idx], tag | LB_A | (agg & LB_VAL));
    u32 excl = 0, j = idx - 1, spins = 0;
    for (;;) {
        const u64 v = ld_ag64(&st[j]);
        const u32 lo = u32(v);
        if (u32(v >> 32) != epoch || (lo & (LB_A | LB_P)) == 0) {
            if (++spins > SPIN_LIMIT) { err |= EB_INTERNAL; break; }
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        excl += lo & LB_VAL;
        if (lo & LB_P) break;
        if (j == 0) { err |= EB_INTERNAL; break; }
        --j;
    }
    st_ag64(&st[idx], tag | LB_P | ((excl + agg) & LB_VAL));
    return excl;
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

// Last-workgroup detection; the last one resets the kernel's two counters.
__device__ __forceinline__ bool finish_block(u32* ctr, u32 tick, u32 exitc, u32* s_flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const u32 prev = __hip_atomic_fetch_add(&ctr[exitc], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        *s_flag = (prev == gridDim.x - 1) ? 1u : 0u;
        if (*s_flag) {
            st_ag(&ctr[tick], 0u);
            st_ag(&ctr[exitc], 0u);
        }
    }
    __syncthreads();
    return *s_flag != 0;
}

// ---------------------------------------------------------------------------
// bitmap helpers (column-major: 5 words per column, bit b of word w is row
// (w % 5)*32 + b of column w / 5)
// ---------------------------------------------------------------------------
__device__ __forceinline__ u32 fired(const u32* bm, u32 lin) { return (bm[lin >> 5] >> (lin & 31u)) & 1u; }

// Bits of word w that start a vertical run (fired, with the pixel above not fired).
__device__ __forceinline__ u32 run_starts(const u32* bm, u32 w) {
    const u32 b = bm[w];
    const u32 carry = (w % WPC) ? (bm[w - 1] >> 31) : 0u;
    return b & ~((b << 1) | carry);
}

// Index of the vertical run containing fired pixel lin: run starts strictly before
// word w plus run starts in w at or below bit b, minus one.
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

// Links of fired pixel lin (column col, row row, run r) to the next column.  Pixel
// (row, col) touches (row-1..row+1, col+1).  If (row, col+1) is fired its run
// contains the other two when they are fired; a pixel whose upper neighbour
// (row-1, col) is fired leaves (row-1, col+1) and (row, col+1) to that neighbour.
__device__ __forceinline__ void link_right(u32* par, const u32* bm, const u16* rpre, u32 lin, u32 row,
                                           u32 col, u32 r) {
    if (col + 1 >= COLS) return;
    const bool up = row > 0 && fired(bm, lin - 1);
    const bool m = fired(bm, lin + ROWS);
    if (m) {
        if (!up) uf_unite(par, r, run_of(bm, rpre, lin + ROWS));
        return;
    }
    if (row + 1 < ROWS && fired(bm, lin + ROWS + 1)) uf_unite(par, r, run_of(bm, rpre, lin + ROWS + 1));
    if (!up && row > 0 && fired(bm, lin + ROWS - 1)) uf_unite(par, r, run_of(bm, rpre, lin + ROWS - 1));
}

// ---------------------------------------------------------------------------
// work-item prefix over the events of a launch (items = modules present)
// ---------------------------------------------------------------------------
template <u32 BS>
__device__ __forceinline__ u32 item_prefix(const LaunchArgs& a, u32 k, u32* pref, u32* wsum, u32 which,
                                           u32 div) {
    // which: 0 = items, 1 = large items, 2 = segmentation chunks of the digis;
    // div: items per ticket (rounded up).  Handles any k <= MAXB with any BS.
    u32 carry = 0;
    for (u32 base = 0; base < k; base += BS) {
        const u32 e = base + threadIdx.x;
        u32 v = 0;
        if (e < k) {
            const EventDesc E = get_event(a, e);
            if (E.n) {
                u32 cnt = E.n;
                if (which != 2) {
                    const u32* ctl = ws_ptr<u32>(E, ev_layout(E.cap).ctl);
                    cnt = which == 0 ? ctl[CTL_ITEMS] : ctl[CTL_LARGE];
                }
                v = (cnt + div - 1) / div;
            }
        }
        u32 tot;
        const u32 ex = block_excl_scan<BS>(v, wsum, tot);
        if (e < k) pref[e] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) pref[k] = carry;
    __syncthreads();
    return pref[k];
}

// ---------------------------------------------------------------------------
// segment: module boundaries -> ordered work items; module range/order checks
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(A_WG) void k_segment(LaunchArgs a) {
    __shared__ u32 s_pref[MAXB + 1];
    __shared__ u32 s_wsum[A_WG / 64];
    __shared__ u32 s_tick, s_flag, s_err, s_p;
    const u32 tid = threadIdx.x;
    const u32 k = num_events(a);

    const u32 total = item_prefix<A_WG>(a, k, s_pref, s_wsum, 2, A_CH);

    for (;;) {
        if (tid == 0) { s_tick = atomicAdd(&a.ctr[A_TICK], 1u); s_err = 0; }
        __syncthreads();
        const u32 t = s_tick;
        if (t >= total) break;
        const u32 e = find_slot(s_pref, k, t);
        const u32 c = t - s_pref[e];
        const EventDesc E = get_event(a, e);
        const EvLayout L = ev_layout(E.cap);
        u32* ctl = ws_ptr<u32>(E, L.ctl);
        u32* item_start = ws_ptr<u32>(E, L.item_start);
        u32* item_mod = ws_ptr<u32>(E, L.item_mod);
        const u32 n = E.n;
        const u32 i0 = c * A_CH + tid * A_PER;

        u32 m[A_PER];
#pragma unroll
        for (u32 j = 0; j < A_PER; ++j) m[j] = (i0 + j < n) ? u32(E.module[i0 + j]) : 0u;
        const u32 prev = (i0 > 0 && i0 < n) ? u32(E.module[i0 - 1]) : 0u;

        u32 flags = 0, err = 0;
#pragma unroll
        for (u32 j = 0; j < A_PER; ++j) {
            const u32 i = i0 + j;
            if (i < n) {
                const u32 pm = (j == 0) ? prev : m[j - 1];
                if (i == 0 || m[j] != pm) flags |= 1u << j;
                if (i > 0 && m[j] < pm) err |= EB_ORDER;
                if (m[j] >= a.n_modules) err |= EB_RANGE;
            }
        }
        u32 T;
        const u32 off = block_excl_scan<A_WG>(__popc(flags), s_wsum, T);
        if (err) atomicOr(&s_err, err);
        if (tid == 0) {
            u32 lerr = 0;
            s_p = lookback(ws_ptr<u64>(E, L.lb_a), c, T, E.epoch, lerr);
            if (lerr) atomicOr(&s_err, lerr);
        }
        __syncthreads();
        const u32 P = s_p;
        u32 f = flags, r = P + off;
        if (P + T > n) {                         // only after an expired wait: keep writes in bounds
            f = 0;
            if (tid == 0) atomicOr(&s_err, EB_INTERNAL);
        }
        while (f) {
            const u32 j = __ffs(f) - 1;
            f &= f - 1;
            item_start[r] = i0 + j;
            item_mod[r] = m[j];
            ++r;
        }
        __syncthreads();
        if (tid == 0) {
            if ((c + 1) * A_CH >= n) {           // last chunk of the event
                const u32 items = min(P + T, n);
                ctl[CTL_ITEMS] = items;
                item_start[items] = n;
            }
            if (s_err) atomicOr(&ctl[CTL_ERR], s_err);
        }
        __syncthreads();
    }
    finish_block(a.ctr, A_TICK, A_EXIT, &s_flag);
}

// ---------------------------------------------------------------------------
// cluster: one module per group of G = WG/MPW threads, everything in LDS
// ---------------------------------------------------------------------------
template <u32 WG, u32 MPW>
struct CclSmem {
    static constexpr u32 G = WG / MPW, RCAP = G * K_PER, KBW = RCAP / 32;
    struct Grp {
        u32 bm[WORDS];     // fired-pixel bitmap
        u64 acc[RCAP];     // union-find parents (as u32, first half), then charge | size<<44
        u32 kb[KBW];       // kept-root bits over run index
        u16 rpre[WORDS];   // run starts before each word
        u16 kpre[KBW];     // kept roots before each kb word
        u32 wsum[G / 64];
        u32 misc[4];
    };
    Grp grp[MPW];
    u32 pref[MAXB + 1];
    u32 wsum[WG / 64];
    u32 tick, flag;
};

template <u32 WG, u32 MPW>
__global__ __launch_bounds__(WG) void k_cluster(LaunchArgs a) {
    using S = CclSmem<WG, MPW>;
    constexpr u32 G = S::G, RCAP = S::RCAP, KBW = S::KBW;
    constexpr u32 WPT = (WORDS + G - 1) / G;
    __shared__ S s;
    const u32 tid = threadIdx.x;
    const u32 g = tid / G, lt = tid % G;
    typename S::Grp& gp = s.grp[g];
    u32* par = reinterpret_cast<u32*>(gp.acc);

    for (u32 w = lt; w < WORDS; w += G) gp.bm[w] = 0u;   // bitmap stays clean between items
    const u32 k = num_events(a);
    const u32 total = item_prefix<WG>(a, k, s.pref, s.wsum, 0, 1);

    for (;;) {
        if (tid == 0) s.tick = atomicAdd(&a.ctr[B_TICK], MPW);
        __syncthreads();
        const u32 t0 = s.tick;
        if (t0 >= total) break;
        const u32 t = t0 + g;
        bool act = t < total;
        EventDesc E{};
        EvLayout L{};
        u32 it = 0, st = 0, n = 0, mod = 0;
        if (act) {
            const u32 e = find_slot(s.pref, k, t);
            E = get_event(a, e);
            L = ev_layout(E.cap);
            it = t - s.pref[e];
            const u32* item_start = ws_ptr<u32>(E, L.item_start);
            st = item_start[it];
            n = item_start[it + 1] - st;
            mod = ws_ptr<u32>(E, L.item_mod)[it];
            if (n > RCAP) {                      // too big for this kernel's LDS: defer
                if (lt == 0) {
                    u32* ctl = ws_ptr<u32>(E, L.ctl);
                    const u32 slot = atomicAdd(&ctl[CTL_LARGE], 1u);
                    ws_ptr<u32>(E, L.large)[slot] = it;
                }
                act = false;
            } else if (mod >= a.n_modules) {     // range error already flagged: no clustering
                int32_t* od = ws_ptr<int32_t>(E, L.digi);
                for (u32 j = lt; j < n; j += G) od[st + j] = -1;
                if (lt == 0) ws_ptr<u32>(E, L.item_kept)[it] = 0;
                act = false;
            }
        }

        // P1: insert the module's digis into the bitmap (registers keep lin and adc)
        u32 LIN[K_PER], ADC[K_PER], RT[K_PER];
        u32 err = 0;
#pragma unroll
        for (u32 q = 0; q < K_PER; ++q) {
            LIN[q] = 0xFFFFFFFFu;
            ADC[q] = 0;
            const u32 j = lt + q * G;
            if (act && j < n) {
                const u32 r = E.row[st + j], c = E.col[st + j];
                ADC[q] = E.adc[st + j];
                if (r < ROWS && c < COLS) {
                    const u32 lin = c * ROWS + r;
                    const u32 bit = 1u << (lin & 31u);
                    const u32 old = atomicOr(&gp.bm[lin >> 5], bit);
                    if (old & bit) err |= EB_DUP;
                    LIN[q] = lin;
                } else {
                    err |= EB_RANGE;
                }
            }
        }
        __syncthreads();

        // P2: run starts per word, prefix over words
        u32 R = 0;
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
            const u32 ex = group_excl_scan<G>(cnt, lt, gp.wsum, R);
            u32 run = ex;
#pragma unroll
            for (u32 i = 0; i < WPT; ++i) {
                const u32 w = w0 + i;
                if (act && w < WORDS) gp.rpre[w] = u16(run);
                run += sw[i];
            }
        }
        // P3: parents
        if (act)
            for (u32 r = lt; r < R; r += G) par[r] = r;
        __syncthreads();

        // P4: unions with the next column
#pragma unroll
        for (u32 q = 0; q < K_PER; ++q) {
            const u32 lin = LIN[q];
            if (lin != 0xFFFFFFFFu) {
                const u32 col = lin / ROWS, row = lin - col * ROWS;
                const u32 r = run_of(gp.bm, gp.rpre, lin);
                RT[q] = r;
                link_right(par, gp.bm, gp.rpre, lin, row, col, r);
            }
        }
        __syncthreads();

        // P5: roots; note which digis start their root's run (one per cluster)
        u32 starts = 0;
#pragma unroll
        for (u32 q = 0; q < K_PER; ++q) {
            const u32 lin = LIN[q];
            if (lin != 0xFFFFFFFFu) {
                const u32 root = uf_find(par, RT[q]);
                const u32 row = lin % ROWS;
                if (root == RT[q] && !(row > 0 && fired(gp.bm, lin - 1))) starts |= 1u << q;
                RT[q] = root;
            }
        }
        __syncthreads();
        if (act) {
            for (u32 r = lt; r < R; r += G) gp.acc[r] = 0ull;
            for (u32 w = lt; w < KBW; w += G) gp.kb[w] = 0u;
        }
        __syncthreads();

        // P6: charge and size per root
#pragma unroll
        for (u32 q = 0; q < K_PER; ++q)
            if (LIN[q] != 0xFFFFFFFFu) atomicAdd(&gp.acc[RT[q]], (1ull << 44) | u64(ADC[q]));
        __syncthreads();

        // P7: charge cut, one bit per kept root
#pragma unroll
        for (u32 q = 0; q < K_PER; ++q)
            if (starts & (1u << q)) {
                const u32 r = RT[q];
                if (u32(gp.acc[r]) >= a.charge_cut) atomicOr(&gp.kb[r >> 5], 1u << (r & 31u));
            }
        __syncthreads();

        // P8: kept roots before each kb word
        u32 Kc;
        {
            const u32 c = (act && lt < KBW) ? __popc(gp.kb[lt]) : 0u;
            const u32 ex = group_excl_scan<G>(c, lt, gp.wsum, Kc);
            if (act && lt < KBW) gp.kpre[lt] = u16(ex);
        }
        __syncthreads();

        // P9a: kept clusters -> staging records at [st + position in the module]
        if (act) {
            int32_t* tid_ = ws_ptr<int32_t>(E, L.tid);
            int32_t* tch = ws_ptr<int32_t>(E, L.tcharge);
            int32_t* tsz = ws_ptr<int32_t>(E, L.tsize);
            const u32 idbase = mod * PIX;
#pragma unroll
            for (u32 q = 0; q < K_PER; ++q)
                if (starts & (1u << q)) {
                    const u32 r = RT[q];
                    const u64 v = gp.acc[r];
                    const u32 charge = u32(v), size = u32(v >> 44);
                    u32 id = 0xFFFFFFFFu;
                    if (charge >= a.charge_cut) {
                        const u32 pos = gp.kpre[r >> 5] + __popc(gp.kb[r >> 5] & ((1u << (r & 31u)) - 1u));
                        id = idbase + LIN[q];
                        tid_[st + pos] = int32_t(id);
                        tch[st + pos] = int32_t(charge);
                        tsz[st + pos] = int32_t(size);
                    }
                    gp.acc[r] = u64(id);
                }
            if (lt == 0) ws_ptr<u32>(E, L.item_kept)[it] = Kc;
        }
        __syncthreads();

        // P9b: per-digi cluster id; P10: clear the bitmap words used
        if (act) {
            int32_t* od = ws_ptr<int32_t>(E, L.digi);
#pragma unroll
            for (u32 q = 0; q < K_PER; ++q) {
                const u32 j = lt + q * G;
                if (j < n) od[st + j] = (LIN[q] != 0xFFFFFFFFu) ? int32_t(u32(gp.acc[RT[q]])) : -1;
            }
#pragma unroll
            for (u32 q = 0; q < K_PER; ++q)
                if (LIN[q] != 0xFFFFFFFFu) gp.bm[LIN[q] >> 5] = 0u;
            if (err) atomicOr(ws_ptr<u32>(E, L.ctl) + CTL_ERR, err);
        }
        __syncthreads();
    }
    finish_block(a.ctr, B_TICK, B_EXIT, &s.flag);
}

// ---------------------------------------------------------------------------
// large: one module per 1024-thread workgroup; parents of up to 33,280 runs in
// LDS, charge and size accumulated in global memory, digis re-read per phase
// ---------------------------------------------------------------------------
struct LargeSmem {
    u32 bm[WORDS];
    u32 par[MAX_RUNS];
    u32 kb[MAX_RUNS / 32];
    u16 rpre[WORDS];
    u16 kpre[MAX_RUNS / 32];
    u32 wsum[L_WG / 64];
    u32 pref[MAXB + 1];
    u32 tick, flag, R, Kc;
};

__global__ __launch_bounds__(L_WG) void k_large(LaunchArgs a) {
    __shared__ LargeSmem s;
    constexpr u32 WPT = (WORDS + L_WG - 1) / L_WG;       // 3
    constexpr u32 KPT = (MAX_RUNS / 32 + L_WG - 1) / L_WG;  // 2
    const u32 tid = threadIdx.x;
    for (u32 w = tid; w < WORDS; w += L_WG) s.bm[w] = 0u;
    const u32 k = num_events(a);
    const u32 total = item_prefix<L_WG>(a, k, s.pref, s.wsum, 1, 1);

    for (;;) {
        if (tid == 0) s.tick = atomicAdd(&a.ctr[L_TICK], 1u);
        __syncthreads();
        const u32 t = s.tick;
        if (t >= total) break;
        const u32 e = find_slot(s.pref, k, t);
        const EventDesc E = get_event(a, e);
        const EvLayout L = ev_layout(E.cap);
        const u32 it = ws_ptr<u32>(E, L.large)[t - s.pref[e]];
        const u32* item_start = ws_ptr<u32>(E, L.item_start);
        const u32 st = item_start[it], n = item_start[it + 1] - st;
        const u32 mod = ws_ptr<u32>(E, L.item_mod)[it];
        u32* chg = ws_ptr<u32>(E, L.charge) + st;   // scratch: final outputs are written later
        u32* acc_sz = ws_ptr<u32>(E, L.size) + st;
        int32_t* od = ws_ptr<int32_t>(E, L.digi);
        u32 err = 0;

        if (mod >= a.n_modules) {
            for (u32 j = tid; j < n; j += L_WG) od[st + j] = -1;
            if (tid == 0) ws_ptr<u32>(E, L.item_kept)[it] = 0;
            __syncthreads();
            continue;
        }
        // P1
        for (u32 j = tid; j < n; j += L_WG) {
            const u32 r = E.row[st + j], c = E.col[st + j];
            if (r < ROWS && c < COLS) {
                const u32 lin = c * ROWS + r, bit = 1u << (lin & 31u);
                if (atomicOr(&s.bm[lin >> 5], bit) & bit) err |= EB_DUP;
            } else {
                err |= EB_RANGE;
            }
        }
        __syncthreads();
        // P2
        {
            u32 sw[WPT], cnt = 0;
#pragma unroll
            for (u32 i = 0; i < WPT; ++i) {
                const u32 w = tid * WPT + i;
                sw[i] = w < WORDS ? __popc(run_starts(s.bm, w)) : 0u;
                cnt += sw[i];
            }
            u32 R;
            u32 run = block_excl_scan<L_WG>(cnt, s.wsum, R);
#pragma unroll
            for (u32 i = 0; i < WPT; ++i) {
                const u32 w = tid * WPT + i;
                if (w < WORDS) s.rpre[w] = u16(run);
                run += sw[i];
            }
            if (tid == 0) s.R = R;
        }
        __syncthreads();
        const u32 R = s.R;
        // P3
        for (u32 r = tid; r < R; r += L_WG) {
            s.par[r] = r;
            chg[r] = 0u;
            acc_sz[r] = 0u;
        }
        for (u32 w = tid; w < MAX_RUNS / 32; w += L_WG) s.kb[w] = 0u;
        __threadfence();
        __syncthreads();
        // P4
        for (u32 j = tid; j < n; j += L_WG) {
            const u32 r = E.row[st + j], c = E.col[st + j];
            if (r < ROWS && c < COLS) {
                const u32 lin = c * ROWS + r;
                link_right(s.par, s.bm, s.rpre, lin, r, c, run_of(s.bm, s.rpre, lin));
            }
        }
        __syncthreads();
        // P5 + P6: roots, charge and size
        for (u32 j = tid; j < n; j += L_WG) {
            const u32 r = E.row[st + j], c = E.col[st + j];
            if (r < ROWS && c < COLS) {
                const u32 root = uf_find(s.par, run_of(s.bm, s.rpre, c * ROWS + r));
                atomicAdd(&chg[root], u32(E.adc[st + j]));
                atomicAdd(&acc_sz[root], 1u);
            }
        }
        __threadfence();
        __syncthreads();
        // P7: cut
        for (u32 j = tid; j < n; j += L_WG) {
            const u32 r = E.row[st + j], c = E.col[st + j];
            if (r < ROWS && c < COLS) {
                const u32 lin = c * ROWS + r;
                const u32 run = run_of(s.bm, s.rpre, lin);
                if (!(r > 0 && fired(s.bm, lin - 1)) && uf_find(s.par, run) == run)
                    if (ld_ag(&chg[run]) >= a.charge_cut) atomicOr(&s.kb[run >> 5], 1u << (run & 31u));
            }
        }
        __syncthreads();
        // P8
        {
            u32 sw[KPT], cnt = 0;
#pragma unroll
            for (u32 i = 0; i < KPT; ++i) {
                const u32 w = tid * KPT + i;
                sw[i] = w < MAX_RUNS / 32 ? __popc(s.kb[w]) : 0u;
                cnt += sw[i];
            }
            u32 Kc;
            u32 run = block_excl_scan<L_WG>(cnt, s.wsum, Kc);
#pragma unroll
            for (u32 i = 0; i < KPT; ++i) {
                const u32 w = tid * KPT + i;
                if (w < MAX_RUNS / 32) s.kpre[w] = u16(run);
                run += sw[i];
            }
            if (tid == 0) s.Kc = Kc;
        }
        __syncthreads();
        // P9a: records; the root's size slot then holds the cluster id (or -1)
        {
            int32_t* tid_ = ws_ptr<int32_t>(E, L.tid);
            int32_t* tch = ws_ptr<int32_t>(E, L.tcharge);
            int32_t* tsz = ws_ptr<int32_t>(E, L.tsize);
            for (u32 j = tid; j < n; j += L_WG) {
                const u32 r = E.row[st + j], c = E.col[st + j];
                if (r < ROWS && c < COLS) {
                    const u32 lin = c * ROWS + r;
                    const u32 run = run_of(s.bm, s.rpre, lin);
                    if (!(r > 0 && fired(s.bm, lin - 1)) && uf_find(s.par, run) == run) {
                        const u32 charge = ld_ag(&chg[run]), size = ld_ag(&acc_sz[run]);
                        u32 id = 0xFFFFFFFFu;
                        if (charge >= a.charge_cut) {
                            const u32 pos = s.kpre[run >> 5] + __popc(s.kb[run >> 5] & ((1u << (run & 31u)) - 1u));
                            id = mod * PIX + lin;
                            tid_[st + pos] = int32_t(id);
                            tch[st + pos] = int32_t(charge);
                            tsz[st + pos] = int32_t(size);
                        }
                        st_ag(&acc_sz[run], id);
                    }
                }
            }
            if (tid == 0) ws_ptr<u32>(E, L.item_kept)[it] = s.Kc;
        }
        __threadfence();
        __syncthreads();
        // P9b
        for (u32 j = tid; j < n; j += L_WG) {
            const u32 r = E.row[st + j], c = E.col[st + j];
            int32_t v = -1;
            if (r < ROWS && c < COLS) {
                const u32 root = uf_find(s.par, run_of(s.bm, s.rpre, c * ROWS + r));
                v = int32_t(ld_ag(&acc_sz[root]));
            }
            od[st + j] = v;
        }
        if (err) atomicOr(ws_ptr<u32>(E, L.ctl) + CTL_ERR, err);
        __syncthreads();
        for (u32 w = tid; w < WORDS; w += L_WG) s.bm[w] = 0u;
        __syncthreads();
    }
    finish_block(a.ctr, L_TICK, L_EXIT, &s.flag);
}

// ---------------------------------------------------------------------------
// compact: per event, exclusive scan of kept counts over items (in module order)
// and copy of the staged records; the last workgroup writes the host status.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(C_WG) void k_compact(LaunchArgs a) {
    __shared__ u32 s_pref[MAXB + 1];
    __shared__ u32 s_wsum[C_WG / 64];
    __shared__ u32 s_loff[C_CH];
    __shared__ u32 s_src[C_CH];
    __shared__ u32 s_tick, s_flag, s_p;
    const u32 tid = threadIdx.x;
    const u32 k = num_events(a);
    const u32 total = item_prefix<C_WG>(a, k, s_pref, s_wsum, 0, C_CH);

    for (;;) {
        if (tid == 0) s_tick = atomicAdd(&a.ctr[C_TICK], 1u);
        __syncthreads();
        const u32 t = s_tick;
        if (t >= total) break;
        const u32 e = find_slot(s_pref, k, t);
        const u32 c = t - s_pref[e];
        const EventDesc E = get_event(a, e);
        const EvLayout L = ev_layout(E.cap);
        u32* ctl = ws_ptr<u32>(E, L.ctl);
        const u32 items = ctl[CTL_ITEMS];
        const u32 i = c * C_CH + tid;
        const u32 kept = i < items ? ws_ptr<u32>(E, L.item_kept)[i] : 0u;
        const u32 src = i < items ? ws_ptr<u32>(E, L.item_start)[i] : 0u;
        u32 T;
        const u32 off = block_excl_scan<C_WG>(kept, s_wsum, T);
        s_loff[tid] = off;
        s_src[tid] = src;
        if (tid == 0) {
            u32 lerr = 0;
            s_p = lookback(ws_ptr<u64>(E, L.lb_c), c, T, E.epoch, lerr);
            if (lerr) atomicOr(&ctl[CTL_ERR], lerr);
        }
        __syncthreads();
        const u32 P = s_p;
        const u32 nloc = min(C_CH, items - c * C_CH);
        const u32 Tw = (P + T <= E.n) ? T : 0u;  // only after an expired wait: keep writes in bounds
        const int32_t* tid_ = ws_ptr<int32_t>(E, L.tid);
        const int32_t* tch = ws_ptr<int32_t>(E, L.tcharge);
        const int32_t* tsz = ws_ptr<int32_t>(E, L.tsize);
        int32_t* oid = ws_ptr<int32_t>(E, L.id);
        int32_t* och = ws_ptr<int32_t>(E, L.charge);
        int32_t* osz = ws_ptr<int32_t>(E, L.size);
        for (u32 j = tid; j < Tw; j += C_WG) {
            const u32 x = find_slot(s_loff, nloc, j);   // last item with loff <= j
            const u32 from = s_src[x] + (j - s_loff[x]);
            oid[P + j] = tid_[from];
            och[P + j] = tch[from];
            osz[P + j] = tsz[from];
        }
        if (tid == 0 && (c + 1) * C_CH >= items) st_ag(&ctl[CTL_NCL], P + T);
        __syncthreads();
    }
    if (finish_block(a.ctr, C_TICK, C_EXIT, &s_flag)) {
        // all workgroups are done: status write-back for every event
        for (u32 e = tid; e < k; e += C_WG) {
            const EventDesc E = get_event(a, e);
            u32* ctl = ws_ptr<u32>(E, ev_layout(E.cap).ctl);
            const u32 items = E.n ? ld_ag(&ctl[CTL_ITEMS]) : 0u;
            const u32 ncl = items ? ld_ag(&ctl[CTL_NCL]) : 0u;
            const u32 err = __hip_atomic_exchange(&ctl[CTL_ERR], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const u32 large = ld_ag(&ctl[CTL_LARGE]);
            st_ag(&ctl[CTL_LARGE], 0u);
            u32* hs = E.hstat;
            hs[HS_ERR] = err;
            hs[HS_NCL] = ncl;
            hs[HS_ITEMS] = items;
            hs[HS_LARGE] = large;
            __threadfence_system();
            __hip_atomic_store(&hs[HS_EPOCH], E.epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        __threadfence_system();
    }
}

// ---------------------------------------------------------------------------
// host-side launch helpers
// ---------------------------------------------------------------------------
typedef void (*ClusterKernel)(LaunchArgs);

static ClusterKernel cluster_kernel(u32 wg, u32 mpw) {
    switch (wg * 8 + mpw) {
        case 64 * 8 + 1: return k_cluster<64, 1>;
        case 128 * 8 + 1: return k_cluster<128, 1>;
        case 128 * 8 + 2: return k_cluster<128, 2>;
        case 256 * 8 + 1: return k_cluster<256, 1>;
        case 256 * 8 + 2: return k_cluster<256, 2>;
        case 256 * 8 + 4: return k_cluster<256, 4>;
        case 512 * 8 + 1: return k_cluster<512, 1>;
        case 512 * 8 + 2: return k_cluster<512, 2>;
        case 512 * 8 + 4: return k_cluster<512, 4>;
        default: return nullptr;
    }
}

bool cluster_config_valid(u32 wg, u32 mpw) { return cluster_kernel(wg, mpw) != nullptr; }
u32 cluster_capacity(u32 wg, u32 mpw) { return (wg / mpw) * K_PER; }

static int occ(const void* fn, int bs) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, bs, 0) != hipSuccess || n < 1) n = 1;
    return n;
}

int occupancy_segment() { return occ(reinterpret_cast<const void*>(k_segment), A_WG); }
int occupancy_cluster(u32 wg, u32 mpw) {
    ClusterKernel f = cluster_kernel(wg, mpw);
    return f ? occ(reinterpret_cast<const void*>(f), int(wg)) : 0;
}
int occupancy_large() { return occ(reinterpret_cast<const void*>(k_large), L_WG); }
int occupancy_compact() { return occ(reinterpret_cast<const void*>(k_compact), C_WG); }

hipError_t launch_segment(const LaunchArgs& a, u32 grid, hipStream_t s) {
    hipLaunchKernelGGL(k_segment, dim3(grid), dim3(A_WG), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_cluster(u32 wg, u32 mpw, const LaunchArgs& a, u32 grid, hipStream_t s) {
    ClusterKernel f = cluster_kernel(wg, mpw);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(grid), dim3(wg), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_large(const LaunchArgs& a, u32 grid, hipStream_t s) {
    hipLaunchKernelGGL(k_large, dim3(grid), dim3(L_WG), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_compact(const LaunchArgs& a, u32 grid, hipStream_t s) {
    hipLaunchKernelGGL(k_compact, dim3(grid), dim3(C_WG), 0, s, a);
    return hipGetLastError();
}

}  // namespace pxcl
