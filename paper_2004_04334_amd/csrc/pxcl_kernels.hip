// Device kernels of the pixel-clustering path (gfx950 / CDNA4, wave64).
//
// One launch processes k >= 1 events through these kernels, in this order:
//
//   segment  (batches) streams the module ids; every digi at a module boundary
//            writes the module's entry of a per-module table (first digi, one past
//            the last, tagged with the launch), module starts go to a list of the
//            modules present; checks module range and order.  A single-event
//            launch has no segmentation kernel: the small kernel finds each
//            module's digis by search and checks the ids itself.
//   small    one module per group of threads (a single wave, or a whole
//            workgroup): fired-pixel bitmap in LDS, vertical runs, union-find over
//            runs, charge/size per cluster, charge cut; the module's kept clusters
//            go in ascending id to a staging area at the module's first digi, and
//            every digi gets its cluster id.  Modules above the group's capacity go
//            to the big-module or the scratch-mode list.  Groups take modules by
//            static rounds, then an atomic ticket, and prefetch the next module
//            while working on the current one.
//   big      one listed module per 512-thread workgroup, digis held in registers
//            (up to 16,384 per module).
//   scratch  one listed module above 16,384 digis per 1,024-thread workgroup, the
//            digis re-read from memory in three passes.
//   compact  a wave per module: the offset of its clusters (the kept counts of the
//            modules before it) and a copy of its staged records to their final
//            position; a wave per event writes the status back to the host.
//
// On demand, after a launch: hits, the charge-weighted centroid of every kept
// cluster.
//
// The clustering: 8-connected components of fired pixels within a module; cluster
// id = smallest linear index module*66560 + col*160 + row; charge = sum of ADC
// (uint32); keep iff charge >= cut.  This is the "ClusterProducer" step of the
// paper's Figure 1 (Sec. 3).  Errors go to a device error word, never to device
// asserts, which would synchronise (Sec. 4.1).
//
// Memory ordering.  Workgroup barriers here order LDS only (global loads and stores
// stay in flight across them).  No workgroup reads what another workgroup of the same
// kernel writes: data crosses kernel boundaries, and the only device-scope atomics
// are counters whose returned values serve as indexes (tickets, list places).  No
// device-scope release/acquire fence is used: on gfx950 those write back and
// invalidate the L2.
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
// Digis in any order: the input position of grouped digi p is perm[p]; per-digi
// outputs go there.  nullptr when the digis came grouped (position p itself).
__device__ __forceinline__ const u32* perm_of(const EventDesc& E, const EvLayout& L) {
    return (E.flags & EF_UNSORTED) ? ws_ptr<const u32>(E, L.perm) : nullptr;
}
__device__ __forceinline__ u32 out_pos(const u32* perm, u32 p) { return perm ? perm[p] : p; }

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

// What event_prefix counts per event: its digis (CNT_DIGIS), the digis of an event
// grouped by module (CNT_SORTED: zero for digis in any order) or in any order
// (CNT_ANY: zero for grouped ones), the modules per event, its work units.
constexpr u32 CNT_DIGIS = 0, CNT_MODULES = 0xFFFFFFFFu, CNT_UNITS = 0xFFFFFFFEu, CNT_SORTED = 0xFFFFFFFDu,
              CNT_ANY = 0xFFFFFFFCu;

// Modules on the event's present-module list.
__device__ __forceinline__ u32 present_count(const LaunchArgs& a, const EventDesc& E) {
    return min(ld_ag(ws_ptr<const u32>(E, ev_layout(E.cap, a.n_modules).ctl) + CTL_PRESENT + (E.slot & 1u)), a.n_modules);
}

// Work units of the kernels after segmentation: when most modules are present, every
// module (unit j is module j; an absent one is recognised by its table entry), else
// the present-module list (unit j is its entry j, one more load away).
__device__ __forceinline__ bool dense_units(const LaunchArgs& a, u32 present) { return 2 * present > a.n_modules; }
__device__ __forceinline__ u32 unit_count(const LaunchArgs& a, const EventDesc& E) {
    if (!E.n) return 0u;
    const u32 p = present_count(a, E);
    return dense_units(a, p) ? a.n_modules : p;
}
__device__ __forceinline__ u32 unit_module(const LaunchArgs& a, const EventDesc& E, const EvLayout& L, u32 units,
                                           u32 j) {
    if (units == a.n_modules) return j;         // dense (a list as long as the module count is all of them)
    return min(ws_ptr<const u32>(E, L.present)[j], a.n_modules - 1);
}

// Prefix over the events of a launch of max(ceil(count / div), at_least) + plus,
// where count is the event's digis (CNT_DIGIS), the modules per event
// (CNT_MODULES), its work units (CNT_UNITS) or one of its control words (CTL_*, at
// most the modules per event); 0 for an empty event.  pref[k] = total.
// Every thread of the workgroup calls it; any k <= MAXB with any BS.
template <u32 BS>
__device__ __forceinline__ u32 event_prefix(const LaunchArgs& a, u32 k, u32* pref, u32* wsum, u32 which, u32 div,
                                            u32 at_least, u32 plus = 0) {
    u32 carry = 0;
    for (u32 base = 0; base < k; base += BS) {
        const u32 e = base + threadIdx.x;
        u32 v = 0;
        if (e < k) {
            const EventDesc E = get_event(a, e);
            u32 cnt = 0;
            if (E.n)
                cnt = which == CNT_DIGIS     ? E.n
                      : which == CNT_SORTED  ? ((E.flags & EF_UNSORTED) ? 0u : E.n)
                      : which == CNT_ANY     ? ((E.flags & EF_UNSORTED) ? E.n : 0u)
                      : which == CNT_MODULES ? a.n_modules
                      : which == CNT_UNITS   ? unit_count(a, E)
                                             : min(ld_ag(ws_ptr<u32>(E, ev_layout(E.cap, a.n_modules).ctl) + which), a.n_modules);
            v = max((cnt + div - 1) / div, at_least) + plus;
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

constexpr u32 NOPIX = 0xFFFFFFFFu;          // no pixel / no index

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

// Links (pairs of runs to unite) found by a group are listed in LDS first and united
// afterwards, evenly over the group: a lane that finds several would otherwise unite
// them one after another while the rest of its wave waits.  A link that does not fit
// the list (capacity cap) is united at once.
__device__ __forceinline__ void put_link(u32* list, u32 cap, u32* par, u32 pos, u32 a, u32 b) {
    if (pos < cap) list[pos] = (a << 16) | b;
    else uf_unite(par, a, b);
}

// Run index of row bit j of word w (fired), given the word's run starts s and the run
// starts before it r0: runs are numbered in column-major order of their first pixel.
__device__ __forceinline__ u32 run_at(u32 r0, u32 s, u32 j) { return r0 + __popc(s & ((2u << j) - 1u)) - 1u; }

// Links between the runs of columns c and c+1 that meet rows 32k..32k+31 of them (both
// columns hold a fired pixel, their run prefixes are set).  Rule B: every run start of
// column c+1 is linked to the run of column c that holds the first fired pixel of the
// start's rows -1..+1.  Rule A: every run start q of column c is linked to the run of
// column c+1 holding the first fired pixel of rows q-1..q+1, when rule B does not
// already make that link, which is when that pixel is at row q-1 and row q-2 is fired
// in either column.  Every pair of touching runs X (column c+1), Y (column c) is linked
// this way: if X's start lies within Y's rows widened by one, rule B links X to Y, or
// to a run of column c ending right above X's start, and then Y starts just below
// X's start, within one row of it, and rule A links Y to X; otherwise Y starts inside
// X's rows widened by one, and rule A (or rule B for X, when X starts one row below
// Y's start) links them.  Everything about the two columns comes from six bitmap
// words and four run prefixes read once; only the unions touch the parents.
__device__ __forceinline__ void link_word(u32* par, u32* list, u32 cap, u32* nlink, const u32* bm, const u16* rpre,
                                          u32 c, u32 k) {
    const u32 wa = c * WPC + k, wb = wa + WPC;
    const bool has_prev = k > 0, has_next = k + 1 < WPC;
    const u32 a = bm[wa], b = bm[wb];
    const u32 pa = has_prev ? bm[wa - 1] : 0u, pb = has_prev ? bm[wb - 1] : 0u;   // rows 32k-32..32k-1
    const u32 ap = pa >> 31, bp = pb >> 31;                                        // row 32k-1
    const u32 an = has_next ? bm[wa + 1] & 1u : 0u;                                // row 32k+32
    const u32 sa = a & ~((a << 1) | ap), sb = b & ~((b << 1) | bp);
    // bit i of x_up / x_up2 / x_dn: the column fired at row i-1 / i-2 / i+1 of this word
    const u32 a_up = (a << 1) | ap, a_dn = (a >> 1) | (an << 31), a_up2 = (a << 2) | (pa >> 30);
    const u32 b_up = (b << 1) | bp, b_up2 = (b << 2) | (pb >> 30);
    u32 ma = sa & b_up & (a_up2 | b_up2), mb = sb & (a_up | a | a_dn);
    if (!(ma | mb)) return;
    const u32 ra0 = rpre[wa], rb0 = rpre[wb];
    const u32 ra1 = has_next ? rpre[wa + 1] : 0u;
    // run of the other column (bits x, starts s, prefixes r0 / r1 of this word and the
    // next) holding its first fired pixel among rows i-1, i, i+1
    auto first_run = [](u32 i, u32 x, u32 x_up, u32 s, u32 r0, u32 r1) -> u32 {
        if ((x_up >> i) & 1u) return i ? run_at(r0, s, i - 1) : r0 - 1u;   // row 32k-1: the last run before the word
        if ((x >> i) & 1u) return run_at(r0, s, i);
        return i < 31 ? run_at(r0, s, i + 1) : r1;   // row 32k+32 starts a run (row 32k+31 is empty)
    };
    u32 pos = atomicAdd(nlink, u32(__popc(mb) + __popc(ma)));
    while (mb) {                                     // starts in column c+1
        const u32 i = __builtin_ctz(mb);
        mb &= mb - 1u;
        put_link(list, cap, par, pos++, run_at(rb0, sb, i), first_run(i, a, a_up, sa, ra0, ra1));
    }
    while (ma) {                                     // starts in column c (row i-1 fired in c+1)
        const u32 i = __builtin_ctz(ma);
        ma &= ma - 1u;
        put_link(list, cap, par, pos++, run_at(ra0, sa, i), i ? run_at(rb0, sb, i - 1) : rb0 - 1u);
    }
}

// The same two rules for one column pair (c, c+1) by one wave, a lane per row (rows
// lane, lane + 64, lane + 128): the scratch mode's walk over the columns.  The ten
// words of the two columns and their run prefixes are read once per step (load_pair,
// issued one step ahead), the rest is register work and the unions.
struct ColPair {
    u32 A[WPC], B[WPC], RA[WPC], RB[WPC];
};
__device__ __forceinline__ void load_pair(ColPair& P, const u32* bm, const u16* rpre, u32 c) {
#pragma unroll
    for (u32 k = 0; k < WPC; ++k) {
        P.A[k] = bm[c * WPC + k];
        P.B[k] = bm[(c + 1) * WPC + k];
        P.RA[k] = rpre[c * WPC + k];
        P.RB[k] = rpre[(c + 1) * WPC + k];
    }
}
__device__ __forceinline__ u32 sel5(const u32 (&v)[WPC], u32 k) {
    return k == 0 ? v[0] : k == 1 ? v[1] : k == 2 ? v[2] : k == 3 ? v[3] : v[4];
}
__device__ __forceinline__ void link_pair(u32* par, const ColPair& P, u32 lane) {
    u32 any = 0;
#pragma unroll
    for (u32 k = 0; k < WPC; ++k) any |= P.A[k] | P.B[k];
    if (!any) return;                                // the same for the whole wave
    u32 SA[WPC], SB[WPC];
#pragma unroll
    for (u32 k = 0; k < WPC; ++k) {
        SA[k] = P.A[k] & ~((P.A[k] << 1) | (k ? P.A[k - 1] >> 31 : 0u));
        SB[k] = P.B[k] & ~((P.B[k] << 1) | (k ? P.B[k - 1] >> 31 : 0u));
    }
    auto bit = [](const u32 (&W)[WPC], u32 row) -> u32 {   // fired at row (any u32: out of range = 0)
        return row < ROWS ? (sel5(W, row >> 5) >> (row & 31u)) & 1u : 0u;
    };
    auto run = [](const u32 (&S)[WPC], const u32 (&R)[WPC], u32 row) -> u32 {
        return run_at(sel5(R, row >> 5), sel5(S, row >> 5), row & 31u);
    };
#pragma unroll
    for (u32 j = 0; j < 3; ++j) {
        const u32 p = lane + 64u * j;
        if (p >= ROWS) break;
        if (bit(SB, p)) {                            // rule B
            const u32 f = bit(P.A, p - 1u) ? p - 1u : bit(P.A, p) ? p : bit(P.A, p + 1u) ? p + 1u : NOPIX;
            if (f != NOPIX) uf_unite(par, run(SB, P.RB, p), run(SA, P.RA, f));
        }
        if (bit(SA, p) && bit(P.B, p - 1u) && (bit(P.A, p - 2u) | bit(P.B, p - 2u)))   // rule A
            uf_unite(par, run(SA, P.RA, p), run(SB, P.RB, p - 1u));
    }
}

// ---------------------------------------------------------------------------
// group (digis in any order): a counting sort by module ahead of the clustering,
// which then reads a grouped copy in the event workspace and writes every per-digi
// output at the digi's input position (perm).  Three kernels:
//   count    per chunk of G_CH digis an LDS histogram over the modules gives each
//            digi its rank among the chunk's digis of its module; one device atomic
//            per (chunk, module present in it) adds the chunk's count to the module's
//            total and returns the chunk's base, so a digi's rank in its module is
//            base + local rank.  The rank is parked in the per-digi output word (the
//            clustering overwrites it).  Module ids at or above the module count set
//            EB_RANGE and the digi takes no part.
//   table    one workgroup per event: an exclusive scan of the module totals gives
//            each module its first grouped position; module-table entries tagged with
//            the launch, the present-module list in ascending module order, kept
//            counts and totals cleared -- the segmentation kernel's outputs.
//   scatter  every digi goes to first[module] + rank of the grouped copy, and its
//            input position to perm.
// A digi's place within its module is not fixed (chunks take their bases in any
// order); the clustering does not depend on it.
// ---------------------------------------------------------------------------
constexpr u32 G_WG = 256, G_PER = 16, G_CH = G_WG * G_PER, G_HMAX = 4096, G_TPM = 8;
constexpr u32 G_SPER = 4, G_SCH = G_WG * G_SPER;   // scatter: smaller chunks, more workgroups

struct GroupArrays {
    u16 *m, *r, *c, *a;
    u32* perm;
};
__device__ __forceinline__ GroupArrays group_arrays(const EventDesc& E, const EvLayout& L) {
    u16* g = ws_ptr<u16>(E, L.grp);
    const size_t N = E.cap;
    return GroupArrays{g, g + N, g + 2 * N, g + 3 * N, ws_ptr<u32>(E, L.perm)};
}

__global__ __launch_bounds__(G_WG) void k_group_count(LaunchArgs a) {
    __shared__ u32 hist[G_HMAX];
    __shared__ u32 s_pref[MAXB + 1];
    __shared__ u32 s_wsum[G_WG / 64];
    __shared__ u32 s_err;
    const u32 tid = threadIdx.x, k = num_events(a), M = a.n_modules;
    const bool lds = M <= G_HMAX;                 // else ranks straight from the totals
    const u32 total = event_prefix<G_WG>(a, k, s_pref, s_wsum, CNT_ANY, G_CH, 0);
    // the small kernel's ticket starts at zero (segmentation, which also resets it,
    // is not launched when every event of the launch is in any order)
    if (blockIdx.x == 0 && tid == 0) st_ag(&a.ctr[S_TICK], 0u);
    for (u32 t = blockIdx.x; t < total; t += gridDim.x) {
        const u32 e = find_slot(s_pref, k, t), c = t - s_pref[e];
        const EventDesc E = get_event(a, e);
        const EvLayout L = ev_layout(E.cap, M);
        u32* gcnt = ws_ptr<u32>(E, L.gcnt);
        u32* rank = reinterpret_cast<u32*>(E.o_digi);
        if (tid == 0) s_err = 0;
        if (lds)
            for (u32 m = tid; m < M; m += G_WG) hist[m] = 0u;
        lds_barrier();
        const u32 i0 = c * G_CH + tid;
        u32 mm[G_PER], lr[G_PER];
#pragma unroll
        for (u32 q = 0; q < G_PER; ++q) {
            const u32 i = i0 + q * G_WG;
            mm[q] = i < E.n ? u32(E.r_module[i]) : NOPIX;
        }
        u32 err = 0;
#pragma unroll
        for (u32 q = 0; q < G_PER; ++q) {
            lr[q] = 0u;
            if (mm[q] == NOPIX) continue;
            if (mm[q] >= M) {
                err |= EB_RANGE;
                mm[q] = NOPIX;
            } else {
                lr[q] = lds ? atomicAdd(&hist[mm[q]], 1u) : atomicAdd(&gcnt[mm[q]], 1u);
            }
        }
        lds_barrier();
        if (lds) {                                // the chunk's bases: independent atomics, all in flight
            constexpr u32 FL = G_HMAX / G_WG;
            u32 h[FL];
#pragma unroll
            for (u32 j = 0; j < FL; ++j) {
                const u32 m = tid + j * G_WG;
                h[j] = m < M ? hist[m] : 0u;
            }
#pragma unroll
            for (u32 j = 0; j < FL; ++j)
                if (h[j]) h[j] = atomicAdd(&gcnt[tid + j * G_WG], h[j]);
#pragma unroll
            for (u32 j = 0; j < FL; ++j)
                if (tid + j * G_WG < M) hist[tid + j * G_WG] = h[j];
        }
        lds_barrier();
#pragma unroll
        for (u32 q = 0; q < G_PER; ++q)
            if (mm[q] != NOPIX) rank[i0 + q * G_WG] = (lds ? hist[mm[q]] : 0u) + lr[q];
        if (err) atomicOr(&s_err, err);
        lds_barrier();
        if (tid == 0 && s_err) atomicOr(ws_ptr<u32>(E, L.ctl) + CTL_ERR, s_err);
        lds_barrier();                            // hist and s_err are reused by the next chunk
    }
}

__global__ __launch_bounds__(G_WG) void k_group_table(LaunchArgs a) {
    __shared__ u32 s_wsum[G_WG / 64];
    const u32 tid = threadIdx.x, k = num_events(a), M = a.n_modules;
    for (u32 e = blockIdx.x; e < k; e += gridDim.x) {
        const EventDesc E = get_event(a, e);
        if (!(E.flags & EF_UNSORTED)) continue;  // the same event for the whole workgroup
        const EvLayout L = ev_layout(E.cap, M);
        u32* gcnt = ws_ptr<u32>(E, L.gcnt);
        u32* kept = ws_ptr<u32>(E, L.kept);
        u32* present = ws_ptr<u32>(E, L.present);
        u32* ctl = ws_ptr<u32>(E, L.ctl);
        ModRange* mt = ws_ptr<ModRange>(E, L.mtab);
        const u64 tag = u64(E.epoch) << 32;
        u32 carry = 0, pcarry = 0;
        for (u32 base = 0; base < M; base += G_WG * G_TPM) {
            const u32 m0 = base + tid * G_TPM;   // this thread's G_TPM consecutive modules
            u32 cnt[G_TPM], sum = 0, pres = 0;
#pragma unroll
            for (u32 j = 0; j < G_TPM; ++j) {
                cnt[j] = (m0 + j < M && E.n) ? gcnt[m0 + j] : 0u;
                sum += cnt[j];
                pres += cnt[j] ? 1u : 0u;
            }
            u32 tot, ptot;
            const u32 ex = group_excl_scan<G_WG>(sum, tid, s_wsum, tot);
            const u32 pex = group_excl_scan<G_WG>(pres, tid, s_wsum, ptot);
            u32 pos = carry + ex, pp = pcarry + pex;
#pragma unroll
            for (u32 j = 0; j < G_TPM; ++j) {
                const u32 m = m0 + j;
                if (m >= M) break;
                if (cnt[j]) {
                    const u32 end = pos + cnt[j];
                    if (end <= E.n) mt[m] = ModRange{tag | pos, tag | end};
                    else atomicOr(&ctl[CTL_ERR], EB_INTERNAL);   // totals left by a launch that did not finish
                    if (pp < M) present[pp] = m;
                    ++pp;
                    gcnt[m] = 0u;
                }
                kept[m] = 0u;
                pos += cnt[j];
            }
            carry += tot;
            pcarry += ptot;
        }
        if (tid == 0) {
            const u32 slot = E.slot & 1u;
            ctl[CTL_BIG] = 0u;
            ctl[CTL_SCR] = 0u;
            ctl[CTL_DEFERRED] = 0u;
            ctl[CTL_PRESENT + slot] = pcarry;
            ctl[CTL_PRESENT + (slot ^ 1u)] = 0u;
        }
    }
}

__global__ __launch_bounds__(G_WG) void k_group_scatter(LaunchArgs a) {
    __shared__ u32 s_pref[MAXB + 1];
    __shared__ u32 s_wsum[G_WG / 64];
    const u32 tid = threadIdx.x, k = num_events(a), M = a.n_modules;
    const u32 total = event_prefix<G_WG>(a, k, s_pref, s_wsum, CNT_ANY, G_SCH, 0);
    for (u32 t = blockIdx.x; t < total; t += gridDim.x) {
        const u32 e = find_slot(s_pref, k, t), c = t - s_pref[e];
        const EventDesc E = get_event(a, e);
        const EvLayout L = ev_layout(E.cap, M);
        const ModRange* mt = ws_ptr<const ModRange>(E, L.mtab);
        const u32* rank = reinterpret_cast<const u32*>(E.o_digi);
        const GroupArrays G = group_arrays(E, L);
        // every load first (module ids, then table entries, ranks and the digis), then
        // the stores: stores to the grouped copy could alias the input for the compiler,
        // which would otherwise keep each digi's loads behind the previous digi's stores
        const u32 i0 = c * G_SCH + tid;
        u32 mm[G_SPER], pos[G_SPER], rr[G_SPER], cc[G_SPER], aa[G_SPER];
#pragma unroll
        for (u32 q = 0; q < G_SPER; ++q) {
            const u32 i = i0 + q * G_WG;
            mm[q] = i < E.n ? u32(E.r_module[i]) : NOPIX;
        }
#pragma unroll
        for (u32 q = 0; q < G_SPER; ++q) {
            const u32 i = i0 + q * G_WG;
            const bool v = mm[q] < M;            // past the end, or out of range (flagged by count)
            const u32 iv = v ? i : 0u;
            const ModRange r = mt[v ? mm[q] : 0u];
            pos[q] = (v && u32(r.first >> 32) == E.epoch) ? u32(r.first) + rank[iv] : NOPIX;
            if (pos[q] != NOPIX && pos[q] >= u32(r.end)) pos[q] = NOPIX;   // only after an internal error
            rr[q] = E.r_row[iv];
            cc[q] = E.r_col[iv];
            aa[q] = E.r_adc[iv];
        }
#pragma unroll
        for (u32 q = 0; q < G_SPER; ++q) {
            const u32 p = pos[q];
            if (p == NOPIX) continue;
            G.m[p] = u16(mm[q]);
            G.r[p] = u16(rr[q]);
            G.c[p] = u16(cc[q]);
            G.a[p] = u16(aa[q]);
            G.perm[p] = i0 + q * G_WG;
        }
    }
}

// ---------------------------------------------------------------------------
// segment: every digi at a module boundary writes the module's entry of the module
// table (first digi, one past the last), tagged with the launch, and the digi that
// starts a module appends it to the present-module list (one atomic per chunk for
// the chunk's place in it); module ids must be non-decreasing (else EB_ORDER) and
// below the module count (else EB_RANGE).  The first chunk of an event also clears
// its kept counts (an absent module keeps nothing) and empties its big-module list.
// ---------------------------------------------------------------------------
template <u32 PER>
__global__ __launch_bounds__(A_WG) void k_segment(LaunchArgs a) {
    constexpr u32 CH = A_WG * PER;
    __shared__ u32 s_pref[MAXB + 1];
    __shared__ u32 s_wsum[A_WG / 64];
    __shared__ u32 s_err, s_base;
    const u32 tid = threadIdx.x;
    const u32 k = num_events(a);
    const u32 total = event_prefix<A_WG>(a, k, s_pref, s_wsum, CNT_SORTED, CH, 0);
    // The small kernel's ticket starts at zero in every launch: the compaction kernel
    // of a finished launch resets it, and this reset also covers a launch whose later
    // kernels were never queued.
    if (blockIdx.x == 0 && tid == 0) st_ag(&a.ctr[S_TICK], 0u);

    for (u32 t = blockIdx.x; t < total; t += gridDim.x) {
        if (tid == 0) s_err = 0;
        const u32 e = find_slot(s_pref, k, t);
        const u32 c = t - s_pref[e];
        const EventDesc E = get_event(a, e);
        const EvLayout L = ev_layout(E.cap, a.n_modules);
        ModRange* mt = ws_ptr<ModRange>(E, L.mtab);
        const u32 n = E.n;
        const u32 i0 = c * CH + tid * PER;
        u32 m[PER];
        if ((reinterpret_cast<uintptr_t>(E.module) & 15u) == 0 && i0 + PER <= n) {
            uint4 v[PER / 8];                             // 16-byte loads, all in flight together
#pragma unroll
            for (u32 q = 0; q < PER / 8; ++q) v[q] = reinterpret_cast<const uint4*>(E.module + i0)[q];
#pragma unroll
            for (u32 q = 0; q < PER / 8; ++q) {
                const u32 w[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
#pragma unroll
                for (u32 j = 0; j < 8; ++j) m[8 * q + j] = (w[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
            }
        } else {
#pragma unroll
            for (u32 j = 0; j < PER; ++j) m[j] = E.module[min(i0 + j, n - 1)];
        }
        const u32 prev = E.module[i0 > 0 ? min(i0 - 1, n - 1) : 0];
        const u32 next = E.module[min(i0 + PER, n - 1)];
        u32* ctl = ws_ptr<u32>(E, L.ctl);
        const u32 slot = E.slot & 1u;
        if (c == 0) {                            // read by the kernels after this one
            if (tid == 0) {
                ctl[CTL_BIG] = 0u;
                ctl[CTL_SCR] = 0u;
                ctl[CTL_DEFERRED] = 0u;
                ctl[CTL_PRESENT + (slot ^ 1u)] = 0u;   // for the next launch (the last one's is done)
            }
            u32* kept = ws_ptr<u32>(E, L.kept);
            for (u32 q = tid; q < a.n_modules; q += A_WG) kept[q] = 0u;
        }
        u32 err = 0, starts = 0;
        const u64 tag = u64(E.epoch) << 32;
#pragma unroll
        for (u32 j = 0; j < PER; ++j) {
            const u32 i = i0 + j;
            if (i < n) {
                const u32 pm = (j == 0) ? prev : m[j - 1];
                const u32 nm = (j + 1 == PER) ? next : m[j + 1];
                if (i > 0 && m[j] < pm) err |= EB_ORDER;
                if (m[j] >= a.n_modules) {
                    err |= EB_RANGE;
                } else {
                    if (i == 0 || m[j] != pm) {
                        mt[m[j]].first = tag | i;
                        starts |= 1u << j;
                    }
                    if (i + 1 == n || m[j] != nm) mt[m[j]].end = tag | (i + 1);
                }
            }
        }
        u32 nstart;
        const u32 ex = group_excl_scan<A_WG>(__popc(starts), tid, s_wsum, nstart);   // also orders s_err
        if (tid == 0) s_base = nstart ? atomicAdd(&ctl[CTL_PRESENT + slot], nstart) : 0u;
        lds_barrier();
        u32* present = ws_ptr<u32>(E, L.present);
        u32 r = s_base + ex;
#pragma unroll
        for (u32 j = 0; j < PER; ++j)
            if (starts & (1u << j)) {
                if (r < a.n_modules) present[r] = m[j];
                else err |= EB_INTERNAL;         // a count left by a launch that did not finish
                ++r;
            }
        if (err) atomicOr(&s_err, err);
        lds_barrier();
        if (tid == 0 && s_err) atomicOr(&ctl[CTL_ERR], s_err);
        lds_barrier();                           // before s_err is cleared for the next chunk
    }
}

// ---------------------------------------------------------------------------
// clustering of one module with its digis in registers (K per thread, group of G)
// ---------------------------------------------------------------------------

constexpr u32 CMW = (COLS + 31) / 32;   // words of a per-module column mask

template <u32 G, u32 K>
struct RegModuleSmem {
    static constexpr u32 RCAP = G * K, KBW = RCAP / 32;
    u32 bm[WORDS];     // fired-pixel bitmap (clear between modules)
    u32 cm[CMW];       // columns holding a fired pixel (clear between modules)
    u64 acc[RCAP];     // union-find parents (u32, first half) and the links found (u32,
                       // second half), then charge | size << 44
    u32 kb[KBW];       // kept-root bits over run index
    u16 rpre[WORDS];   // run starts before each word
    u16 kpre[KBW];     // kept roots before each kb word
    u32 wsum[G / 64];
    u32 nlink;         // links found (entries of the link list)
};


// A module as a group sees it.
struct Item {
    u32 e, it, st, n, mod;
    bool ok;
};

// The value of lane 0 in every lane (for values the whole wave holds alike: the
// compiler then keeps them in scalar registers and branches on them uniformly).
__device__ __forceinline__ u32 wave_uniform(u32 v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename T>
__device__ __forceinline__ T* wave_uniform(T* p) {
    const u64 x = reinterpret_cast<u64>(p);
    return reinterpret_cast<T*>(u64(wave_uniform(u32(x))) | (u64(wave_uniform(u32(x >> 32))) << 32));
}
__device__ __forceinline__ Item wave_uniform(const Item& I) {
    return Item{wave_uniform(I.e), wave_uniform(I.it), wave_uniform(I.st), wave_uniform(I.n), wave_uniform(I.mod),
                wave_uniform(I.ok ? 1u : 0u) != 0};
}
__device__ __forceinline__ EventDesc wave_uniform(const EventDesc& E) {
    EventDesc U{};
    U.module = wave_uniform(E.module);
    U.row = wave_uniform(E.row);
    U.col = wave_uniform(E.col);
    U.adc = wave_uniform(E.adc);
    U.r_module = wave_uniform(E.r_module);
    U.r_row = wave_uniform(E.r_row);
    U.r_col = wave_uniform(E.r_col);
    U.r_adc = wave_uniform(E.r_adc);
    U.ws = wave_uniform(E.ws);
    U.hstat = wave_uniform(E.hstat);
    U.o_digi = wave_uniform(E.o_digi);
    U.o_id = wave_uniform(E.o_id);
    U.o_charge = wave_uniform(E.o_charge);
    U.o_size = wave_uniform(E.o_size);
    U.n = wave_uniform(E.n);
    U.cap = wave_uniform(E.cap);
    U.epoch = wave_uniform(E.epoch);
    U.slot = wave_uniform(E.slot);
    U.flags = wave_uniform(E.flags);
    return U;
}

// Issue the loads of the module's digis j = lt + q*G < n: row and column packed in
// one register (row | col << 16, half-word loads into each half), adc in another; the
// values are only used when the module is clustered, so the loads stay in flight
// meanwhile.  With few slots per thread, slots past the module's end are not
// loaded; with many (the big-module kernel) every slot loads a digi of the module
// (unconditional loads keep that kernel's register allocation within bounds).
template <u32 G, u32 K>
__device__ __forceinline__ void fetch_digis(const EventDesc& E, const Item& I, u32 lt, u32* RC, u32* A) {
#pragma unroll
    for (u32 q = 0; q < K; ++q) {
        const u32 j = lt + q * G;
        if constexpr (K <= 8) {
            RC[q] = A[q] = 0u;
            if (q * G < I.n && j < I.n) {
                RC[q] = u32(E.row[I.st + j]) | (u32(E.col[I.st + j]) << 16);
                A[q] = E.adc[I.st + j];
            }
        } else {
            const u32 i = I.st + (j < I.n ? j : 0u);     // always inside the module
            RC[q] = u32(E.row[i]) | (u32(E.col[i]) << 16);
            A[q] = E.adc[i];
        }
    }
}

// f(q) for the digi slots q < nq (nq uniform over the group).  With few slots per
// thread the loop is not unrolled, so a large body appears once in the code (the
// register arrays it indexes with the uniform q stay in registers).
template <u32 K, typename F>
__device__ __forceinline__ void for_slots(u32 nq, F f) {
    if constexpr (K <= 8) {
#pragma unroll 1
        for (u32 q = 0; q < nq; ++q) f(q);
    } else {
#pragma unroll
        for (u32 q = 0; q < K; ++q)
            if (q < nq) f(q);
    }
}

// Cluster module I (n <= G*K) whose raw digis are in RC/A (fetch_digis).  Every
// thread of the group calls it; with G > 64 all groups of the workgroup call it
// together.  `mid(stage)` runs at the end of phase 1, at the start of phase 3, at
// the end of phase 5 and at the end of phase 8 (the next module's prefetch).
template <u32 G, u32 K, typename Mid>
__device__ __forceinline__ void cluster_regs(const LaunchArgs& a, const EventDesc& E, const EvLayout& L,
                                             const Item& I, RegModuleSmem<G, K>& gp, u32 lt, const u32* RC,
                                             const u32* A, Mid mid) {
    static_assert(G * K <= 65536, "run indices are kept in 16 bits");
    constexpr u32 KBW = G * K / 32, CPT = (COLS + G - 1) / G;
    // dense modules (the big-module kernel): unions per (column, word) of the bitmap
    // and roots per run; sparse ones: unions and roots per digi
    constexpr bool WORD_LINKS = K > 8;
    const bool hits = (E.flags & EF_HITS) != 0;
    u64* hs = ws_ptr<u64>(E, L.hsum);
    u32* par = reinterpret_cast<u32*>(gp.acc);
    const bool act = I.ok;
    const u32 nq = act ? min((I.n + G - 1) / G, K) : 0u;   // slots that may hold a digi
    u32 err = 0;
    // LIN: linear pixel index or NOPIX; AR: adc in the low 16 bits, then run / root
    u32 LIN[K], AR[K];
    // P1: insert the module's digis into the bitmap
#pragma unroll
    for (u32 q = 0; q < K; ++q) {
        const u32 j = lt + q * G;
        LIN[q] = NOPIX;
        AR[q] = A[q] & 0xFFFFu;
        if (q < nq && j < I.n) {
            const u32 rq = RC[q] & 0xFFFFu, cq = RC[q] >> 16;
            if (rq < ROWS && cq < COLS) {
                const u32 lin = cq * ROWS + rq;
                const u32 bit = 1u << (lin & 31u);
                if (atomicOr(&gp.bm[lin >> 5], bit) & bit) err |= EB_DUP;
                atomicOr(&gp.cm[cq >> 5], 1u << (cq & 31u));
                LIN[q] = lin;
            } else {
                err |= EB_RANGE;
            }
        }
    }
    mid(0);
    gsync<G>();
    // P2: run starts per word of the columns holding a fired pixel (the only words
    // whose run index is ever asked for), prefix over them in column order; parents.
    // A thread takes CPT consecutive columns; per column the five word counts are kept
    // packed, 6 bits each.
    u32 nruns = 0;
    {
        u32 pk[CPT];
        u32 cnt = 0;
        const u32 c0 = lt * CPT;
#pragma unroll
        for (u32 i = 0; i < CPT; ++i) {
            const u32 c = c0 + i;
            pk[i] = 0u;
            if (act && c < COLS && ((gp.cm[c >> 5] >> (c & 31u)) & 1u)) {
#pragma unroll
                for (u32 k = 0; k < WPC; ++k) {
                    const u32 v = __popc(run_starts(gp.bm, c * WPC + k));
                    pk[i] |= v << (6 * k);
                    cnt += v;
                }
                pk[i] |= 1u << 31;                       // column fired
            }
        }
        const u32 ex = group_excl_scan<G>(cnt, lt, gp.wsum, nruns);
        u32 run = ex;
#pragma unroll
        for (u32 i = 0; i < CPT; ++i) {
            if (pk[i] >> 31) {
                const u32 c = c0 + i;
#pragma unroll
                for (u32 k = 0; k < WPC; ++k) {
                    gp.rpre[c * WPC + k] = u16(run);
                    run += (pk[i] >> (6 * k)) & 63u;
                }
            }
        }
    }
    if (act)
        for (u32 r = lt; r < nruns; r += G) par[r] = r;
    if (lt == 0) gp.nlink = 0u;
    gsync<G>();
    mid(1);
    u32 starts = 0;
    constexpr u32 LCAPL = G * K;                     // link list capacity
    u32* links = reinterpret_cast<u32*>(gp.acc) + G * K;
    // unite the listed links, evenly over the group
    auto unite_links = [&]() {
        gsync<G>();
        if (act) {
            const u32 nl = min(ld_wg(&gp.nlink), LCAPL);
            for (u32 t = lt; t < nl; t += G) {
                const u32 l = links[t];
                uf_unite(par, l >> 16, l & 0xFFFFu);
            }
        }
    };
    if constexpr (WORD_LINKS) {
        // P3: links between adjacent fired columns, one (column, word) unit at a time
        if (act)
            for (u32 u = lt; u < (COLS - 1) * WPC; u += G) {
                const u32 c = u / WPC, k = u - c * WPC;
                if (((gp.cm[c >> 5] >> (c & 31u)) & 1u) && ((gp.cm[(c + 1) >> 5] >> ((c + 1) & 31u)) & 1u))
                    link_word(par, links, LCAPL, &gp.nlink, gp.bm, gp.rpre, c, k);
            }
        unite_links();
        gsync<G>();
        // P4: every run points at its root (walks only read; each store writes a root,
        // so a walk through a stored entry still ends at the same root)
        if (act)
            for (u32 r = lt; r < nruns; r += G) {
                u32 x = ld_wg(&par[r]);
                for (u32 it = 0; it < MAX_RUNS; ++it) {
                    const u32 y = ld_wg(&par[x]);
                    if (y == x) break;
                    x = y;
                }
                st_wg(&par[r], x);
            }
        gsync<G>();
        // each digi's run and root; the digi that starts its root's run speaks for the cluster
        u32 RN[K];
#pragma unroll
        for (u32 q = 0; q < K; ++q) RN[q] = (q < nq && LIN[q] != NOPIX) ? run_of(gp.bm, gp.rpre, LIN[q]) : 0u;
#pragma unroll
        for (u32 q = 0; q < K; ++q)
            if (q < nq && LIN[q] != NOPIX) {
                const u32 lin = LIN[q], root = ld_wg(&par[RN[q]]);
                if (root == RN[q] && !((lin % ROWS) > 0 && fired(gp.bm, lin - 1))) starts |= 1u << q;
                AR[q] = (AR[q] & 0xFFFFu) | (root << 16);
            }
        gsync<G>();
    } else {
        // P3: the two rules of link_word, from the digi that starts each run: rule B
        // links the run to the run of the column on its left holding the first fired
        // pixel of rows -1..+1, rule A to the run of the column on its right at row -1
        // when row -2 is fired in either column.
        u32 RS = 0;                                  // slots whose digi starts its run
        const u32 lane = lt & 63u;
        const u64 below = (1ull << lane) - 1ull;
        for_slots<K>(nq, [&](u32 q) {                // every lane of the group runs every slot
            const u32 lin = LIN[q];
            u32 r = 0, ob = NOPIX, oa = NOPIX;       // the run, its links' other runs
            if (lin != NOPIX) {
                const u32 col = lin / ROWS, row = lin - col * ROWS;
                // every bitmap word the rules look at, read at once: rows -2..+1 of
                // this column and of the columns on either side (clamped into the
                // module; out-of-module rows and columns are masked off below)
                const u32 lo = row >= 2 ? lin - 2 : lin - row, hi = row + 1 < ROWS ? lin + 1 : lin;
                const u32 lcol = col > 0 ? ROWS : 0u, rcol = col + 1 < COLS ? ROWS : 0u;
                const u32 w0 = lo >> 5, w1 = hi >> 5;                      // this column
                const u32 l0 = (lo - lcol) >> 5, l1 = (hi - lcol) >> 5;    // left
                const u32 r0 = (lo + rcol) >> 5, r1 = (hi + rcol) >> 5;    // right
                const u32 bw0 = gp.bm[w0], bw1 = gp.bm[w1], bl0 = gp.bm[l0], bl1 = gp.bm[l1];
                const u32 br0 = gp.bm[r0], br1 = gp.bm[r1];
                const u32 bp = gp.bm[w0 ? w0 - 1 : 0u], rp = gp.rpre[lin >> 5];
                // fired(pixel at this column's row `rr`, column offset d in {-1, 0, +1})
                auto at = [&](u32 rr, int d) -> u32 {
                    if (rr >= ROWS) return 0u;
                    if ((d < 0 && !col) || (d > 0 && col + 1 >= COLS)) return 0u;
                    const u32 x = lin - row + rr + (d < 0 ? 0u - ROWS : d > 0 ? ROWS : 0u);
                    const u32 base = d < 0 ? l0 : d > 0 ? r0 : w0;
                    const u32 word = (x >> 5) == base ? (d < 0 ? bl0 : d > 0 ? br0 : bw0) : (d < 0 ? bl1 : d > 0 ? br1 : bw1);
                    return (word >> (x & 31u)) & 1u;
                };
                {   // own run: run starts in this word up to this row
                    const u32 w = lin >> 5, b = lin & 31u;
                    const u32 bwd = (w == w0) ? bw0 : bw1;
                    const u32 carry = (w % WPC) ? (((w == w0) ? bp : bw0) >> 31) : 0u;
                    const u32 st = bwd & ~((bwd << 1) | carry);
                    r = u32(rp) + __popc(st & ((2u << b) - 1u)) - 1u;
                }
                AR[q] |= r << 16;
                if (!at(row - 1u, 0)) {                      // the digi starts its run
                    RS |= 1u << q;
                    const u32 f = at(row - 1u, -1) ? row - 1u : at(row, -1) ? row : at(row + 1u, -1) ? row + 1u : NOPIX;
                    const bool la = at(row - 1u, 1) && (at(row - 2u, 0) || at(row - 2u, 1));
                    // run lookups (independent of each other)
                    if (f != NOPIX) ob = run_of(gp.bm, gp.rpre, lin - row + f - ROWS);
                    if (la) oa = run_of(gp.bm, gp.rpre, lin + ROWS - 1u);
                }
            }
            // places in the list: one LDS atomic per wave
            const u64 mb = __ballot(ob != NOPIX), ma = __ballot(oa != NOPIX);
            const u32 nb = u32(__popcll(mb)), na = u32(__popcll(ma));
            if (nb + na) {
                u32 base = 0;
                if (lane == 0) base = atomicAdd(&gp.nlink, nb + na);
                base = __shfl(base, 0, 64);
                if (ob != NOPIX) put_link(links, LCAPL, par, base + u32(__popcll(mb & below)), r, ob);
                if (oa != NOPIX) put_link(links, LCAPL, par, base + nb + u32(__popcll(ma & below)), r, oa);
            }
        });
        unite_links();
        gsync<G>();
        // P4: every run points at its root (read-only walks, each store a root), then
        // each digi's root in one load; the digi that starts its root's run speaks for
        // the cluster
        if (act)
            for (u32 r = lt; r < nruns; r += G) {
                u32 x = ld_wg(&par[r]);
                for (u32 it = 0; it < MAX_RUNS; ++it) {
                    const u32 y = ld_wg(&par[x]);
                    if (y == x) break;
                    x = y;
                }
                st_wg(&par[r], x);
            }
        gsync<G>();
#pragma unroll
        for (u32 q = 0; q < K; ++q)
            if (q < nq && LIN[q] != NOPIX) {
                const u32 run = AR[q] >> 16, root = ld_wg(&par[run]);
                if (root == run && ((RS >> q) & 1u)) starts |= 1u << q;
                AR[q] = (AR[q] & 0xFFFFu) | (root << 16);
            }
        gsync<G>();
    }
    if (act) {
        for (u32 r = lt; r < nruns; r += G) gp.acc[r] = 0ull;
        for (u32 w = lt; w < KBW; w += G) gp.kb[w] = 0u;
    }
    gsync<G>();
    // P5: charge and size per root
#pragma unroll
    for (u32 q = 0; q < K; ++q)
        if (q < nq && LIN[q] != NOPIX) atomicAdd(&gp.acc[AR[q] >> 16], (1ull << 44) | u64(AR[q] & 0xFFFFu));
    mid(2);
    gsync<G>();
    // P6: charge cut, one bit per kept root
#pragma unroll
    for (u32 q = 0; q < K; ++q)
        if (q < nq && (starts & (1u << q))) {
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
            if (q < nq && (starts & (1u << q))) {
                const u32 r = AR[q] >> 16;
                const u64 v = gp.acc[r];
                const u32 charge = u32(v), size = u32(v >> 44);
                u32 id = NOPIX, pos = 0;
                if (charge >= a.charge_cut) {
                    pos = gp.kpre[r >> 5] + __popc(gp.kb[r >> 5] & ((1u << (r & 31u)) - 1u));
                    id = idbase + LIN[q];
                    tid_[I.st + pos] = int32_t(id);
                    tch[I.st + pos] = int32_t(charge);
                    tsz[I.st + pos] = int32_t(size);
                }
                gp.acc[r] = u64(id) | (u64(pos) << 32);        // id (or -1) and record for P9
            }
        if (lt == 0) ws_ptr<u32>(E, L.kept)[I.it] = Kc;
    }
    mid(3);
    gsync<G>();
    // P9: per-digi cluster id (and, with fused hits, its weighted coordinates added
    // to its cluster's sums); clear the bitmap words used
    if (act) {
        int32_t* od = E.o_digi;
        const u32* perm = perm_of(E, L);
        if (hits) {
#pragma unroll
            for (u32 q = 0; q < K; ++q)
                if (q < nq && LIN[q] != NOPIX) {
                    const u64 v = gp.acc[AR[q] >> 16];
                    if (u32(v) != NOPIX) {
                        const u32 p = I.st + u32(v >> 32), lin = LIN[q], col = lin / ROWS;
                        const u64 w = AR[q] & 0xFFFFu;
                        atomicAdd(&hs[2 * p], w * col);
                        atomicAdd(&hs[2 * p + 1], w * (lin - col * ROWS));
                    }
                }
        }
#pragma unroll
        for (u32 q = 0; q < K; ++q) {
            const u32 j = lt + q * G;
            if (q < nq && j < I.n)
                od[out_pos(perm, I.st + j)] = (LIN[q] != NOPIX) ? int32_t(u32(gp.acc[AR[q] >> 16])) : -1;
        }
#pragma unroll
        for (u32 q = 0; q < K; ++q)
            if (q < nq && LIN[q] != NOPIX) st_wg(&gp.bm[LIN[q] >> 5], 0u);   // several digis may share a word
        if (lt < CMW) gp.cm[lt] = 0u;
        if (err) atomicOr(ws_ptr<u32>(E, L.ctl) + CTL_ERR, err);
    }
    gsync<G>();
}

// ---------------------------------------------------------------------------
// XCD-aware order of workgroups: consecutive workgroup ids go to the eight XCDs in
// turn, so the order (id % 8, id / 8) gives each XCD a contiguous share of the work
// and the data its modules read and write stays in that XCD's L2.  A bijection on
// [0, n) for any n.
// ---------------------------------------------------------------------------
constexpr u32 N_XCD = 8;
__device__ __forceinline__ u32 xcd_order(u32 b, u32 n) {
    const u32 q = n / N_XCD, r = n % N_XCD, x = b % N_XCD, i = b / N_XCD;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// ---------------------------------------------------------------------------
// Module ranges by search (launches without the segmentation kernel): with the
// module ids sorted, module m's digis are [lower bound of m, lower bound of m + 1).
// One wave finds both.  The first round probes 64 points SEARCH_STEP apart around
// where module m would start if the modules were evenly filled; when that brackets
// a bound, it is within SEARCH_STEP digis and the last round (up to 128 candidates,
// two per lane) finds it: two dependent loads.  Otherwise each further round probes
// 64 evenly spaced points of the remaining range and keeps the stretch the ballot
// points to (about 65 times shorter).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void narrow_range(u32& lo, u32& hi, u64 ge) {
    const u32 s = hi - lo;                      // > 64; probe l at lo + (l + 1) * s / 65
    if (ge) {
        const u32 f = __builtin_ctzll(ge);      // first probe at or above the key
        hi = lo + u32((u64(f) + 1) * s / 65);
        lo = f ? lo + u32(u64(f) * s / 65) + 1 : lo;
    } else {
        lo = lo + u32(u64(64) * s / 65) + 1;
    }
}

constexpr u32 SEARCH_STEP = 128, SEARCH_LAST = 128;

// Narrow [lo, hi] by a ballot over probes at q(l) = clamp(guess + (l - 32) * step),
// non-decreasing in l; the answer is the first index whose id is >= the key.
__device__ __forceinline__ void narrow_window(u32& lo, u32& hi, u64 ge, long long guess, u32 n) {
    auto q = [&](u32 l) -> u32 {
        const long long p = guess + (static_cast<long long>(l) - 32) * SEARCH_STEP;
        return u32(p < 0 ? 0 : (p >= (long long)n ? (long long)n - 1 : p));
    };
    if (ge) {
        const u32 f = __builtin_ctzll(ge);
        hi = q(f);
        if (f) lo = q(f - 1) + 1;
    } else {
        lo = q(63) + 1;
    }
}

__device__ __forceinline__ void module_range(const EventDesc& E, u32 n_modules, u32 key, u32 lane, u32& first,
                                             u32& end) {
    const u16* mod = E.module;
    const u32 n = E.n;
    u32 lo0 = 0, hi0 = n, lo1 = 0, hi1 = n;       // each answer lies in [lo, hi]
    {
        const long long guess = static_cast<long long>((u64(key) * n) / n_modules);
        const long long p = guess + (static_cast<long long>(lane) - 32) * SEARCH_STEP;
        const u32 v = mod[p < 0 ? 0 : (p >= (long long)n ? n - 1 : u32(p))];
        const u64 b0 = __ballot(v >= key), b1 = __ballot(v >= key + 1);
        narrow_window(lo0, hi0, b0, guess, n);
        narrow_window(lo1, hi1, b1, guess, n);
    }
    while (hi0 - lo0 > SEARCH_LAST || hi1 - lo1 > SEARCH_LAST) {
        const bool w0 = hi0 - lo0 > SEARCH_LAST, w1 = hi1 - lo1 > SEARCH_LAST;
        const u32 q0 = lo0 + u32((u64(lane) + 1) * (hi0 - lo0) / 65);   // < hi0 <= n
        const u32 q1 = lo1 + u32((u64(lane) + 1) * (hi1 - lo1) / 65);
        const bool g0 = w0 && mod[q0] >= key;
        const bool g1 = w1 && mod[q1] >= key + 1;
        const u64 b0 = __ballot(g0), b1 = __ballot(g1);
        if (w0) narrow_range(lo0, hi0, b0);
        if (w1) narrow_range(lo1, hi1, b1);
    }
    // at most SEARCH_LAST = 128 candidates per bound: positions lo + lane, lo + 64 + lane
    const bool g0 = lo0 + lane < hi0 && mod[lo0 + lane] >= key;
    const bool h0 = lo0 + 64 + lane < hi0 && mod[lo0 + 64 + lane] >= key;
    const bool g1 = lo1 + lane < hi1 && mod[lo1 + lane] >= key + 1;
    const bool h1 = lo1 + 64 + lane < hi1 && mod[lo1 + 64 + lane] >= key + 1;
    const u64 b0 = __ballot(g0), c0 = __ballot(h0), b1 = __ballot(g1), c1 = __ballot(h1);
    first = b0 ? lo0 + u32(__builtin_ctzll(b0)) : c0 ? lo0 + 64 + u32(__builtin_ctzll(c0)) : hi0;
    end = b1 ? lo1 + u32(__builtin_ctzll(b1)) : c1 ? lo1 + 64 + u32(__builtin_ctzll(c1)) : hi1;
}

// Order and range checks of every digi's module id (launches without the
// segmentation kernel), one coalesced pass over the whole grid.  The first stride's
// ids are loaded by id_check_load (before the first range search, so that the two
// latencies overlap) and checked, with the rest, by id_check_finish.
struct IdCheck {
    u32 m0, m1;
};
template <u32 WG>
__device__ __forceinline__ IdCheck id_check_load(const EventDesc& E) {
    const u32 i = blockIdx.x * WG + threadIdx.x;
    IdCheck c{0u, 0xFFFFFFFFu};
    if (i < E.n) {
        c.m0 = E.module[i];
        if (i + 1 < E.n) c.m1 = E.module[i + 1];
    }
    return c;
}
template <u32 WG>
__device__ __forceinline__ void id_check_finish(const LaunchArgs& a, const EventDesc& E, IdCheck c) {
    u32 err = 0;
    for (u32 i = blockIdx.x * WG + threadIdx.x; i < E.n; i += gridDim.x * WG) {
        if (i >= gridDim.x * WG) {               // strides after the first
            c.m0 = E.module[i];
            c.m1 = i + 1 < E.n ? E.module[i + 1] : 0xFFFFFFFFu;
        }
        if (c.m0 >= a.n_modules) err |= EB_RANGE;
        if (c.m1 < c.m0) err |= EB_ORDER;
    }
    if (err) atomicOr(ws_ptr<u32>(E, ev_layout(E.cap, a.n_modules).ctl) + CTL_ERR, err);
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

// Waves per SIMD the shape's LDS allows, at most four (at most 128 registers):
// modules in flight bound throughput, so registers should not bound them first.
template <u32 WG, u32 MPW, u32 K>
constexpr u32 small_waves_per_simd() {
    constexpr u32 lds_groups = 163840u / u32(sizeof(SmallSmem<WG, MPW, K>));
    constexpr u32 w = lds_groups * (WG / 64) / 4;
    return w < 1 ? 1 : (w > 4 ? 4 : w);
}
#ifndef PXCL_WAVES_PER_EU
#define PXCL_WAVES_PER_EU(...) __attribute__((amdgpu_waves_per_eu(__VA_ARGS__)))
#endif
template <u32 WG, u32 MPW, u32 K>
__global__ __launch_bounds__(WG) PXCL_WAVES_PER_EU(small_waves_per_simd<WG, MPW, K>()) void k_small(LaunchArgs a) {
    using S = SmallSmem<WG, MPW, K>;
    constexpr u32 G = S::G;
    constexpr bool WAVE = (G == 64);          // groups of one wave run independently
    constexpr u32 STEP = WAVE ? 1u : MPW;     // modules per ticket
    __shared__ S s;
    const u32 tid = threadIdx.x, g = tid / G, lt = tid % G;
    const u32 gofs = WAVE ? 0u : g;
    RegModuleSmem<G, K>& gp = s.grp[g];
    for (u32 w = lt; w < WORDS; w += G) gp.bm[w] = 0u;
    if (lt < CMW) gp.cm[lt] = 0u;
    const u32 k = num_events(a);
    // Without the segmentation kernel (one event): every module is a unit, its
    // digis found by search; this kernel then checks the module ids, writes the
    // module table entries of the modules present and sets the unit count the
    // kernels after it read.
    const bool fused = (a.flags & LF_FUSED) != 0 && k == 1;
    u32 total;
    IdCheck idc{0u, 0xFFFFFFFFu};
    if (k == 1) {                             // one event, alone or in a header
        const EventDesc E0 = get_event(a, 0);
        if (fused) {
            total = E0.n ? a.n_modules : 0u;
            idc = id_check_load<WG>(E0);
            if (blockIdx.x == 0 && tid == 0 && E0.n) {
                u32* ctl = ws_ptr<u32>(E0, ev_layout(E0.cap, a.n_modules).ctl);
                ctl[CTL_PRESENT + (E0.slot & 1u)] = a.n_modules;
                ctl[CTL_PRESENT + ((E0.slot & 1u) ^ 1u)] = 0u;
            }
        } else {
            total = unit_count(a, E0);
        }
        if (tid == 0) {
            s.pref[0] = 0;
            s.pref[1] = total;
        }
        lds_barrier();
    } else {
        total = event_prefix<WG>(a, k, s.pref, s.wsum, CNT_UNITS, 1, 0);
    }
    // Work unit t: unit t - pref[e] of event e, and its module's table entry.
    auto entry_of = [&](u32 t, EventDesc& Ev, u32& e, u32& mod) -> ModRange {
        e = k == 1 ? 0u : find_slot(s.pref, k, t);
        Ev = get_event(a, e);
        const EvLayout L = ev_layout(Ev.cap, a.n_modules);
        if (fused) {
            mod = t;
            u32 f, en;
            module_range(Ev, a.n_modules, mod, lt & 63u, f, en);
            const u64 tag = u64(Ev.epoch) << 32;
            const ModRange r{tag | f, tag | en};
            if (lt == 0 && en > f) ws_ptr<ModRange>(Ev, L.mtab)[mod] = r;   // for the big kernel, compaction, hits
            return r;
        }
        mod = unit_module(a, Ev, L, s.pref[e + 1] - s.pref[e], t - s.pref[e]);
        return ws_ptr<const ModRange>(Ev, L.mtab)[mod];
    };
    // I.n = 0 for an entry that is not this launch's (or inconsistent after an
    // ordering error); ok only for a present module the group can hold.
    auto make_item = [&](const ModRange& r, const EventDesc& Ev, u32 e, u32 mod, bool valid) {
        Item I{e, mod, 0, 0, mod, false};
        if (valid && u32(r.first >> 32) == Ev.epoch && u32(r.end >> 32) == Ev.epoch) {
            const u32 st = u32(r.first), en = u32(r.end);
            if (st < en && en <= Ev.n) {
                I.st = st;
                I.n = en - st;
            }
        }
        I.ok = I.n > 0 && I.n <= G * K;
        return I;
    };
    // A module larger than the group goes to the big-module list, or above BIG_RCAP
    // digis to the scratch-mode list (or, when that kernel is not launched, keeps
    // nothing and flags the size hint; with LF_DEFER it is listed all the same, for
    // the second launch).  Other units not clustered (absent modules,
    // entries not of this launch) keep nothing: the segmentation kernel cleared the
    // kept counts, without it this kernel does.
    auto skip = [&](const EventDesc& Ev, const Item& Is) {
        const EvLayout L = ev_layout(Ev.cap, a.n_modules);
        u32* ctl = ws_ptr<u32>(Ev, L.ctl);
        const bool scr = Is.n > BIG_RCAP;
        const bool listed = (a.flags & LF_DEFER) || !(a.flags & (scr ? (LF_NO_BIG | LF_NO_SCRATCH) : LF_NO_BIG));
        if (Is.n > G * K && listed) {
            const u32 r = atomicAdd(&ctl[scr ? CTL_SCR : CTL_BIG], 1u);
            if (r < a.n_modules) ws_ptr<u32>(Ev, scr ? L.scr : L.big)[r] = Is.mod;
            else atomicOr(&ctl[CTL_ERR], EB_INTERNAL);
            return;
        }
        if (Is.n > G * K) atomicOr(&ctl[CTL_ERR], EB_HINT);
        if (fused || Is.n > G * K) ws_ptr<u32>(Ev, L.kept)[Is.mod] = 0u;
    };

    // Modules are assigned statically in rounds (round r: module r*per_round + the
    // group's index) for about three quarters of the work, the rest comes from a
    // ticket counter, which every group contends for.  The ticket of the module after
    // next is drawn while the current one is clustered, and the next module's
    // table entry (or range, by search) and digis are loaded meanwhile.
    const u32 per_round = gridDim.x * MPW;
    u32 base = xcd_order(blockIdx.x, gridDim.x) * MPW + (WAVE ? g : 0u);
    EventDesc E{};
    Item I{0, 0, 0, 0, 0, false};
    u32 RC[K], A[K];
    {
        const u32 t = base + gofs;
        if (t < total) {
            u32 e, mod;
            const ModRange r = entry_of(t, E, e, mod);
            I = make_item(r, E, e, mod, true);
        }
        I = wave_uniform(I);                      // one module per wave (or per group of waves)
        E = wave_uniform(E);
        if (I.ok) fetch_digis<G, K>(E, I, lt, RC, A);
    }
    if (fused) id_check_finish<WG>(a, get_event(a, 0), idc);
    const u32 nrounds = per_round < total ? max(1u, u32((3ull * total) / (4ull * per_round))) : 1u;   // static
    const u32 nstatic = nrounds * per_round;
    const bool dyn = nstatic < total;             // tickets needed at all
    u32 round = 0;                                // round of the current module (>= nrounds: dynamic)
    u32 nv = total;                               // ticket of the next dynamic module (in flight)
    if (dyn && nrounds == 1 && ((WAVE && lt == 0) || (!WAVE && tid == 0))) nv = atomicAdd(&a.ctr[S_TICK], STEP) + nstatic;

    while (base < total) {
        u32 nbase = total, nv2 = 0, ne = 0, nmod = 0;
        EventDesc En{};
        bool have = false;
        ModRange ent{0, 0};
        Item In{0, 0, 0, 0, 0, false};
        u32 NRC[K], NA[K];
        auto issue_entry = [&]() {
            const u32 t = nbase + gofs;
            if (t < total) {
                ent = entry_of(t, En, ne, nmod);  // a table load: issued here, used at stage 2
                have = true;
            }
        };
        auto mid = [&](int stage) {
            if (stage == 0) {
                const bool snext = round + 1 < nrounds;            // next module static
                const bool draw = dyn && round + 2 >= nrounds;     // module after next dynamic
                if constexpr (WAVE) {
                    nbase = snext ? base + per_round : __builtin_amdgcn_readfirstlane(nv);
                    nv2 = total;
                    if (draw && lt == 0 && nbase < total) nv2 = atomicAdd(&a.ctr[S_TICK], 1u) + nstatic;
                    issue_entry();
                } else if (tid == 0) {
                    const u32 nx = snext ? base + per_round : nv;
                    s.tick[1] = nx;
                    nv2 = (draw && nx < total) ? atomicAdd(&a.ctr[S_TICK], STEP) + nstatic : total;
                }
            } else if (stage == 1) {
                if constexpr (!WAVE) {
                    nbase = s.tick[1];
                    issue_entry();
                }
            } else if (stage == 2) {
                In = wave_uniform(make_item(ent, En, ne, nmod, have));
                En = wave_uniform(En);
                if (In.ok) fetch_digis<G, K>(En, In, lt, NRC, NA);
            }
        };
        if (base + gofs < total && !I.ok && lt == 0) skip(E, I);
        if (!WAVE || I.ok) {
            const EvLayout L = ev_layout(E.cap, a.n_modules);
            cluster_regs<G, K>(a, E, L, I, gp, lt, RC, A, mid);
        } else {
            mid(0);
            mid(1);
            mid(2);
            mid(3);
        }
        base = nbase;
        E = En;
        I = In;
        nv = nv2;
        ++round;
#pragma unroll
        for (u32 q = 0; q < K; ++q) { RC[q] = NRC[q]; A[q] = NA[q]; }
    }
}

// ---------------------------------------------------------------------------
// big: one module per 512-thread workgroup
// ---------------------------------------------------------------------------
// Scratch mode (more than BIG_RCAP digis).  Connectivity is computed on the bitmap
// alone: every vertical run is linked to the runs of the next column that touch it,
// with the parents of up to MAX_RUNS runs in LDS.  The roots, in run order (= order
// of their smallest linear index), number the clusters.  Three passes over the digis
// follow: charge and size (device atomics into the module's slice of the event's
// final charge/size arrays, which the compaction kernel overwrites later; a wave
// whose digis all belong to one cluster adds once), then per-digi ids.
template <u32 BW>
struct BigScratchSmem {
    u32 bm[WORDS];
    u32 par[MAX_RUNS];
    u32 rootb[MAX_RUNS / 32];   // root runs, then kept clusters (over cluster index)
    u16 rpre[WORDS];
    u16 rootp[MAX_RUNS / 32];   // roots before each word, then kept clusters before each word
    u32 wsum[BW / 64];
    u32 misc[4];
};

constexpr u32 UNR = 8;                        // digis per thread fetched at once

__device__ __forceinline__ u32 clampj(u32 j, u32 n) { return j < n ? j : 0u; }

// Add `val` at base[key] for every lane with `valid`; one atomic per wave when all
// valid lanes share the key.  Called by all lanes of the wave.
__device__ __forceinline__ void wave_add(u32* base, u32 key, u32 val, bool valid) {
    const u64 vm = __ballot(valid);
    if (!vm) return;
    const u32 first = __ffsll((unsigned long long)vm) - 1;
    const u32 lead = __shfl(key, first, 64);
    const u64 same = __ballot(valid && key == lead);
    if (same == vm) {
        u32 sum = valid ? val : 0u;
#pragma unroll
        for (u32 d = 32; d >= 1; d >>= 1) sum += __shfl_xor(sum, d, 64);
        if ((threadIdx.x & 63u) == first) atomicAdd(&base[lead], sum);
    } else if (valid) {
        atomicAdd(&base[key], val);
    }
}

// The same for 64-bit sums in LDS.
__device__ __forceinline__ void wave_add_lds64(u64* base, u32 key, u64 val, bool valid) {
    const u64 vm = __ballot(valid);
    if (!vm) return;
    const u32 first = __ffsll((unsigned long long)vm) - 1;
    const u32 lead = __shfl(key, first, 64);
    const u64 same = __ballot(valid && key == lead);
    if (same == vm) {
        u64 sum = valid ? val : 0ull;
#pragma unroll
        for (u32 d = 32; d >= 1; d >>= 1) sum += __shfl_xor(sum, d, 64);
        if ((threadIdx.x & 63u) == first) atomicAdd(&base[lead], sum);
    } else if (valid) {
        atomicAdd(&base[key], val);
    }
}

template <u32 BW>
__device__ __forceinline__ void cluster_scratch(const LaunchArgs& a, const EventDesc& E, const EvLayout& L,
                                                const Item& I, BigScratchSmem<BW>& s) {
    constexpr u32 WPT = (WORDS + BW - 1) / BW;
    constexpr u32 KW = MAX_RUNS / 32, KPT = (KW + BW - 1) / BW;
    constexpr u32 SPAN = UNR * BW;
    const u32 tid = threadIdx.x, n = I.n, st = I.st;
    u32* cid = reinterpret_cast<u32*>(E.o_id) + st;       // per cluster: id (or -1 once cut)
    u32* cch = reinterpret_cast<u32*>(E.o_charge) + st;   // per cluster: charge
    u32* csz = reinterpret_cast<u32*>(E.o_size) + st;     // per cluster: size
    int32_t* od = E.o_digi;
    const u32* perm = perm_of(E, L);
    const bool hits = (E.flags & EF_HITS) != 0;
    u64* hs = ws_ptr<u64>(E, L.hsum);
    u32 err = 0;
    // UNR digis' linear index (NOPIX when absent or out of range), loads first
    auto fetch = [&](u32 base, u32* lin, u32* adc) {
        u32 r[UNR], c[UNR];
#pragma unroll
        for (u32 u = 0; u < UNR; ++u) {
            const u32 i = st + clampj(base + u * BW + tid, n);
            r[u] = E.row[i];
            c[u] = E.col[i];
            if (adc) adc[u] = E.adc[i];
        }
#pragma unroll
        for (u32 u = 0; u < UNR; ++u) {
            const u32 j = base + u * BW + tid;
            lin[u] = (j < n && r[u] < ROWS && c[u] < COLS) ? c[u] * ROWS + r[u] : NOPIX;
            if (j < n && lin[u] == NOPIX) err |= EB_RANGE;
        }
    };
    const u32 wv = tid >> 6, lane = tid & 63u;
    // cluster index of run `run` (after the flattening below, par[run] is its root)
    auto cluster_of = [&](u32 run) {
        const u32 root = ld_wg(&s.par[run]);
        return u32(s.rootp[root >> 5]) + __popc(s.rootb[root >> 5] & ((1u << (root & 31u)) - 1u));
    };
    // s.rootb[] over all KW words: bit r set iff pred(r); a wave forms 64 bits at a time
    // from 64 consecutive indices (ballot), so lanes touch consecutive words
    auto set_bits = [&](auto pred) {
        for (u32 base = wv * 64; base < KW * 32; base += BW) {
            const u64 m = __ballot(pred(base + lane) ? 1 : 0);
            if (lane == 0) {
                s.rootb[base >> 5] = u32(m);
                s.rootb[(base >> 5) + 1] = u32(m >> 32);
            }
        }
    };
    for (u32 base = 0; base < n; base += SPAN) {               // pass 1: bitmap
        u32 lin[UNR];
        fetch(base, lin, nullptr);
#pragma unroll
        for (u32 u = 0; u < UNR; ++u)
            if (lin[u] != NOPIX) {
                const u32 bit = 1u << (lin[u] & 31u);
                if (atomicOr(&s.bm[lin[u] >> 5], bit) & bit) err |= EB_DUP;
            }
    }
    lds_barrier();
    u32 nruns;
    {                                                           // runs
        u32 sw[WPT], cnt = 0;
#pragma unroll
        for (u32 i = 0; i < WPT; ++i) {
            const u32 w = tid * WPT + i;
            sw[i] = w < WORDS ? __popc(run_starts(s.bm, w)) : 0u;
            cnt += sw[i];
        }
        u32 run = group_excl_scan<BW>(cnt, tid, s.wsum, nruns);
#pragma unroll
        for (u32 i = 0; i < WPT; ++i) {
            const u32 w = tid * WPT + i;
            if (w < WORDS) s.rpre[w] = u16(run);
            run += sw[i];
        }
    }
    for (u32 r = tid; r < nruns; r += BW) s.par[r] = r;
    lds_barrier();
    // Unions from the bitmap only.  Wave v links the runs of its block of columns to the
    // next column, one column at a time from left to right, a lane per row.
    // A run of the next column is then hooked straight under a root found in an earlier
    // column, so the trees stay shallow even along chains that cross the module (a
    // serpentine); unordered unions would build paths as long as the chain.
    {
        constexpr u32 NWV = BW / 64;
        const u32 c0 = wv * COLS / NWV, c1 = (wv + 1) * COLS / NWV;
        ColPair cur;
        if (c0 < c1 && c0 + 1 < COLS) load_pair(cur, s.bm, s.rpre, c0);
        for (u32 col = c0; col < c1 && col + 1 < COLS; ++col) {
            ColPair nxt;
            const bool more = col + 1 < c1 && col + 2 < COLS;
            if (more) load_pair(nxt, s.bm, s.rpre, col + 1);   // the bitmap is read-only here
            link_pair(s.par, cur, lane);
            gsync<64>();                                        // this column's hooks before the next
            if (more) cur = nxt;
        }
    }
    lds_barrier();
    // flatten: every run points at its root.  Walks only read, and each store writes a
    // root, so a concurrent walk through a stored entry still ends at the same root.
    for (u32 r = tid; r < nruns; r += BW) {
        u32 x = ld_wg(&s.par[r]);
        for (u32 it = 0; it < MAX_RUNS; ++it) {
            const u32 y = ld_wg(&s.par[x]);
            if (y == x) break;
            x = y;
        }
        st_wg(&s.par[r], x);
    }
    lds_barrier();
    // roots (parent == self) number the clusters in order of their smallest index
    set_bits([&](u32 r) { return r < nruns && ld_wg(&s.par[r]) == r; });
    lds_barrier();
    u32 ncl;
    {
        u32 sw[KPT], cnt = 0;
#pragma unroll
        for (u32 i = 0; i < KPT; ++i) {
            const u32 w = tid * KPT + i;
            sw[i] = w < KW ? __popc(s.rootb[w]) : 0u;
            cnt += sw[i];
        }
        u32 run = group_excl_scan<BW>(cnt, tid, s.wsum, ncl);
#pragma unroll
        for (u32 i = 0; i < KPT; ++i) {
            const u32 w = tid * KPT + i;
            if (w < KW) s.rootp[w] = u16(run);
            run += sw[i];
        }
    }
    lds_barrier();
    // Every run's cluster as a u16 over the first half of the parents (each thread reads
    // its RPT consecutive runs before any is written); the second half then holds the
    // first LCAP clusters' charge | size << 44 (LDS atomics), the others' sums go to
    // device memory.
    constexpr u32 RPT = (MAX_RUNS + BW - 1) / BW, LCAP = MAX_RUNS * 2 / 8;
    u16* cl = reinterpret_cast<u16*>(s.par);
    u64* acc = reinterpret_cast<u64*>(reinterpret_cast<u8*>(s.par) + size_t(MAX_RUNS) * 2);
    {
        u32 cv[(RPT + 1) / 2];
#pragma unroll
        for (u32 i = 0; i < RPT; ++i) {
            const u32 r = tid * RPT + i;
            const u32 c = r < nruns ? cluster_of(r) : 0u;
            if (i & 1u) cv[i / 2] |= c << 16;
            else cv[i / 2] = c;
        }
        lds_barrier();
#pragma unroll
        for (u32 i = 0; i < RPT; ++i) {
            const u32 r = tid * RPT + i;
            if (r < nruns) cl[r] = u16(cv[i / 2] >> (16 * (i & 1u)));
        }
    }
    lds_barrier();
    // per cluster: id from the start of its root run; zero the sums
    for (u32 c = tid; c < min(ncl, LCAP); c += BW) acc[c] = 0ull;
    for (u32 w = tid; w < WORDS; w += BW) {
        u32 sb = run_starts(s.bm, w);
        u32 r = s.rpre[w];
        while (sb) {
            const u32 b = __ffs(sb) - 1;
            sb &= sb - 1;
            if (s.rootb[r >> 5] & (1u << (r & 31u))) {
                const u32 c = u32(s.rootp[r >> 5]) + __popc(s.rootb[r >> 5] & ((1u << (r & 31u)) - 1u));
                cid[c] = I.mod * PIX + (w << 5) + b;
                if (c >= LCAP) {
                    cch[c] = 0u;
                    csz[c] = 0u;
                }
            }
            ++r;
        }
    }
    wait_all_mem();
    lds_barrier();
    for (u32 base = 0; base < n; base += SPAN) {               // pass 2: charge and size
        u32 lin[UNR], adc[UNR];
        fetch(base, lin, adc);
        u32 c[UNR];
#pragma unroll
        for (u32 u = 0; u < UNR; ++u) c[u] = lin[u] != NOPIX ? u32(cl[run_of(s.bm, s.rpre, lin[u])]) : 0u;
        // when each thread's digis here belong to one cluster (a cluster spanning the
        // module, as in a serpentine), the thread adds them up first: one wave sum
        // instead of one per slot
        u32 c0 = NOPIX;
        u64 tot = 0;
        bool one = true;
#pragma unroll
        for (u32 u = 0; u < UNR; ++u)
            if (lin[u] != NOPIX) {
                one = one && (c0 == NOPIX || c[u] == c0);
                c0 = c[u];
                tot += (1ull << 44) | adc[u];
            }
        if (__ballot(!one) == 0ull) {
            const bool v = c0 != NOPIX;
            wave_add_lds64(acc, c0, tot, v && c0 < LCAP);
            wave_add(cch, c0, u32(tot & 0xFFFFFFFFFFFull), v && c0 >= LCAP);
            wave_add(csz, c0, u32(tot >> 44), v && c0 >= LCAP);
        } else {
#pragma unroll
            for (u32 u = 0; u < UNR; ++u) {
                const bool v = lin[u] != NOPIX;
                wave_add_lds64(acc, c[u], (1ull << 44) | adc[u], v && c[u] < LCAP);
                wave_add(cch, c[u], adc[u], v && c[u] >= LCAP);
                wave_add(csz, c[u], 1u, v && c[u] >= LCAP);
            }
        }
    }
    wait_all_mem();
    lds_barrier();
    // cut; kept clusters -> staging records in cluster (= ascending id) order
    set_bits([&](u32 c) { return c < ncl && (c < LCAP ? u32(acc[c]) : ld_ag(&cch[c])) >= a.charge_cut; });
    lds_barrier();
    u32 Kc;
    {
        u32 sw[KPT], cnt = 0;
#pragma unroll
        for (u32 i = 0; i < KPT; ++i) {
            const u32 w = tid * KPT + i;
            sw[i] = w < KW ? __popc(s.rootb[w]) : 0u;
            cnt += sw[i];
        }
        u32 run = group_excl_scan<BW>(cnt, tid, s.wsum, Kc);
        u32 keep_pre[KPT];
#pragma unroll
        for (u32 i = 0; i < KPT; ++i) {
            keep_pre[i] = run;
            run += sw[i];
        }
        int32_t* tid_ = ws_ptr<int32_t>(E, L.tid);
        int32_t* tch = ws_ptr<int32_t>(E, L.tcharge);
        int32_t* tsz = ws_ptr<int32_t>(E, L.tsize);
#pragma unroll
        for (u32 i = 0; i < KPT; ++i) {
            const u32 w = tid * KPT + i;
            if (w >= KW) continue;
            u32 pos = keep_pre[i];
            s.rootp[w] = u16(pos);                              // kept clusters before word w
            for (u32 b = 0; b < 32; ++b) {
                const u32 c = w * 32 + b;
                if (c >= ncl) break;
                const bool lds = c < LCAP;
                if (s.rootb[w] & (1u << b)) {
                    const u32 id = ld_ag(&cid[c]);
                    const u64 v = lds ? acc[c] : 0ull;
                    tid_[st + pos] = int32_t(id);
                    tch[st + pos] = int32_t(lds ? u32(v) : ld_ag(&cch[c]));
                    tsz[st + pos] = int32_t(lds ? u32(v >> 44) : ld_ag(&csz[c]));
                    ++pos;
                    if (lds) acc[c] = u64(id);                  // for the per-digi ids
                } else if (lds) {
                    acc[c] = u64(NOPIX);
                } else {
                    st_ag(&cid[c], NOPIX);
                }
            }
        }
        if (tid == 0) ws_ptr<u32>(E, L.kept)[I.it] = Kc;
    }
    wait_all_mem();
    lds_barrier();
    for (u32 base = 0; base < n; base += SPAN) {               // pass 3: per-digi ids
        u32 lin[UNR], adc3[UNR];
        fetch(base, lin, hits ? adc3 : nullptr);
        u32 c[UNR];
#pragma unroll
        for (u32 u = 0; u < UNR; ++u) c[u] = lin[u] != NOPIX ? u32(cl[run_of(s.bm, s.rpre, lin[u])]) : 0u;
#pragma unroll
        for (u32 u = 0; u < UNR; ++u) {
            const u32 j = base + u * BW + tid;
            const u32 id = c[u] < LCAP ? u32(acc[c[u]]) : ld_ag(&cid[c[u]]);
            if (j < n) od[out_pos(perm, st + j)] = lin[u] != NOPIX ? int32_t(id) : -1;
            if (hits && lin[u] != NOPIX && id != NOPIX) {           // kept: add to its record's sums
                const u32 cw = c[u] >> 5, q = st + s.rootp[cw] + __popc(s.rootb[cw] & ((1u << (c[u] & 31u)) - 1u));
                const u64 w = adc3[u], col = lin[u] / ROWS;
                atomicAdd(&hs[2 * q], w * col);
                atomicAdd(&hs[2 * q + 1], w * (lin[u] - col * ROWS));
            }
        }
    }
    if (err) atomicOr(ws_ptr<u32>(E, L.ctl) + CTL_ERR, err);
    lds_barrier();                                              // every thread is done with the bitmap
    for (u32 w = tid; w < WORDS; w += BW) s.bm[w] = 0u;
    lds_barrier();
}

// Entry t of the launch's big-module (or scratch-mode) lists (prefix s_pref): the
// module and its digis; ok when it is one the small kernel listed (above its
// capacity).
__device__ __forceinline__ Item big_item(const LaunchArgs& a, const u32* s_pref, u32 k, u32 t, bool scr) {
    Item I{0, 0, 0, 0, 0, false};
    I.e = find_slot(s_pref, k, t);
    const EventDesc E = get_event(a, I.e);
    const EvLayout L = ev_layout(E.cap, a.n_modules);
    I.mod = I.it = ws_ptr<const u32>(E, scr ? L.scr : L.big)[t - s_pref[I.e]];
    if (I.mod < a.n_modules) {
        const ModRange r = ws_ptr<const ModRange>(E, L.mtab)[I.mod];
        const u32 st = u32(r.first), en = u32(r.end);
        if (u32(r.first >> 32) == E.epoch && u32(r.end >> 32) == E.epoch && st < en && en <= E.n) {
            I.st = st;
            I.n = en - st;
            I.ok = scr ? I.n > BIG_RCAP : (I.n > a.dcap && I.n <= BIG_RCAP);
        }
    }
    if (!I.ok && threadIdx.x == 0) atomicOr(ws_ptr<u32>(E, L.ctl) + CTL_ERR, EB_INTERNAL);
    return I;
}

// big, register mode: the modules of the big-module list (above the small kernel's
// capacity, up to BIG_RCAP digis)
__global__ __launch_bounds__(B_WG) void k_big(LaunchArgs a) {
    __shared__ RegModuleSmem<B_WG, K_BIG> s;
    __shared__ u32 s_pref[MAXB + 1];
    __shared__ u32 s_wsum[B_WG / 64];
    const u32 tid = threadIdx.x;
    for (u32 w = tid; w < WORDS; w += B_WG) s.bm[w] = 0u;
    if (tid < CMW) s.cm[tid] = 0u;
    const u32 k = num_events(a);
    const u32 total = event_prefix<B_WG>(a, k, s_pref, s_wsum, CTL_BIG, 1, 0);
    for (u32 t = blockIdx.x; t < total; t += gridDim.x) {
        const Item I = big_item(a, s_pref, k, t, false);
        if (!I.ok) continue;
        const EventDesc E = get_event(a, I.e);
        const EvLayout L = ev_layout(E.cap, a.n_modules);
        u32 RC[K_BIG], A[K_BIG];
        fetch_digis<B_WG, K_BIG>(E, I, tid, RC, A);
        cluster_regs<B_WG, K_BIG>(a, E, L, I, s, tid, RC, A, [](int) {});
    }
}

// big, scratch mode: the modules of the scratch-mode list (above BIG_RCAP digis), in
// workgroups of S_WG threads (more waves for the column-ordered unions, a chain of
// steps per wave)
__global__ __launch_bounds__(S_WG) void k_scratch(LaunchArgs a) {
    __shared__ BigScratchSmem<S_WG> s;
    __shared__ u32 s_pref[MAXB + 1];
    __shared__ u32 s_wsum[S_WG / 64];
    const u32 tid = threadIdx.x;
    for (u32 w = tid; w < WORDS; w += S_WG) s.bm[w] = 0u;
    const u32 k = num_events(a);
    const u32 total = event_prefix<S_WG>(a, k, s_pref, s_wsum, CTL_SCR, 1, 0);
    for (u32 t = blockIdx.x; t < total; t += gridDim.x) {
        const Item I = big_item(a, s_pref, k, t, true);
        if (!I.ok) continue;
        const EventDesc E = get_event(a, I.e);
        cluster_scratch<S_WG>(a, E, ev_layout(E.cap, a.n_modules), I, s);
    }
}

// ---------------------------------------------------------------------------
// compact: S waves per block of C_BLK consecutive modules of an event (every module,
// present or not: an absent module keeps nothing).  The block's first output
// position is the sum of the kept counts of the modules before it, which each of its
// waves adds up (PS_UNR loads per lane in flight); a wave scan over the block's 64
// counts gives every module its position, and wave s of the block copies the s-th
// of S equal shares of the block's records, 64 at a time, each lane finding its
// record's module by a search over that scan.  S (a power of two, at most C_SPLIT)
// follows from the grid: launches of few blocks (one event of few modules) spread
// each block's copy over many waves, launches of many blocks keep one wave per
// block.  Wave 0 of an event's last block has the event's total and writes the
// status back to the host.  Loads per event grow as (modules / 64)^2 * 64 * S.
// ---------------------------------------------------------------------------
constexpr u32 CP_UNR = 4, PS_UNR = 16, C_WAVES = C_WG / 64, C_BLK = 64, C_SPLIT = 32;

__device__ __forceinline__ u32 compact_blocks(u32 n_modules) { return (n_modules + C_BLK - 1) / C_BLK; }

// Waves per block for a launch of `waves` waves over `blocks` blocks.
__host__ __device__ __forceinline__ u32 compact_split(u32 waves, u32 blocks) {
    u32 sp = 1;
    while (sp < C_SPLIT && u64(sp) * 2 * blocks <= waves) sp *= 2;
    return sp;
}

// Sum of kept[0, end) over the wave (end a multiple of 64).
__device__ __forceinline__ u32 kept_before(const u32* kept, u32 end, u32 lane) {
    u32 part = 0;
    for (u32 b = 0; b < end; b += 64 * PS_UNR) {
        u32 v[PS_UNR];
#pragma unroll
        for (u32 q = 0; q < PS_UNR; ++q) {
            const u32 i = b + q * 64 + lane;
            v[q] = i < end ? kept[i] : 0u;
        }
#pragma unroll
        for (u32 q = 0; q < PS_UNR; ++q) part += v[q];
    }
    return __shfl(wave_incl_scan(part), 63, 64);
}

__global__ __launch_bounds__(C_WG) void k_compact(LaunchArgs a) {
    const u32 tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    const u32 k = num_events(a), M = a.n_modules, nblk = compact_blocks(M);
    if (blockIdx.x == 0 && tid == 0) st_ag(&a.ctr[S_TICK], 0u);   // the small kernel has finished
    const u32 sp = compact_split(gridDim.x * C_WAVES, k * nblk);
    const u32 total = k * nblk * sp;
    for (u32 u = wave_uniform(xcd_order(blockIdx.x, gridDim.x) * C_WAVES + wv); u < total; u += gridDim.x * C_WAVES) {
        const u32 eb = u / sp, part = u - eb * sp;
        const u32 e = eb / nblk, b = eb - e * nblk;
        const EventDesc E = wave_uniform(get_event(a, e));
        const EvLayout L = ev_layout(E.cap, M);
        u32* ctl = ws_ptr<u32>(E, L.ctl);
        const u32* kept = ws_ptr<const u32>(E, L.kept);
        if ((a.flags & LF_DEFER) && (ld_ag(ctl + CTL_BIG) | ld_ag(ctl + CTL_SCR)) != 0u) {
            // modules wait for the big-module kernels of a second launch: nothing is
            // compacted, the lists and error bits stay for it, the host learns why
            if (b + 1 == nblk && part == 0 && lane == 0) {
                ctl[CTL_DEFERRED] = 1u;
                u32* hs = E.hstat;
                st_sys(&hs[HS_ERR], ctl[CTL_ERR] | EB_DEFER);
                st_sys(&hs[HS_NCL], 0u);
                st_sys(&hs[HS_EPOCH], E.epoch);
            }
            continue;
        }
        if ((a.flags & LF_SECOND) && ld_ag(ctl + CTL_DEFERRED) == 0u) continue;   // finished by the first launch
        const u32 m = b * C_BLK + lane;
        // an empty event's kept counts were never written: it has no clusters
        const bool live = E.n != 0 && m < M;
        u32 cnt = live ? kept[m] : 0u;
        const u32 src = live ? u32(ws_ptr<const ModRange>(E, L.mtab)[m].first) : 0u;
        const u32 base = E.n ? wave_uniform(kept_before(kept, b * C_BLK, lane)) : 0u;
        if (cnt > E.n) cnt = 0u;                           // inconsistent (only after an input error)
        const u32 incl = wave_incl_scan(cnt), excl = incl - cnt;
        const u32 T = wave_uniform(__shfl(incl, 63, 64));
        const bool fits = base <= E.n && T <= E.n - base;  // every position below n
        if (b + 1 == nblk && part == 0 && lane == 0) {     // the event's status
            const u32 ncl = fits ? base + T : E.n;
            const u32 err = ctl[CTL_ERR];
            ctl[CTL_ERR] = 0u;
            st_ag(ctl + CTL_BIG, 0u);                      // the big kernels have run (other waves
            st_ag(ctl + CTL_SCR, 0u);                      // of the event may read them atomically)
            ctl[CTL_NCL] = ncl;
            u32* hs = E.hstat;
            st_sys(&hs[HS_ERR], err);
            st_sys(&hs[HS_NCL], ncl);
            st_sys(&hs[HS_EPOCH], E.epoch);
        }
        if (!fits || T == 0) continue;
        if (cnt && part == 0) ws_ptr<u32>(E, L.off)[m] = base + excl;
        const bool src_ok = cnt == 0 || src <= E.n - cnt;
        const int32_t* tid_ = ws_ptr<const int32_t>(E, L.tid);
        const int32_t* tch = ws_ptr<const int32_t>(E, L.tcharge);
        const int32_t* tsz = ws_ptr<const int32_t>(E, L.tsize);
        int32_t* oid = E.o_id;
        int32_t* och = E.o_charge;
        int32_t* osz = E.o_size;
        const bool hits = (E.flags & EF_HITS) != 0;
        u64* hsm = ws_ptr<u64>(E, L.hsum);
        float* hx = ws_ptr<float>(E, L.hit_x);
        float* hy = ws_ptr<float>(E, L.hit_y);
        const u32 mod_src = src_ok ? src : NOPIX;          // a record of a bad module is skipped
        const u32 j_lo = u32(u64(T) * part / sp), j_hi = u32(u64(T) * (part + 1) / sp);
        for (u32 j0 = j_lo; j0 < j_hi; j0 += 64 * CP_UNR) {
            int32_t r0[CP_UNR], r1[CP_UNR], r2[CP_UNR];
            u64 sx[CP_UNR], sy[CP_UNR];
            u32 from[CP_UNR];
#pragma unroll
            for (u32 q = 0; q < CP_UNR; ++q) {
                const u32 j = j0 + q * 64 + lane;
                // the module holding record j: the first lane whose inclusive count exceeds j
                u32 lo = 0;
#pragma unroll
                for (u32 step = 32; step; step >>= 1)
                    if (__shfl(incl, lo + step - 1, 64) <= j) lo += step;
                const u32 s0 = __shfl(mod_src, lo, 64), x0 = __shfl(excl, lo, 64);
                from[q] = (j < j_hi && s0 != NOPIX) ? s0 + (j - x0) : NOPIX;
                const u32 fs = from[q] != NOPIX ? from[q] : 0u;
                r0[q] = tid_[fs];
                r1[q] = tch[fs];
                r2[q] = tsz[fs];
                sx[q] = sy[q] = 0ull;
                if (hits && from[q] != NOPIX) {
                    sx[q] = hsm[2 * fs];
                    sy[q] = hsm[2 * fs + 1];
                }
            }
#pragma unroll
            for (u32 q = 0; q < CP_UNR; ++q) {
                const u32 j = j0 + q * 64 + lane;
                if (from[q] != NOPIX) {
                    oid[base + j] = r0[q];
                    och[base + j] = r1[q];
                    osz[base + j] = r2[q];
                    if (hits) {                            // the centroid, as the hits kernel computes it
                        const u32 ch = u32(r1[q]);
                        hx[base + j] = ch ? float(double(sx[q]) / double(ch)) : __int_as_float(0x7FC00000);
                        hy[base + j] = ch ? float(double(sy[q]) / double(ch)) : __int_as_float(0x7FC00000);
                        hsm[2 * from[q]] = 0ull;           // the sums are zero again for the next launch
                        hsm[2 * from[q] + 1] = 0ull;
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// hits: per kept cluster the charge-weighted centroid of its pixels, x = sum(adc*col)
// / charge and y = sum(adc*row) / charge, from exact 64-bit sums, divided in double
// and rounded to float (NaN for zero charge).  One workgroup per module with kept
// clusters: the module's cluster ids (ascending) go to LDS, H_CAP at a time; every
// digi of the module whose id falls in the held range finds its cluster by binary
// search and adds its weighted coordinates with LDS atomics.
// ---------------------------------------------------------------------------
constexpr u32 H_WG = 64, H_CAP = 512;     // one wave, ~10 KB of LDS: every module resident at once

__global__ __launch_bounds__(H_WG) void k_hits(LaunchArgs a) {
    __shared__ u32 s_pref[MAXB + 1];
    __shared__ u32 s_wsum[H_WG / 64];
    __shared__ int32_t s_id[H_CAP];
    __shared__ u64 s_sx[H_CAP], s_sy[H_CAP];
    const u32 tid = threadIdx.x;
    const u32 k = num_events(a);
    const u32 total = event_prefix<H_WG>(a, k, s_pref, s_wsum, CNT_UNITS, 1, 0);
    for (u32 t = xcd_order(blockIdx.x, gridDim.x); t < total; t += gridDim.x) {
        const u32 e = find_slot(s_pref, k, t);
        const EventDesc E = get_event(a, e);
        const EvLayout L = ev_layout(E.cap, a.n_modules);
        const u32 mod = unit_module(a, E, L, s_pref[e + 1] - s_pref[e], t - s_pref[e]);
        const u32 cnt = ws_ptr<const u32>(E, L.kept)[mod];
        if (cnt == 0) continue;                            // absent, or nothing kept
        const ModRange r = ws_ptr<const ModRange>(E, L.mtab)[mod];
        const u32 st = u32(r.first), nd = u32(r.end) - st;
        const u32 off = ws_ptr<const u32>(E, L.off)[mod];
        if (cnt > E.n || off > E.n - cnt || st > E.n || nd > E.n - st) continue;
        const int32_t* ids = E.o_id + off;
        const int32_t* chg = E.o_charge + off;
        const int32_t* dcl = E.o_digi;
        const u32* perm = perm_of(E, L);
        float* hx = ws_ptr<float>(E, L.hit_x) + off;
        float* hy = ws_ptr<float>(E, L.hit_y) + off;
        for (u32 c0 = 0; c0 < cnt; c0 += H_CAP) {
            const u32 len = min(H_CAP, cnt - c0);
            for (u32 c = tid; c < len; c += H_WG) {
                s_id[c] = ids[c0 + c];
                s_sx[c] = 0ull;
                s_sy[c] = 0ull;
            }
            lds_barrier();
            const int32_t lo = s_id[0], hi = s_id[len - 1];
            for (u32 j = tid; j < nd; j += H_WG) {
                const int32_t id = dcl[out_pos(perm, st + j)];
                if (id < lo || id > hi) continue;          // cut (-1) or held by another chunk
                u32 l = 0, h = len;
                while (h - l > 1) {
                    const u32 m = (l + h) >> 1;
                    if (s_id[m] <= id) l = m; else h = m;
                }
                if (s_id[l] != id) continue;
                const u64 w = E.adc[st + j];
                atomicAdd(&s_sx[l], w * E.col[st + j]);
                atomicAdd(&s_sy[l], w * E.row[st + j]);
            }
            lds_barrier();
            for (u32 c = tid; c < len; c += H_WG) {
                const u32 q = u32(chg[c0 + c]);
                hx[c0 + c] = q ? float(double(s_sx[c]) / double(q)) : __int_as_float(0x7FC00000);
                hy[c0 + c] = q ? float(double(s_sy[c]) / double(q)) : __int_as_float(0x7FC00000);
            }
            lds_barrier();
        }
    }
}

// ---------------------------------------------------------------------------
// fill: n words at p set to v (clears control words with a kernel node, which a
// caller's graph capture may record, instead of a memset node)
// ---------------------------------------------------------------------------
constexpr u32 F_WG = 256;
__global__ __launch_bounds__(F_WG) void k_fill(u32* p, u32 n, u32 v) {
    for (u32 i = blockIdx.x * F_WG + threadIdx.x; i < n; i += gridDim.x * F_WG) p[i] = v;
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

int occupancy_segment() {
    return std::min(occ(reinterpret_cast<const void*>(k_segment<A_PER_N>), A_WG),
                    occ(reinterpret_cast<const void*>(k_segment<A_PER_W>), A_WG));
}
int occupancy_cluster(u32 wg, u32 mpw) {
    SmallKernel f = small_kernel(wg, mpw);
    return f ? occ(reinterpret_cast<const void*>(f), int(wg)) : 0;
}
int occupancy_big() { return occ(reinterpret_cast<const void*>(k_big), B_WG); }
int occupancy_scratch() { return occ(reinterpret_cast<const void*>(k_scratch), S_WG); }
int occupancy_compact() { return occ(reinterpret_cast<const void*>(k_compact), C_WG); }

int occupancy_group() {
    return std::min(occ(reinterpret_cast<const void*>(k_group_count), G_WG),
                    occ(reinterpret_cast<const void*>(k_group_scatter), G_WG));
}
u32 group_chunk() { return G_CH; }
u32 group_scatter_chunk() { return G_SCH; }
// The grouping kernels of the events in any order: count over `grid` workgroups,
// the table over `grid_events`, scatter over `grid_scatter`.
hipError_t launch_group(const LaunchArgs& a, u32 grid, u32 grid_events, u32 grid_scatter, hipStream_t s) {
    hipLaunchKernelGGL(k_group_count, dim3(grid), dim3(G_WG), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_group_table, dim3(grid_events), dim3(G_WG), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_group_scatter, dim3(grid_scatter), dim3(G_WG), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_segment(const LaunchArgs& a, u32 grid, hipStream_t s) {
    if (a.flags & LF_SEG_WIDE) hipLaunchKernelGGL(k_segment<A_PER_W>, dim3(grid), dim3(A_WG), 0, s, a);
    else hipLaunchKernelGGL(k_segment<A_PER_N>, dim3(grid), dim3(A_WG), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_small(u32 wg, u32 mpw, const LaunchArgs& a, u32 grid, hipStream_t s) {
    SmallKernel f = small_kernel(wg, mpw);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(grid), dim3(wg), 0, s, a);
    return hipGetLastError();
}
// The two big-module kernels (register mode, then scratch mode unless LF_NO_SCRATCH).
hipError_t launch_big(const LaunchArgs& a, u32 grid, u32 grid_scratch, hipStream_t s) {
    hipLaunchKernelGGL(k_big, dim3(grid), dim3(B_WG), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || (a.flags & LF_NO_SCRATCH)) return e;
    hipLaunchKernelGGL(k_scratch, dim3(grid_scratch), dim3(S_WG), 0, s, a);
    return hipGetLastError();
}
u32 compact_waves_per_block(u32 waves, u32 blocks) { return compact_split(waves, blocks); }
hipError_t launch_compact(const LaunchArgs& a, u32 grid, hipStream_t s) {
    hipLaunchKernelGGL(k_compact, dim3(grid), dim3(C_WG), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_fill(u32* p, u32 n, u32 v, hipStream_t s) {
    if (!n) return hipSuccess;
    const u32 grid = std::min<u32>((n + F_WG - 1) / F_WG, 1024u);
    hipLaunchKernelGGL(k_fill, dim3(grid), dim3(F_WG), 0, s, p, n, v);
    return hipGetLastError();
}
int occupancy_hits() { return occ(reinterpret_cast<const void*>(k_hits), H_WG); }
hipError_t launch_hits(const LaunchArgs& a, u32 grid, hipStream_t s) {
    hipLaunchKernelGGL(k_hits, dim3(grid), dim3(H_WG), 0, s, a);
    return hipGetLastError();
}

}  // namespace pxcl
