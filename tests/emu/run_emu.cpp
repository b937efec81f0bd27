// Runs the device kernel source on the CPU (tests/emu/hip/hip_runtime.h) for one
// launch of k events and writes the results; built with AddressSanitizer so that
// any out-of-bounds access of the kernels aborts the run.  Test infrastructure.
//
// input:  u32 k, n_modules, cut, wg, mpw, grid_a, grid_b, grid_s, grid_c, header
//         (1: the events go through a batch header even when k == 1), launch flags
//         (LF_NO_BIG: the big-module kernel is not run; LF_SEG_WIDE: segmentation in
//         wide chunks; LF_FUSED: no segmentation kernel; LF_DEFER with LF_NO_BIG |
//         LF_NO_SCRATCH: big-module kernels deferred to a second launch, which is run
//         when the first reports it (one event); bit 31: the ticket counter starts
//         non-zero), hits (1: run the hits kernel after the launch);
//         per event: u32 n, u32 cap, u32 flags (1: digis in any order), u16 module[n],
//         row[n], col[n], adc[n]
// output: u32 launches (2 when a deferred launch needed its second one), then per
//         event: u32 err, u32 n_clusters, i32 digi[n], id[nc], charge[nc], size[nc]
//         (with hits: then f32 x[nc], y[nc])
#include "../../paper_2004_04334_amd/csrc/pxcl_kernels.hip"

#include <algorithm>
#include <cstdlib>
#include <random>

using namespace pxcl;

static void rd(FILE* f, void* p, size_t b) {
    if (b && fread(p, 1, b, f) != b) { fprintf(stderr, "short read\n"); exit(2); }
}

int main(int argc, char** argv) {
    if (argc != 3) { fprintf(stderr, "usage: run_emu in out\n"); return 2; }
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    u32 h[12];
    rd(f, h, sizeof(h));
    const u32 k = h[0], M = h[1];
    std::vector<EventDesc> evs(k);
    std::vector<std::vector<u16>> in(k);
    std::vector<u8*> ws(k);
    std::vector<u32*> hs(k);
    std::mt19937 rng(7);
    for (u32 e = 0; e < k; ++e) {
        u32 nc[3];
        rd(f, nc, 12);
        const u32 n = nc[0], cap = nc[1];
        const bool any = (nc[2] & 1u) != 0;
        const bool fused_hits = (nc[2] & 2u) != 0;
        in[e].resize(4 * size_t(n) + 4);
        rd(f, in[e].data(), 8 * size_t(n));
        const EvLayout L = ev_layout(cap, M);
        ws[e] = static_cast<u8*>(aligned_alloc(256, (L.total + 255) / 256 * 256));
        for (size_t i = 0; i < L.total; ++i) ws[e][i] = u8(rng());        // garbage, as fresh device memory
        memset(ws[e] + L.ctl, 0, CTL_WORDS * 4);                           // what binding clears
        // what an earlier launch leaves: module-table entries with its tag and any
        // range; without the fused form also a big-module count that launch did not
        // reset (the segmentation kernel resets it; the fused form relies on the
        // compaction of every finished launch and the host's clear after a failed one)
        ModRange* mt = reinterpret_cast<ModRange*>(ws[e] + L.mtab);
        const u64 old_tag = u64(999 + e) << 32;
        for (u32 m = 0; m < M; ++m) {
            mt[m].first = old_tag | (rng() % (n + 1));
            mt[m].end = old_tag | (rng() % (n + 1));
        }
        if (!(h[10] & LF_FUSED)) reinterpret_cast<u32*>(ws[e] + L.ctl)[CTL_BIG] = 3;
        memset(ws[e] + L.gcnt, 0, size_t(4) * M);                          // what binding clears
        memset(ws[e] + L.hsum, 0, size_t(16) * cap);
        hs[e] = static_cast<u32*>(aligned_alloc(64, HS_BYTES));
        memset(hs[e], 0, HS_BYTES);
        EventDesc& d = evs[e];
        d.module = in[e].data();
        d.row = in[e].data() + n;
        d.col = in[e].data() + 2 * size_t(n);
        d.adc = in[e].data() + 3 * size_t(n);
        if (fused_hits) d.flags |= EF_HITS;
        if (any) {                        // the kernels read the raw digis and cluster a grouped copy
            d.flags |= EF_UNSORTED;
            d.r_module = d.module; d.r_row = d.row; d.r_col = d.col; d.r_adc = d.adc;
            const u16* g = reinterpret_cast<const u16*>(ws[e] + L.grp);
            d.module = g; d.row = g + cap; d.col = g + 2 * size_t(cap); d.adc = g + 3 * size_t(cap);
        }
        d.ws = ws[e];
        d.hstat = hs[e];
        d.o_digi = reinterpret_cast<int32_t*>(ws[e] + L.digi);
        d.o_id = reinterpret_cast<int32_t*>(ws[e] + L.id);
        d.o_charge = reinterpret_cast<int32_t*>(ws[e] + L.charge);
        d.o_size = reinterpret_cast<int32_t*>(ws[e] + L.size);
        d.n = n;
        d.cap = cap;
        d.epoch = 1000 + e;
        d.slot = e & 1u;
    }
    fclose(f);
    LaunchArgs a;
    memset(&a, 0, sizeof(a));
    std::vector<u8> hdr;
    u32 ctr[N_CTR] = {};
    a.ctr = ctr;
    a.n_modules = M;
    a.charge_cut = h[2];
    a.dcap = cluster_capacity(h[3], h[4]);
    // bit 31 of the flags word is the driver's own: the launch starts with a ticket
    // counter left non-zero (a launch before it stopped after the small kernel)
    const bool stale_ticket = (h[10] >> 31) != 0;
    a.flags = h[10] & 0x7FFFFFFFu;
    const bool use_header = h[9] != 0;
    if (k == 1 && !use_header) {
        a.single = evs[0];
    } else {
        hdr.resize(header_bytes(k));
        memcpy(hdr.data(), &k, 4);
        memcpy(hdr.data() + HDR_EV_OFFSET, evs.data(), k * sizeof(EventDesc));
        a.hdr = reinterpret_cast<const u32*>(hdr.data());
        a.ctr = reinterpret_cast<u32*>(aligned_alloc(64, 64));
        memset(a.ctr, 0, 64);
    }
    if (stale_ticket) a.ctr[S_TICK] = 1000003u;
    if (((a.flags & LF_GROUP) && launch_group(a, h[5], h[5], h[5], nullptr)) ||
        (!(a.flags & (LF_FUSED | LF_NO_SEG)) && launch_segment(a, h[5], nullptr)) || launch_small(h[3], h[4], a, h[7], nullptr) ||
        (!(a.flags & LF_NO_BIG) && launch_big(a, h[6], h[6], nullptr)) || launch_compact(a, h[8], nullptr)) {
        fprintf(stderr, "launch failed\n");
        return 3;
    }
    // deferred big-module kernels: the host's second launch when the first reported
    // modules above the small kernel's capacity (one event: with no error; a batch: in
    // any event, and then the compaction takes only the events left unfinished)
    u32 passes = 1;
    bool second = false;
    if (a.flags & LF_DEFER) {
        if (a.hdr) {
            for (u32 e = 0; e < k; ++e)
                second |= hs[e][HS_EPOCH] == evs[e].epoch && (hs[e][HS_ERR] & EB_DEFER) != 0;
        } else {
            second = hs[0][HS_EPOCH] == evs[0].epoch && hs[0][HS_ERR] == EB_DEFER;
        }
    }
    if (second) {
        LaunchArgs a2 = a;
        a2.flags = (a.flags & ~(LF_NO_BIG | LF_NO_SCRATCH | LF_DEFER)) | (a.hdr ? LF_SECOND : 0u);
        if (launch_big(a2, h[6], h[6], nullptr) || launch_compact(a2, h[8], nullptr)) {
            fprintf(stderr, "second launch failed\n");
            return 3;
        }
        passes = 2;
    }
    if (h[11] == 1 && launch_hits(a, h[8], nullptr)) {
        fprintf(stderr, "hits launch failed\n");
        return 3;
    }
    FILE* o = fopen(argv[2], "wb");
    fwrite(&passes, 4, 1, o);
    for (u32 e = 0; e < k; ++e) {
        const EvLayout L = ev_layout(evs[e].cap, M);
        const u32 err = hs[e][HS_ERR], ncl = std::min(hs[e][HS_NCL], evs[e].n);
        const u32 tag = hs[e][HS_EPOCH];
        const u32 hdr2[2] = {tag == evs[e].epoch ? err : (err | 0x80000000u), ncl};
        fwrite(hdr2, 4, 2, o);
        fwrite(ws[e] + L.digi, 4, evs[e].n, o);
        fwrite(ws[e] + L.id, 4, ncl, o);
        fwrite(ws[e] + L.charge, 4, ncl, o);
        fwrite(ws[e] + L.size, 4, ncl, o);
        if (h[11]) {
            fwrite(ws[e] + L.hit_x, 4, ncl, o);
            fwrite(ws[e] + L.hit_y, 4, ncl, o);
        }
    }
    fclose(o);
    for (u32 e = 0; e < k; ++e) { free(ws[e]); free(hs[e]); }
    if (a.hdr) free(a.ctr);
    return 0;
}
