// Internal layout shared by the device kernels and the host runtime of the
// pixel-clustering library.  Not part of the C ABI (include/pxcl.h is).
#pragma once
#include <stddef.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define PXCL_HD __host__ __device__
#else
#define PXCL_HD
#endif

namespace pxcl {

typedef uint8_t u8;
typedef uint16_t u16;
typedef uint32_t u32;
typedef uint64_t u64;

// Module geometry.  Linear pixel index inside a module is column-major,
// lin = col*ROWS + row, so a column is 5 consecutive 32-bit bitmap words and a
// word never straddles two columns.
constexpr u32 ROWS = 160, COLS = 416, PIX = ROWS * COLS;
constexpr u32 WORDS = PIX / 32;          // 2080 bitmap words per module
constexpr u32 WPC = ROWS / 32;           // 5 words per column
constexpr u32 MAX_RUNS = PIX / 2;        // vertical runs in a module (alternating pixels)
constexpr u32 MAXB = 128;                // events per batch

// Kernel shapes.
constexpr u32 A_WG = 256;                                   // segmentation: ids per thread,
constexpr u32 A_PER_N = 8, A_PER_W = 32;                    // narrow chunks for launches that
                                                            // cannot fill the device, wide ones
                                                            // (fewer end-of-chunk atomics) else
constexpr u32 C_WG = 256;                                   // compaction: a wave per module
constexpr u32 K_SMALL = 8;                                  // digis per thread (small-module kernel)
constexpr u32 B_WG = 512, K_BIG = 32;                       // big-module kernel
constexpr u32 BIG_RCAP = B_WG * K_BIG;                      // 16384: larger modules use scratch mode
constexpr u32 S_WG = 1024;                                  // scratch-mode kernel

// Per-event control words (u32) at the start of an event workspace.
enum : u32 {
    CTL_ERR = 0,      // accumulated PXCL_ERRBIT_* of the launch in progress
    CTL_NCL = 2,      // kept clusters
    CTL_BIG = 4,      // modules on the big-module list (register mode)
    CTL_SCR = 3,      // modules on the scratch-mode list
    CTL_PRESENT = 5,  // words 5-6: modules on the present-module list, one count per
                      // launch parity (EventDesc::slot); a launch clears the other one
    CTL_DEFERRED = 7, // 1: a batch launch with LF_DEFER left this event to its second
                      // launch (set by the compaction, cleared by segmentation or grouping)
    CTL_CTR = 8,      // launch counters when the event is launched on its own
    CTL_WORDS = 64
};
// Launch counters: the small-module kernel's ticket.
enum : u32 { S_TICK = 0, N_CTR = 8 };
// Host status block (pinned) written by the compaction kernel.
enum : u32 { HS_EPOCH = 0, HS_ERR = 1, HS_NCL = 2, HS_WORDS = 16 };
constexpr u32 HS_BYTES = HS_WORDS * 4;

// Error bits (same values as PXCL_ERRBIT_*).
constexpr u32 EB_RANGE = 1, EB_ORDER = 2, EB_DUP = 4, EB_INTERNAL = 8, EB_HINT = 16;
// Not an error: a launch with LF_DEFER found modules above the small kernel's
// capacity, listed them and left the compaction to a second launch (big-module
// kernels, then the compaction), which the host queues.
constexpr u32 EB_DEFER = 32;

// Launch flags.
constexpr u32 LF_NO_BIG = 1;     // the big-module kernel is not launched (size hint)
constexpr u32 LF_SEG_WIDE = 2;   // segmentation in wide chunks
constexpr u32 LF_FUSED = 4;      // one event, no segmentation kernel: the small kernel
                                 // finds every module's digis by search
constexpr u32 LF_NO_SCRATCH = 8; // the scratch-mode kernel is not launched (size hint)
constexpr u32 LF_GROUP = 16;     // some event is in any order: the grouping kernels run first
constexpr u32 LF_NO_SEG = 32;    // no event is grouped by module: no segmentation kernel
constexpr u32 LF_DEFER = 64;     // with LF_NO_BIG | LF_NO_SCRATCH: modules above the small
                                 // kernel's capacity are listed as usual, and an event with
                                 // any is not compacted but reported with EB_DEFER
constexpr u32 LF_SECOND = 128;   // the second launch of a deferred batch: the compaction
                                 // takes only the events the first one left (CTL_DEFERRED)
PXCL_HD constexpr u32 seg_chunk(u32 flags) { return A_WG * ((flags & LF_SEG_WIDE) ? A_PER_W : A_PER_N); }

// Event flags (EventDesc::flags).
constexpr u32 EF_UNSORTED = 1;   // the digis are in any order: the grouping kernels read them
                                 // from r_*, write a copy grouped by module to the workspace
                                 // (module..adc point there) and each grouped digi's input
                                 // position (perm), where its per-digi output goes
constexpr u32 EF_HITS = 2;       // hits fused into the clustering: every kept digi adds
                                 // adc*col and adc*row to its cluster's staging sums (hsum),
                                 // the compaction writes x and y beside each record and
                                 // zeroes the sums it read: they are zero between launches
                                 // (binding clears them, and so does the host after a
                                 // launch that failed or reported an error)

// One event as the kernels see it (144 bytes).
struct EventDesc {
    const u16* module;   // digis grouped by module (the input, or the workspace's grouped copy)
    const u16* row;
    const u16* col;
    const u16* adc;
    const u16* r_module; // with EF_UNSORTED: the digis as given (any order)
    const u16* r_row;
    const u16* r_col;
    const u16* r_adc;
    u8* ws;              // event workspace (device)
    u32* hstat;          // status block (pinned host memory or device memory)
    int32_t* o_digi;     // per-digi cluster ids [n], in input order
    int32_t* o_id;       // kept clusters (ascending id); room for n entries each, used as
    int32_t* o_charge;   // per-cluster temporaries of the big-module kernel's scratch mode
    int32_t* o_size;
    u32 n;               // digis
    u32 cap;             // workspace capacity in digis
    u32 epoch;           // launch tag of the module-table words
    u32 slot;            // launch parity: which present-module count this launch uses
    u32 flags;           // EF_*
    u32 pad[3];
};
static_assert(sizeof(EventDesc) == 144, "EventDesc is 144 bytes");

// A module's digis [first, end), each word tagged with the launch (epoch << 32):
// written by the digis at the module's boundaries, so an entry whose tags are not
// the current launch's belongs to an absent module and needs no clearing.
struct ModRange {
    u64 first, end;
};

// Batch header in device memory: u32 k, padding to 64 bytes, then EventDesc[k].
constexpr u32 HDR_EV_OFFSET = 64;
PXCL_HD inline size_t header_bytes(u32 max_events) { return HDR_EV_OFFSET + size_t(max_events) * sizeof(EventDesc); }

struct LaunchArgs {
    const u32* hdr;     // batch header (device) or nullptr: then `single` is the only event
    u32* ctr;           // N_CTR launch counters (device)
    u32 n_modules;
    u32 charge_cut;
    u32 dcap;           // largest module (digis) the small-module kernel takes
    u32 flags;          // LF_*
    EventDesc single;
};

PXCL_HD constexpr size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Byte offsets of the arrays of an event workspace with capacity N digis and M
// modules per event.
struct EvLayout {
    size_t ctl, in_mod, in_row, in_col, in_adc;
    size_t digi, id, charge, size;           // outputs
    size_t tid, tcharge, tsize;              // cluster records before compaction
    size_t mtab;                             // per module: ModRange
    size_t kept;                             // per module: kept clusters
    size_t big;                              // module ids for the big-module kernel
    size_t scr;                              // module ids for the scratch-mode kernel
    size_t present;                          // module ids of the modules present (any order)
    size_t off;                              // per module: its first cluster in the outputs
    size_t hit_x, hit_y;                     // hits (per kept cluster), when asked for
    size_t perm;                             // digis in any order: input index of each grouped digi
    size_t grp;                              // digis in any order: the grouped copy (4 x u16[N])
    size_t gcnt;                             // digis in any order: per module, digis counted (zero between launches)
    size_t hsum;                             // fused hits: per staged record, sum(adc*col), sum(adc*row) (u64)
    size_t total;
};

PXCL_HD constexpr EvLayout ev_layout(u32 N, u32 M) {
    EvLayout L{};
    size_t o = 0;
    const size_t n = N, m = M;
    L.ctl = o;        o = al256(o + CTL_WORDS * 4);
    L.in_mod = o;     o = al256(o + 2 * n);
    L.in_row = o;     o = al256(o + 2 * n);
    L.in_col = o;     o = al256(o + 2 * n);
    L.in_adc = o;     o = al256(o + 2 * n);
    L.digi = o;       o = al256(o + 4 * n);
    L.id = o;         o = al256(o + 4 * n);
    L.charge = o;     o = al256(o + 4 * n);
    L.size = o;       o = al256(o + 4 * n);
    L.tid = o;        o = al256(o + 4 * n);
    L.tcharge = o;    o = al256(o + 4 * n);
    L.tsize = o;      o = al256(o + 4 * n);
    L.mtab = o;       o = al256(o + 16 * m);
    L.kept = o;       o = al256(o + 4 * m);
    L.big = o;        o = al256(o + 4 * m);
    L.scr = o;        o = al256(o + 4 * m);
    L.present = o;    o = al256(o + 4 * m);
    L.off = o;        o = al256(o + 4 * m);
    L.hit_x = o;      o = al256(o + 4 * n);
    L.hit_y = o;      o = al256(o + 4 * n);
    L.perm = o;       o = al256(o + 4 * n);
    L.grp = o;        o = al256(o + 8 * n);
    L.gcnt = o;       o = al256(o + 4 * m);
    L.hsum = o;       o = al256(o + 16 * n);
    L.total = o;
    return L;
}

// Batch workspace: counters then the header.
constexpr size_t BW_CTR = 0;
constexpr size_t BW_HDR = 256;
PXCL_HD inline size_t batch_ws_bytes(u32 max_events) { return al256(BW_HDR + header_bytes(max_events)); }

}  // namespace pxcl
