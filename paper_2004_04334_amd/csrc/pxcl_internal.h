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
constexpr u32 A_WG = 256, A_PER = 8, A_CH = A_WG * A_PER;   // segmentation: digis per chunk
constexpr u32 C_WG = 256, C_CH = 256;                       // compaction: items per chunk
constexpr u32 K_PER = 8;                                    // digis per thread held in registers
constexpr u32 DCAP_MIN = 64 * K_PER;                        // smallest in-LDS module capacity
constexpr u32 L_WG = 1024;                                  // large-module kernel

// Per-event control words (u32) at the start of an event workspace.
enum : u32 {
    CTL_ERR = 0,      // accumulated PXCL_ERRBIT_* of the launch in progress
    CTL_ITEMS = 1,    // number of modules present (work items)
    CTL_NCL = 2,      // kept clusters
    CTL_LARGE = 3,    // items deferred to the large-module kernel
    CTL_CTR = 8,      // 8 launch counters when the event is launched on its own
    CTL_WORDS = 64
};
// Launch counters (tickets and exit counts of the four persistent kernels).
enum : u32 { A_TICK = 0, A_EXIT, B_TICK, B_EXIT, L_TICK, L_EXIT, C_TICK, C_EXIT, N_CTR };
// Host status block (pinned) written by the last kernel of a launch.
enum : u32 { HS_EPOCH = 0, HS_ERR = 1, HS_NCL = 2, HS_ITEMS = 3, HS_LARGE = 4, HS_WORDS = 16 };
constexpr u32 HS_BYTES = HS_WORDS * 4;

// Error bits (same values as PXCL_ERRBIT_*).
constexpr u32 EB_RANGE = 1, EB_ORDER = 2, EB_DUP = 4, EB_INTERNAL = 8;

// One event as the kernels see it (64 bytes).
struct EventDesc {
    const u16* module;
    const u16* row;
    const u16* col;
    const u16* adc;
    u8* ws;          // event workspace (device)
    u32* hstat;      // host status block (pinned, device-accessible)
    u32 n;           // digis
    u32 cap;         // workspace capacity in digis
    u32 epoch;       // launch tag for look-back status words
    u32 pad;
};
static_assert(sizeof(EventDesc) == 64, "EventDesc is 64 bytes");

// Batch header in device memory: u32 k, padding to 64 bytes, then EventDesc[k].
constexpr u32 HDR_EV_OFFSET = 64;
PXCL_HD inline size_t header_bytes(u32 max_events) { return HDR_EV_OFFSET + size_t(max_events) * sizeof(EventDesc); }

struct LaunchArgs {
    const u32* hdr;     // batch header (device) or nullptr: then `single` is the only event
    u32* ctr;           // N_CTR launch counters (device)
    u32 n_modules;
    u32 charge_cut;
    EventDesc single;
};

PXCL_HD inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Byte offsets of the arrays of an event workspace with capacity N digis.
struct EvLayout {
    size_t ctl, in_mod, in_row, in_col, in_adc;
    size_t digi, id, charge, size;           // outputs
    size_t tid, tcharge, tsize;              // cluster records before compaction
    size_t item_start, item_mod, item_kept;  // modules present (work items)
    size_t large;                            // items deferred to the large-module kernel
    size_t lb_a, lb_c;                       // look-back status words
    size_t total;
};

PXCL_HD inline EvLayout ev_layout(u32 N) {
    EvLayout L;
    size_t o = 0;
    const size_t n = N;
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
    L.item_start = o; o = al256(o + 4 * (n + 1));
    L.item_mod = o;   o = al256(o + 4 * n);
    L.item_kept = o;  o = al256(o + 4 * n);
    L.large = o;      o = al256(o + 4 * (n / DCAP_MIN + 2));
    L.lb_a = o;       o = al256(o + 8 * ((n + A_CH - 1) / A_CH + 1));
    L.lb_c = o;       o = al256(o + 8 * ((n + C_CH - 1) / C_CH + 1));
    L.total = o;
    return L;
}

// Bytes that must be zeroed when a workspace is bound: control words and look-back
// status words (everything else is written before it is read).
PXCL_HD inline size_t ev_ctl_bytes() { return CTL_WORDS * 4; }

// Batch workspace: counters then the header.
constexpr size_t BW_CTR = 0;
constexpr size_t BW_HDR = 256;
PXCL_HD inline size_t batch_ws_bytes(u32 max_events) { return al256(BW_HDR + header_bytes(max_events)); }

}  // namespace pxcl
