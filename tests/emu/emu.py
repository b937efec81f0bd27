"""Build and run the device kernels on the CPU (hip_runtime.h shim + run_emu.cpp,
AddressSanitizer on) -- test infrastructure for checking kernel indexing and
results without a GPU."""
from __future__ import annotations

import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
BIN = os.path.join(tempfile.gettempdir(), f"pxcl_run_emu_{os.getuid()}")


def build(force: bool = False, sanitizer: str = "address") -> str:
    """Build the emulator and return its path; `sanitizer` is "address" (out-of-bounds
    and null accesses) or "thread" (unsynchronised accesses between the work items of
    a workgroup)."""
    assert sanitizer in ("address", "thread")
    exe = BIN + ("" if sanitizer == "address" else "_tsan")
    srcs = [os.path.join(HERE, "run_emu.cpp"), os.path.join(HERE, "hip", "hip_runtime.h"),
            os.path.join(ROOT, "paper_2004_04334_amd", "csrc", "pxcl_kernels.hip"),
            os.path.join(ROOT, "paper_2004_04334_amd", "csrc", "pxcl_internal.h")]
    if force or not os.path.exists(exe) or os.path.getmtime(exe) < max(os.path.getmtime(s) for s in srcs):
        tmp = exe + f".tmp{os.getpid()}"
        subprocess.check_call(["g++", "-std=c++20", "-O1", "-g", "-x", "c++", f"-fsanitize={sanitizer}",
                               "-fno-omit-frame-pointer", "-pthread", "-I" + HERE,
                               "-I" + os.path.join(ROOT, "paper_2004_04334_amd", "csrc"),
                               os.path.join(HERE, "run_emu.cpp"), "-o", tmp])
        os.replace(tmp, exe)
    return exe


def run(events, n_modules: int, cut: int = 2000, wg: int = 256, mpw: int = 1, grids=(2, 2, 2, 2), caps=None,
        header: bool = False, sanitizer: str = "address", no_big: bool = False, hits: bool = False,
        seg_wide: bool = False, fused: bool = False, stale_ticket: bool = False, any_order=None,
        fused_hits: bool = False, defer: bool = False):
    """Cluster `events` (list of dicts of uint16 arrays) as one launch; returns a list
    of result dicts like the oracle's (status from the error bits).  With `header` the
    events are passed through a batch header even when there is only one; with
    `no_big` the big-module kernel is not run (the launch of a small size hint); with
    `hits` the hits kernel runs after the launch and the results carry "x" and "y";
    `seg_wide` segments in wide chunks (the launch form of many digis); with `fused`
    (one event) there is no segmentation kernel and the small kernel finds the
    module ranges by search (the single-event launch form); with `stale_ticket` the
    launch counters hold a ticket a launch that stopped after its small kernel left.
    `any_order` (one bool per event) flags events whose digis are in any order: the
    grouping kernels run first, and segmentation only if some event is grouped.
    `fused_hits`: every event asks for hits fused into the clustering (no hits kernel;
    the results carry "x" and "y").  `defer` (one event): the big-module kernels are
    deferred, and run with a second compaction only when the first launch reports
    modules for them (through a header: a batch, whose second compaction takes only
    the events left unfinished); every result carries "launches" (1 or 2)."""
    any_order = [False] * len(events) if any_order is None else list(any_order)
    lflags = int(no_big) | (int(seg_wide) << 1) | (int(fused) << 2) | (int(stale_ticket) << 31)
    if defer:
        assert len(events) == 1 or header, "deferred big-module kernels: one event, or a batch header"
        lflags |= 1 | 8 | 64                                  # LF_NO_BIG, LF_NO_SCRATCH, LF_DEFER
    if any(any_order):
        lflags |= 16 | (32 if all(any_order) else 0)        # LF_GROUP, LF_NO_SEG
    exe = build(sanitizer=sanitizer)
    with tempfile.TemporaryDirectory() as d:
        fin, fout = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
        with open(fin, "wb") as f:
            np.array([len(events), n_modules, cut, wg, mpw, *grids, int(header), lflags,
                      2 if fused_hits else int(hits)],
                     dtype=np.uint32).tofile(f)
            for i, ev in enumerate(events):
                n = ev["module"].size
                cap = max(1, n) if caps is None else caps[i]
                np.array([n, cap, int(any_order[i]) | (2 if fused_hits else 0)], dtype=np.uint32).tofile(f)
                for key in ("module", "row", "col", "adc"):
                    np.ascontiguousarray(ev[key], dtype=np.uint16).tofile(f)
        env = dict(os.environ)
        if sanitizer == "thread":        # a smaller history per thread: thousands of short threads
            env["TSAN_OPTIONS"] = "history_size=2 " + env.get("TSAN_OPTIONS", "")
        r = subprocess.run([exe, fin, fout], capture_output=True, text=True, env=env)
        if r.returncode != 0:
            raise RuntimeError(f"emulated kernels failed ({r.returncode}):\n{r.stderr[-4000:]}")
        raw = np.fromfile(fout, dtype=np.int32)
    launches = int(raw[0])
    out, p = [], 1
    for ev in events:
        n = ev["module"].size
        err, ncl = int(np.uint32(raw[p])), int(raw[p + 1])
        p += 2
        digi = raw[p:p + n]; p += n
        cid = raw[p:p + ncl]; p += ncl
        chg = raw[p:p + ncl]; p += ncl
        siz = raw[p:p + ncl]; p += ncl
        hx = hy = None
        if hits or fused_hits:
            hx = raw[p:p + ncl].view(np.float32); p += ncl
            hy = raw[p:p + ncl].view(np.float32); p += ncl
        if err & 32:                      # deferred and not finished: as the host reports it
            err = (err & ~32) | (8 if err == 32 else 0)
        st = 0
        if err & 0x80000000:
            st = -10
        elif err & 1:
            st = -6
        elif err & 2:
            st = -7
        elif err & 16:
            st = -12
        elif err & 4:
            st = -5
        elif err & 8:
            st = -10
        r = {"status": st, "err_bits": err, "n_clusters": ncl, "digi": digi.copy(), "id": cid.copy(),
             "charge": chg.copy(), "size": siz.copy(), "launches": launches}
        if hits or fused_hits:
            r["x"], r["y"] = hx.copy(), hy.copy()
        out.append(r)
    return out
