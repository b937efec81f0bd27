#!/usr/bin/env python3
"""Benchmark of the pixel-clustering path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload all|stress|batch|serve|async|plain|hits|fusedhits]

Default ("all"): one JSON line whose headline (``value``) is the high-pileup stress
configuration, the largest one that runs on one GPU: batches of 16 events of ~320k
digis (16 modules at 20 % occupancy with mean-40 clusters, 142 sparse modules, a
full-column track and a serpentine per event).  A step is one batch launch (the whole
pipeline over 16 events); W untimed launches, then exactly K timed ones, replayed
from captured graphs and spread over 4 streams, with inputs resident in HBM.  The
same line carries, under ``workloads``, the other configurations measured in the
same run with fixed step counts of their own (independent of --steps): ``batch`` (64
events of 10k-120k digis per launch), ``serve`` (Poisson arrivals at 0.5, 0.7 and 0.9
of the saturated rate, continuous batching), ``async`` (~50k-digi events through the
non-blocking acquire/produce boundary from 4 host threads, device- and host-resident
input) and ``plain`` (46,912-digi events, one synchronous launch each).

``roofline`` describes the dominant kernel of the headline: its algorithmic bytes per
launch divided by its mean duration, from hipEvents recorded on the launch stream
around every kernel of launches made one after another on one stream without a
graph (hipEvents cannot be timed inside captured graphs, and on one stream no other
launch shares the compute units); ``--roofline-only`` runs just those launches, which
is the command the committed rocprofv3 summaries profile.  ``cpu_baseline`` times the
plain CPU oracle on the host, on one thread and on all available cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
KERNELS = ["segment", "big", "small", "compact", "hits"]
KERNEL_SYMBOLS = {"segment": "k_segment", "big": "k_big", "small": "k_small", "compact": "k_compact", "hits": "k_hits"}
# kernels behind each timing slot: the big-module slot times register and scratch mode
KERNEL_PARTS = {"big": ["k_big", "k_scratch"]}
ALL_SYMBOLS = list(KERNEL_SYMBOLS.values()) + ["k_scratch"]
METRIC = "events/s + digis/s clustered (frac HBM peak); p50/p99 event latency; host block time"

COPY_BYTES = 1 << 30
SERVE_LOADS = (0.5, 0.7, 0.9)   # serving: offered load as fractions of the saturated rate
SERVE_REQUESTS = 10000          # requests per serving run (p99 over 10,000)
SERVE_SLOTS = 1024              # serving: event slots at most (within the 16 GB budget)
SERVE_INFLIGHT = 6              # serving: batches on the device at once (no batching delay)
LLC_BYTES = 256 << 20           # last-level (Infinity) cache: one-event forms rotate more input than this
SHAPE_TRIAL_LAUNCHES = 160      # batched forms: launches per shape in the throughput trial
N_STREAMS = 4                   # streams the batched workloads spread their launches over
SUB_STEPS = {"batch": 200, "async": 2000, "plain": 2000}   # fixed step counts of the sub-records
ROOFLINE_LAUNCHES = 32          # one-stream graph-free launches timed for the roofline
MAX_CPU_THREADS = 16            # the oracle's N-thread baseline uses at most this many cores


def event_bytes(n_digis: int, n_kept: int) -> int:
    """Algorithmic HBM bytes of one event: read the 8 B/digi SoA, write a 4 B per-digi
    id, 12 B per kept cluster and a 4 B count."""
    return 8 * n_digis + 4 * n_digis + 12 * n_kept + 4


def kernel_src_sha() -> str:
    p = os.path.join(ROOT, "paper_2004_04334_amd", "csrc", "pxcl_kernels.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def load_traffic(workload: str, kernel: str, shape):
    """HBM traffic per launch from the committed rocprofv3 counter summaries of the
    kernels behind a timing slot at the run's small-kernel shape, if they were taken on
    the current kernel source (a kernel without a summary did not run in that
    workload; no summary at all: None)."""
    total, found = 0, False
    if not os.path.exists(os.path.join(ROOT, "profiles", f"kernels_{profile_tag(workload, shape)}.txt")):
        return None
    for sym in KERNEL_PARTS.get(kernel, [KERNEL_SYMBOLS[kernel]]):
        p = os.path.join(ROOT, "profiles", f"pmc_{sym}_{profile_tag(workload, shape)}.json")
        if not os.path.exists(p):
            continue
        d = json.load(open(p))
        if d.get("kernel_src_sha") != kernel_src_sha():
            return None
        total += d.get("traffic_bytes_per_launch", 0)
        found = True
    return total if found else None


def profile_kernel_us(workload: str, shape):
    """Mean kernel durations (us) from the committed rocprofv3 kernel-trace summary of
    the workload at the run's small-kernel shape, if it was taken on the current kernel
    source."""
    p = os.path.join(ROOT, "profiles", f"kernels_{profile_tag(workload, shape)}.txt")
    if not os.path.exists(p):
        return None
    lines = open(p).read().splitlines()
    if not any(l.startswith("kernel source sha256[:16]: ") and l.split(": ")[1].strip() == kernel_src_sha()
               for l in lines):
        return None
    out = {}
    for l in lines:
        f = l.split()
        if len(f) >= 6 and f[0] in ALL_SYMBOLS:
            out[f[0]] = out.get(f[0], 0.0) + float(f[2])
    return out


def roofline(ctx, bytes_per_launch: float, workload: str):
    """Roofline of the dominant kernel from the context's per-kernel hipEvent sums, and
    the same figure from the committed kernel-trace summary of the same launches."""
    ms, cnt = ctx.timing(reset=True)
    avg = {k: (ms[i] / cnt[i] if cnt[i] else 0.0) for i, k in enumerate(KERNELS)}
    if not cnt[KERNELS.index("hits")]:
        del avg["hits"]
    tot = {k: ms[i] for i, k in enumerate(KERNELS)}
    dom = max(tot, key=tot.get)
    t = avg[dom] * 1e-3
    achieved = bytes_per_launch / t / 1e9 if t > 0 else 0.0
    pipe = sum(avg.values()) * 1e-3
    parts = KERNEL_PARTS.get(dom, [KERNEL_SYMBOLS[dom]])
    kt = profile_kernel_us(workload, tuple(ctx.kernel_config()))
    kt_us = sum(kt.get(x, 0.0) for x in parts) if kt else None
    return {
        "bound": "hbm", "kernel": "+".join(parts), "achieved": round(achieved, 2),
        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
        "traffic": load_traffic(workload, dom, tuple(ctx.kernel_config())),
        "algorithmic_bytes_per_launch": int(bytes_per_launch),
        "kernel_mean_us": {k: round(v * 1e3, 3) for k, v in avg.items()},
        "timed_launches": int(max(cnt)),
        "pipeline_us": round(pipe * 1e6, 3),
        "pipeline_GBps": round(bytes_per_launch / pipe / 1e9, 2) if pipe > 0 else 0.0,
        "kernel_trace_us": round(kt_us, 3) if kt_us else None,
        "frac_kernel_trace": round(bytes_per_launch / (kt_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 5) if kt_us else None,
    }


def profile_tag(workload: str, shape) -> str:
    return f"{workload}_{shape[0]}x{shape[1]}"


def profile_commands(workload: str, shape) -> dict:
    """The rocprofv3 commands whose output --summarize-profiles reads (run from the
    repository root with the output directory DIR): the one-stream roofline launches
    of the workload with the small kernel's shape pinned."""
    tag = profile_tag(workload, shape)
    b = f"python3 bench.py --workload {workload} --roofline-only --kernel-config {shape[0]}x{shape[1]}"
    return {
        "kt": f"rocprofv3 --kernel-trace --stats --output-format csv -d DIR/kt_{tag} -o run -- {b}",
        "fetch": f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR/fetch_{tag} -o run -- {b}",
        "write": f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d DIR/write_{tag} -o run -- {b}",
        "copy_fetch": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR/fetch_copy -o run -- "
                      "python3 bench.py --copy-calibration 5",
        "copy_write": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d DIR/write_copy -o run -- "
                      "python3 bench.py --copy-calibration 5",
    }


def copy_bandwidth(torch, reps: int = 10):
    """Achievable HBM bandwidth on this device: a plain device-to-device copy of
    COPY_BYTES (read + write counted), timed with hipEvents."""
    src = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        dst.copy_(src)
    t1.record()
    t1.synchronize()
    dt = t0.elapsed_time(t1) * 1e-3 / reps
    del src, dst
    return round(2 * COPY_BYTES / dt / 1e9, 1)


def copy_calibration(torch, reps: int):
    """Only the device copy (reps launches of COPY_BYTES): the reference for scaling
    rocprofv3 FETCH_SIZE / WRITE_SIZE counters to bytes."""
    gbs = copy_bandwidth(torch, reps)
    print(json.dumps({"copy_bytes": COPY_BYTES, "reps": reps, "copy_GBps": gbs}), flush=True)


# ---------------------------------------------------------------------------
# CPU oracle baseline
# ---------------------------------------------------------------------------
def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_threads() -> int:
    return max(1, min(len(os.sched_getaffinity(0)), MAX_CPU_THREADS))


def oracle_rate(events, seconds: float, threads: int):
    """The oracle as it stands over `events` (cycled) for about `seconds`: one event
    per call, `threads` threads (ctypes releases the interpreter lock during a call)."""
    import threading

    import oracle
    oracle.build()
    stop = time.perf_counter() + seconds
    counts = [[0, 0] for _ in range(threads)]

    def work(t):
        i = t
        while time.perf_counter() < stop:
            ev = events[i % len(events)]
            oracle.cluster_event(ev, 2000)
            counts[t][0] += 1
            counts[t][1] += ev["module"].size
            i += threads

    t0 = time.perf_counter()
    th = [threading.Thread(target=work, args=(t,)) for t in range(threads)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    dt = time.perf_counter() - t0
    n_ev, n_dg = sum(c[0] for c in counts), sum(c[1] for c in counts)
    return n_ev / dt, n_dg / dt, n_ev, n_dg, dt


def cpu_baseline(events, seconds: float, what: str):
    """The oracle on the host: one thread, then every available core (up to
    MAX_CPU_THREADS), each over about `seconds`."""
    n = cpu_threads()
    e1, d1, n1, g1, t1 = oracle_rate(events, seconds, 1)
    en, dn, nn, gn, tn = oracle_rate(events, seconds, n)
    return {"value": round(en, 2), "unit": "events/s", "cores": n, "kind": "oracle",
            "digis_per_s": round(dn, 1), "one_thread": {"value": round(e1, 2), "digis_per_s": round(d1, 1)},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{what}: {nn} events ({gn} digis) on {n} threads in {tn:.1f} s and {n1} events ({g1} digis) "
                      f"on one thread in {t1:.1f} s, cycled from the workload's {len(events)} distinct events"}


# ---------------------------------------------------------------------------
# rocprofv3 summaries
# ---------------------------------------------------------------------------
def _read_csv(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _short(name: str) -> str:
    for k in ALL_SYMBOLS:
        if f"::{k}(" in name or f"::{k}<" in name:
            return k
    return name


def summarize_profiles(prof: str, workload: str, shape, command: dict):
    """Turn rocprofv3 output of one workload at one small-kernel shape into the
    committed summaries: profiles/kernels_<workload>_<shape>.txt (kernel-trace
    statistics) and profiles/pmc_<kernel>_<workload>_<shape>.json per kernel
    (FETCH_SIZE and WRITE_SIZE per dispatch, in KiB, scaled to bytes by the same
    counters on a device copy of COPY_BYTES, whose true traffic is COPY_BYTES read and
    COPY_BYTES written)."""
    out_dir = os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)
    tag = profile_tag(workload, shape)
    stats = _read_csv(os.path.join(prof, f"kt_{tag}", "run_kernel_stats.csv"))
    lines = [f"rocprofv3 kernel-trace statistics, workload {workload} (one-stream roofline launches)",
             f"command: {command['kt']}", f"kernel source sha256[:16]: {kernel_src_sha()}", "",
             f"{'kernel':<40}{'calls':>8}{'avg_us':>10}{'min_us':>10}{'max_us':>10}{'pct':>8}"]
    for r in stats:
        lines.append(f"{_short(r['Name'])[:39]:<40}{int(r['Calls']):>8}{float(r['AverageNs']) / 1e3:>10.2f}"
                     f"{float(r['MinNs']) / 1e3:>10.2f}{float(r['MaxNs']) / 1e3:>10.2f}{float(r['Percentage']):>8.2f}")
    open(os.path.join(out_dir, f"kernels_{tag}.txt"), "w").write("\n".join(lines) + "\n")

    def per_kernel(kind):
        rows = _read_csv(os.path.join(prof, f"{kind}_{tag}", "run_counter_collection.csv"))
        acc = {}
        for r in rows:
            acc.setdefault(_short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
        return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}

    def copy_factor(kind):
        rows = _read_csv(os.path.join(prof, f"{kind}_copy", "run_counter_collection.csv"))
        vals = [float(r["Counter_Value"]) for r in rows]
        return COPY_BYTES / (sum(vals) / len(vals) * 1024.0)

    fetch, write = per_kernel("fetch"), per_kernel("write")
    ff, fw = copy_factor("fetch"), copy_factor("write")
    sha = kernel_src_sha()
    for k in ALL_SYMBOLS:
        if k not in fetch or k not in write:
            continue
        fk, nf = fetch[k]
        wk, nw = write[k]
        d = {"kernel": k, "workload": workload, "kernel_src_sha": sha,
             "fetch_kib_per_dispatch": round(fk, 1), "write_kib_per_dispatch": round(wk, 1),
             "dispatches": [nf, nw], "copy_scale_fetch": round(ff, 4), "copy_scale_write": round(fw, 4),
             "traffic_bytes_per_launch": int(fk * 1024 * ff + wk * 1024 * fw),
             "commands": {"fetch": command["fetch"], "write": command["write"],
                          "copy_fetch": command["copy_fetch"], "copy_write": command["copy_write"]}}
        json.dump(d, open(os.path.join(out_dir, f"pmc_{k}_{tag}.json"), "w"), indent=1)
    print(json.dumps({"workload": workload, "fetch_scale": ff, "write_scale": fw,
                      "kernels": {k: [fetch.get(k), write.get(k)] for k in ALL_SYMBOLS}}))


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def _gen(args):
    kind, i = args
    from paper_2004_04334_amd import synth
    return getattr(synth, f"{kind}_event")(i)


def gen_events(kind: str, count: int):
    """`count` seeded events of a configuration, drawn in parallel processes."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=min(count, cpu_threads()),
                             mp_context=multiprocessing.get_context("spawn")) as ex:
        return list(ex.map(_gen, [(kind, i) for i in range(count)]))


def tune(px, ctx, args, events, digis, slots=None, batch=None):
    """Pin the kernel shape (--kernel-config), keep the default (--no-autotune), or run
    the library's autotuner on one representative launch (every kernel shape, a few
    replays each) and keep the fastest; returns the table of mean microseconds."""
    if args.kernel_config:
        ctx.set_kernel_config(*map(int, args.kernel_config.split("x")))
        return None
    if args.no_autotune:
        return None
    own_b = batch is None
    b = batch or px.Batch(ctx, len(events))
    own_s = slots is None
    sl = slots or [px.Event(ctx, max(1, e["module"].size)) for e in events]
    times = px.autotune(ctx, b, sl[:len(events)], digis, reps=5)
    if own_s:
        for x in sl:
            x.close()
    if own_b:
        b.close()
    return {f"{wg}x{mpw}": round(t, 1) for (wg, mpw), t in sorted(times.items())}


def shuffled(evs, seed=2004):
    """The same events with their digis in a seeded random order (every event's own
    permutation): the input of the any-order form."""
    out = []
    for i, e in enumerate(evs):
        p = np.random.default_rng([seed, i]).permutation(e["module"].size)
        out.append({k: (v[p] if isinstance(v, np.ndarray) else v) for k, v in e.items()})
    return out


def _batched(px, torch, args, evs, n_copies, per_batch, workload, desc, steps, warmup, hint=False,
             timed=True, any_order=False):
    """Graph-replayed batches over `n_copies` device-resident copies of the events (a
    working set larger than the 256 MB Infinity Cache); each copy has its own batch
    object and event slots, so the host only waits when it wraps around.  Then the
    roofline launches: the same batches one after another on one stream, without a
    graph, every kernel timed with hipEvents."""
    ctx = px.Context(1856, 2000)
    # consecutive launches go to different streams, so that one batch's completion
    # (a device -> host -> device round trip) overlaps the next batch's kernels
    streams = [torch.cuda.Stream() for _ in range(N_STREAMS)]
    cap = max(e["module"].size for e in evs)
    groups = []
    for c in range(n_copies if timed else 1):
        digis = [px.Digis.from_numpy(e, "cuda", hint=hint, any_order=any_order) for e in evs]
        slots = [px.Event(ctx, cap) for _ in range(per_batch)]
        groups.append((px.Batch(ctx, per_batch), slots, digis, px.BatchInputs(slots, digis)))
    n_groups = len(groups)
    flags = [px.Flag() for _ in range(n_groups)]
    tuned = tune(px, ctx, args, evs, groups[0][2], slots=groups[0][1], batch=groups[0][0])

    def launch(i, graph, stream=None):
        b, _, _, prepared = groups[i % n_groups]
        while px.batch_query(b) == px.E_NOT_READY:     # this copy's previous launch
            time.sleep(0)
        px.acquire_batch(b, prepared, None, stream or streams[i % N_STREAMS], flag=flags[i % n_groups], graph=graph)

    def drain():
        torch.cuda.synchronize()
        for g in groups:
            while px.batch_query(g[0]) == px.E_NOT_READY:
                time.sleep(0)

    graph = not args.no_graph
    trial = None
    if timed and tuned and not args.kernel_config:
        # the autotuner times one launch alone; with launches overlapping on several
        # streams another shape can give more throughput: the three fastest alone run
        # briefly in the timed loop's form, and the best is kept
        trial = {}
        for sh in sorted(tuned, key=tuned.get)[:3]:
            ctx.set_kernel_config(*map(int, sh.split("x")))
            for i in range(n_groups):                   # captures this shape's graphs
                launch(i, graph)
            drain()
            t0 = time.perf_counter()
            for i in range(SHAPE_TRIAL_LAUNCHES):
                launch(i, graph)
            drain()
            trial[sh] = round((time.perf_counter() - t0) * 1e6 / SHAPE_TRIAL_LAUNCHES, 1)
        ctx.set_kernel_config(*map(int, min(trial, key=trial.get).split("x")))
    out = {}
    if timed:
        for i in range(max(warmup, n_groups)):          # also captures every graph
            launch(i, graph)
        drain()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        host = 0.0
        for i in range(steps):
            h0 = time.perf_counter()
            launch(i, graph)
            host += time.perf_counter() - h0
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        drain()
        n_dg = sum(e["module"].size for e in evs)
        out = {"value": per_batch * steps / wall, "ms_per_step": wall * 1e3 / steps,
               "digis_per_s": n_dg * steps / wall, "host_us_per_launch": host * 1e6 / steps}
    # roofline launches: one stream, no graph, every kernel timed
    launch(0, False, streams[0])
    drain()
    res = [px.produce(s).n_clusters for s in groups[0][1]]
    assert all(px.produce(s).status == 0 for s in groups[0][1])
    b_batch = float(sum(event_bytes(e["module"].size, k) for e, k in zip(evs, res)))
    ctx.set_timing(True, 1)
    ctx.timing(reset=True)
    for i in range(ROOFLINE_LAUNCHES):
        launch(i, False, streams[0])
    drain()
    for b, slots, _, _ in groups:
        b.close()
        for s in slots:
            s.close()
    rl = roofline(ctx, b_batch, workload)
    rl["kernel_times_from"] = f"{ROOFLINE_LAUNCHES} graph-free launches of the same batches on one stream"
    ctx.set_timing(False)
    if timed:
        out["hbm_frac_whole_job"] = round(b_batch / per_batch * out["value"] / 1e9 / HBM_PEAK_GBS, 5)
    out.update({
        "config": {"workload": desc, "n_modules": 1856, "events_per_launch": per_batch,
                   "mean_digis": int(np.mean([e["module"].size for e in evs])), "device_copies": n_groups,
                   "streams": N_STREAMS, "size_hint": bool(hint), "any_order": bool(any_order),
                   "kernel_config": list(ctx.kernel_config()),
                   "autotune_us": tuned, "shape_trial_us_per_launch": trial},
        "roofline": rl})
    ctx.close()
    return out


STRESS_DESC = ("stress: 16 events/launch of ~320k digis (16 modules at 20% occupancy with mean-40 clusters, "
               "142 sparse modules, a full-column track and a serpentine per event), 1856 modules of 160x416, "
               "persistent kernels replayed from captured graphs over 4 streams")
BATCH_DESC = ("batch: 64 events/launch (persistent kernels, captured graph), 1856 modules, 10k-120k digis/event, "
              "log-normal module occupancy")


def bench_stress(px, torch, args, evs, steps, warmup, timed=True):
    return _batched(px, torch, args, evs, 4, 16, "stress", STRESS_DESC, steps, warmup, timed=timed)


def bench_batch(px, torch, args, evs, steps, warmup, timed=True):
    r = _batched(px, torch, args, evs, 8, 64, "batch", BATCH_DESC, steps, warmup, timed=timed)
    if timed:
        h = _batched(px, torch, args, evs, 8, 64, "batch", BATCH_DESC, steps, warmup, hint=True)
        r["with_size_hint"] = {"value": round(h["value"], 2), "digis_per_s": round(h["digis_per_s"], 1),
                               "note": "every event's largest module passed as max_module_digis (host-side "
                                       "bincount outside the timed region): the scratch-mode kernel is skipped"}
        u = _batched(px, torch, args, shuffled(evs), 8, 64, "batch", BATCH_DESC, steps, warmup, any_order=True)
        r["any_order"] = {"value": round(u["value"], 2), "digis_per_s": round(u["digis_per_s"], 1),
                          "kernel_mean_us": u["roofline"]["kernel_mean_us"],
                          "note": "the same events with their digis shuffled, grouped by module on the device "
                                  "(counting sort: count, table, scatter) in the segment slot"}
    return r


def device_copies(evs) -> int:
    """Copies of the events' inputs that together exceed the last-level cache, so that
    a rotation over them reads its inputs from HBM."""
    b = sum(8 * e["module"].size for e in evs)
    return max(1, -(-int(1.25 * LLC_BYTES) // max(1, b)))


def bench_async(px, torch, args, evs, events_per_thread, hits=False, where="cuda", hint=False, shape=None,
                any_order=False, fused_hits=False, defer=False):
    """4 host threads, one event in flight each, synthetic 20 us CPU tasks while waiting;
    the rate is over the driver's own timed window (after its threads are ready)."""
    n_threads = 4
    ctx = px.Context(1856, 2000)
    reps = device_copies(evs) if where == "cuda" else 1
    pool = [px.Digis.from_numpy(e, where, hint=hint, any_order=any_order, hits=fused_hits, defer_big=defer)
            for _ in range(reps) for e in evs]
    hits = hits or fused_hits
    cap = max(e["module"].size for e in evs)
    slots = [px.Event(ctx, cap) for _ in range(n_threads)]
    streams = [torch.cuda.Stream() for _ in range(n_threads)]
    tuned = None
    if shape:
        ctx.set_kernel_config(*shape)
    else:
        tuned = tune(px, ctx, args, evs[:1], [px.Digis.from_numpy(evs[0], where, hint=hint, any_order=any_order,
                                                                   hits=fused_hits)])   # batches: no deferral
        if tuned and not args.kernel_config:
            # one event alone does not show how shapes share the GPU across the streams:
            # the three fastest shapes are run briefly in the driver itself, the best kept
            best, best_rate = None, 0.0
            for sh in sorted(tuned, key=tuned.get)[:3]:
                ctx.set_kernel_config(*map(int, sh.split("x")))
                px.run_async(ctx, slots, streams, pool, 25, cpu_task_ns=args.cpu_task_ns, hits=hits)
                st = px.run_async(ctx, slots, streams, pool, 150, cpu_task_ns=args.cpu_task_ns, hits=hits)
                rate = st["events"] / st["wall_s"]
                if rate > best_rate:
                    best, best_rate = sh, rate
            ctx.set_kernel_config(*map(int, best.split("x")))
    kept = []
    for d in pool[:len(evs)]:            # one pass for the kept-cluster counts (bytes per event)
        px.acquire(slots[0], d)
        px.wait(slots[0])
        kept.append(px.produce(slots[0]).n_clusters)
    px.run_async(ctx, slots, streams, pool, 100, cpu_task_ns=args.cpu_task_ns, hits=hits)
    torch.cuda.synchronize()
    st = px.run_async(ctx, slots, streams, pool, events_per_thread, cpu_task_ns=args.cpu_task_ns, hits=hits)
    torch.cuda.synchronize()
    # kernel times from a second run with timing events on every 8th launch of each slot
    ctx.timing(reset=True)
    ctx.set_timing(True, 8)
    px.run_async(ctx, slots, streams, pool, 400, cpu_task_ns=args.cpu_task_ns, hits=hits)
    torch.cuda.synchronize()
    ctx.set_timing(False)
    b_mean = float(np.mean([event_bytes(e["module"].size, k) for e, k in zip(evs, kept)]))
    rl = roofline(ctx, b_mean, "hits" if hits else "async")
    rl["kernel_times_from"] = "a second run of the same workload with timing events on every 8th launch"
    rate = st["events"] / st["wall_s"]
    out = {
        "value": rate, "digis_per_s": st["digis"] / st["wall_s"], "events": st["events"],
        "lat_p50_us": st["lat_p50_us"], "lat_p99_us": st["lat_p99_us"],
        "host_blocked_us_per_event": st["blocked_us_per_event"], "cpu_tasks_per_s": st["cpu_tasks_per_s"],
        "errors": st["errors"], "hbm_frac_whole_job": round(b_mean * rate / 1e9 / HBM_PEAK_GBS, 5),
        "config": {"workload": "async: 1856 modules x 160x416, ~50k digis/event, 4 host threads x 1 event "
                               "in flight, synthetic 20 us CPU tasks while waiting" +
                               (", hits fused into the clustering" if fused_hits else
                                ", hits queued behind every event" if hits else "") +
                               (", input in pinned host memory (PCIe copy per event)" if where == "pinned" else ""),
                   "mean_digis": int(np.mean([e["module"].size for e in evs])), "input": where,
                   "device_copies": reps, "size_hint": bool(hint), "kernel_config": list(ctx.kernel_config()),
                   "autotune_us": tuned},
        "roofline": rl,
    }
    for s in slots:
        s.close()
    ctx.close()
    return out


def bench_plain(px, torch, args, evs, steps, defer=False, shape=None):
    ctx = px.Context(64, 2000)
    reps = device_copies(evs)
    pool = [px.Digis.from_numpy(e, "cuda", defer_big=defer) for _ in range(reps) for e in evs]
    slot = px.Event(ctx, max(e["module"].size for e in evs))
    stream = torch.cuda.Stream()
    tuned = None
    if shape:
        ctx.set_kernel_config(*shape)
    else:
        tuned = tune(px, ctx, args, evs[:1], [px.Digis.from_numpy(evs[0], "cuda")])
    kept = []
    for d in pool[:len(evs)]:
        px.acquire(slot, d)
        px.wait(slot)
        kept.append(px.produce(slot).n_clusters)
    px.run_async(ctx, [slot], [stream], pool, 100, blocking=True)
    torch.cuda.synchronize()
    st = px.run_async(ctx, [slot], [stream], pool, steps, blocking=True)
    torch.cuda.synchronize()
    ctx.timing(reset=True)              # kernel times: a second run with timing events
    ctx.set_timing(True, 1)
    px.run_async(ctx, [slot], [stream], pool, 200, blocking=True)
    torch.cuda.synchronize()
    ctx.set_timing(False)
    b_mean = float(np.mean([event_bytes(e["module"].size, k) for e, k in zip(evs, kept)]))
    rate = st["events"] / st["wall_s"]
    out = {
        "value": rate, "digis_per_s": st["digis"] / st["wall_s"], "events": st["events"],
        "lat_p50_us": st["lat_p50_us"], "lat_p99_us": st["lat_p99_us"],
        "host_blocked_us_per_event": st["blocked_us_per_event"], "errors": st["errors"],
        "hbm_frac_whole_job": round(b_mean * rate / 1e9 / HBM_PEAK_GBS, 5),
        "config": {"workload": "plain: 64 modules x 160x416, 46,912 digis/event, one event per synchronous launch",
                   "device_copies": reps, "kernel_config": list(ctx.kernel_config()), "autotune_us": tuned},
        "roofline": roofline(ctx, b_mean, "plain"),
    }
    slot.close()
    ctx.close()
    return out


def bench_serve(px, torch, args, evs):
    """Calibration: the saturated rate (all requests arrive at once, the largest
    batches); then Poisson arrivals at SERVE_LOADS of it."""
    ctx = px.Context(1856, 2000)
    pool = [px.Digis.from_numpy(e, "cuda") for e in evs]
    arena = torch.empty(16 << 30, dtype=torch.uint8, device="cuda")
    n_slots, n_b, max_batch = SERVE_SLOTS, 8, 64
    pinned = torch.empty(n_slots * 64, dtype=torch.uint8, pin_memory=True)
    batches = [px.Batch(ctx, max_batch) for _ in range(n_b)]
    streams = [torch.cuda.Stream() for _ in range(n_b)]
    tuned = tune(px, ctx, args, evs[:16], pool[:16])      # a typical continuous batch
    # results are consumed at the callback only, so batches defer the big-module
    # kernels to a second launch that a batch gets only when one of its events needs it;
    # plain launches: a graph replay now and then holds the launching thread (the
    # dispatcher) for milliseconds, a few small kernel launches do not
    common = dict(budget_bytes=16 << 30, n_slots=n_slots, max_batch=max_batch, n_cpu_threads=16,
                  cpu_task_ns=args.cpu_task_ns, graph=False, max_inflight=SERVE_INFLIGHT, batch_delay_us=0,
                  defer_big=True)
    cal, _, _ = px.serve(ctx, arena, pinned, batches, streams, pool, rate_hz=1e9, n_requests=SERVE_REQUESTS,
                         seed=7, **common)
    sat = cal["events"] / cal["wall_s"]
    mean_b = float(np.mean([event_bytes(e["module"].size, 0) for e in evs]))

    def sweep(**kw):
        runs = []
        for load in SERVE_LOADS:
            torch.cuda.synchronize()
            st, status, ncl = px.serve(ctx, arena, pinned, batches, streams, pool, rate_hz=load * sat,
                                       n_requests=SERVE_REQUESTS, seed=11, **{**common, **kw})
            rate = st["events"] / st["wall_s"]
            runs.append({"load": load, "arrival_rate_hz": round(load * sat, 1), "value": round(rate, 2),
                         "digis_per_s": round(st["digis"] / st["wall_s"], 1),
                         "lat_p50_us": round(st["lat_p50_us"], 2), "lat_p99_us": round(st["lat_p99_us"], 2),
                         "host_blocked_us_per_event": round(st["blocked_us_per_event"], 3),
                         "cpu_tasks_per_s": round(st["cpu_tasks_per_s"], 1), "errors": st["errors"],
                         "mean_events_per_launch": round(st["events"] / max(1, st["batches"]), 2),
                         "stage_p50_us": [round(x, 1) for x in st["stage_p50_us"]],
                         "stage_p99_us": [round(x, 1) for x in st["stage_p99_us"]],
                         "cpu_tasks_per_s_idle": round(st["cpu_tasks_per_s_idle"], 1),
                         "offered_per_s": round(st["offered_per_s"], 1),
                         "kept_up": bool(rate >= 0.95 * st["offered_per_s"]),
                         "hbm_frac_whole_job": round(mean_b * rate / 1e9 / HBM_PEAK_GBS, 5)})
        return runs

    runs = sweep()
    for b in batches:
        b.close()
    shape = list(ctx.kernel_config())
    ctx.close()
    mid = runs[1]
    return {
        "value": mid["value"], "digis_per_s": mid["digis_per_s"], "lat_p50_us": mid["lat_p50_us"],
        "lat_p99_us": mid["lat_p99_us"], "host_blocked_us_per_event": mid["host_blocked_us_per_event"],
        "saturated_events_per_s": round(sat, 1), "runs": runs,
        "config": {"workload": "serve: Poisson arrivals, 10k-200k digis/event, 16 GB admission budget, "
                               "continuous batching over 8 streams with at most 6 batches on the device "
                               "(plain launches, big-module kernels deferred to a second launch when needed), "
                               "16 CPU threads with 20 us synthetic tasks",
                   "requests_per_run": SERVE_REQUESTS, "kernel_config": shape,
                   "autotune_us": tuned, "value_is": "the run at 0.7 of the saturated rate",
                   "stages": "arrival->admission, admission->launch, launch->completion callback, "
                             "callback->produce",
                   "host_cpus": cpu_threads(),
                   "placement": "dispatcher on the last core, CPU threads off the last two"},
    }


def _round(d):
    if isinstance(d, float):
        return round(d, 3)
    if isinstance(d, dict):
        return {k: _round(v) for k, v in d.items()}
    if isinstance(d, list):
        return [_round(v) for v in d]
    return d


def sub_record(r, evs, args, with_oracle=True):
    out = _round(r)
    if with_oracle and not args.no_cpu_baseline:
        e1, d1, *_ = oracle_rate(evs, args.sub_cpu_seconds, 1)
        n = cpu_threads()
        en, dn, *_ = oracle_rate(evs, args.sub_cpu_seconds, n)
        out["oracle"] = {"events_per_s_1_thread": round(e1, 2), "events_per_s_n_threads": round(en, 2),
                         "threads": n, "digis_per_s_n_threads": round(dn, 1)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400,
                    help="timed batch launches of the headline workload (400: a ~55 ms window)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=["all", "stress", "batch", "serve", "async", "plain", "hits", "fusedhits"],
                    default="all")
    ap.add_argument("--cpu-task-ns", type=int, default=20000)
    ap.add_argument("--cpu-seconds", type=float, default=8.0, help="oracle baseline of the headline, per thread count")
    ap.add_argument("--sub-cpu-seconds", type=float, default=2.0, help="oracle rates of the sub-records")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="batched workloads: plain launches, no captured graph")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default kernel shape")
    ap.add_argument("--kernel-config", metavar="WGxMPW", help="pin the small kernel's shape (no autotuning)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the one-stream roofline launches of the workload (the profiled command)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="REPS",
                    help="only run REPS device copies of 1 GiB (counter calibration) and exit")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="write profiles/ summaries of the workload from rocprofv3 output in DIR and exit")
    args = ap.parse_args()
    if args.summarize_profiles:
        if not args.kernel_config:
            sys.exit("--summarize-profiles needs the profiled shape (--kernel-config WGxMPW)")
        shape = tuple(map(int, args.kernel_config.split("x")))
        summarize_profiles(args.summarize_profiles, args.workload, shape, profile_commands(args.workload, shape))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the work is per event, and events shard across GPUs "
              "with no exchange between them", file=sys.stderr)
        sys.exit(2)

    wl = args.workload
    head = "stress" if wl == "all" else wl
    need = {"stress": ("stress", 16), "batch": ("batch", 64), "serve": ("serve", 32), "async": ("async", 32),
            "hits": ("async", 32), "fusedhits": ("async", 32), "plain": ("plain", 32)}
    kinds = [head] if wl != "all" else ["stress", "batch", "serve", "async", "plain"]
    evsets = {}
    if not args.copy_calibration:             # drawn before the GPU is touched
        print(f"bench: drawing events for {kinds}", file=sys.stderr, flush=True)
        evsets = {k: gen_events(*need[k]) for k in kinds}

    import torch
    from paper_2004_04334_amd import pxcl as px
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(torch, args.copy_calibration)
        return
    px.lib()
    if args.roofline_only:
        fn = {"stress": bench_stress, "batch": bench_batch}.get(head)
        if fn is None:
            r = bench_async(px, torch, args, evsets[head], 50, hits=(head == "hits"))
        else:
            r = fn(px, torch, args, evsets[head], 0, 0, timed=False)
        print(json.dumps(_round({"workload": head, "roofline": r["roofline"]})), flush=True)
        return
    copy_gbs = copy_bandwidth(torch)
    print(f"bench: headline {head}", file=sys.stderr, flush=True)
    if head == "stress":
        r = bench_stress(px, torch, args, evsets["stress"], args.steps, args.warmup)
    elif head == "batch":
        r = bench_batch(px, torch, args, evsets["batch"], args.steps, args.warmup)
    elif head == "serve":
        r = bench_serve(px, torch, args, evsets["serve"])
    elif head in ("async", "hits", "fusedhits"):
        r = bench_async(px, torch, args, evsets[head], args.steps, hits=(head == "hits"),
                        fused_hits=(head == "fusedhits"))
    else:
        r = bench_plain(px, torch, args, evsets["plain"], args.steps)
    if "roofline" in r:
        r["roofline"]["copy_GBps"] = copy_gbs
        r["roofline"]["frac_of_copy"] = round(r["roofline"]["achieved"] / copy_gbs, 5) if copy_gbs else None
    line = {
        "metric": METRIC, "value": round(r.pop("value"), 2), "unit": "events/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r.pop("ms_per_step", 0.0), 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u16/i32", "data": "synthetic",
    }
    line.update(_round(r))
    line["device"] = torch.cuda.get_device_name(0)
    if wl == "all":
        subs = {}
        print("bench: batch", file=sys.stderr, flush=True)
        subs["batch"] = sub_record(bench_batch(px, torch, args, evsets["batch"], SUB_STEPS["batch"], 10),
                                   evsets["batch"], args)
        print("bench: serve", file=sys.stderr, flush=True)
        subs["serve"] = sub_record(bench_serve(px, torch, args, evsets["serve"]), evsets["serve"], args)
        print("bench: async", file=sys.stderr, flush=True)
        a = bench_async(px, torch, args, evsets["async"], SUB_STEPS["async"])
        shape = tuple(a["config"]["kernel_config"])
        a["with_size_hint"] = _round({k: bench_async(px, torch, args, evsets["async"], SUB_STEPS["async"],
                                                     hint=True, shape=shape)[k]
                                      for k in ("value", "digis_per_s", "lat_p50_us", "lat_p99_us")})
        a["with_size_hint"]["note"] = ("every event's largest module passed as max_module_digis (host-side "
                                       "bincount outside the timed region): neither big-module kernel is launched")
        dfr = bench_async(px, torch, args, evsets["async"], SUB_STEPS["async"], defer=True, shape=shape)
        a["with_deferred_big_kernels"] = _round({k: dfr[k] for k in ("value", "digis_per_s", "lat_p50_us",
                                                                      "lat_p99_us", "host_blocked_us_per_event")})
        a["with_deferred_big_kernels"]["kernel_mean_us"] = dfr["roofline"]["kernel_mean_us"]
        a["with_deferred_big_kernels"]["note"] = (
            "no size hint: every event is launched without the big-module kernels, which the library queues in a "
            "second launch only when the small kernel lists a module for them (none in these events); results are "
            "final at the callback")
        hs = bench_async(px, torch, args, evsets["async"], SUB_STEPS["async"] // 4, where="pinned", shape=shape)
        a["host_staged"] = _round({k: hs[k] for k in ("value", "digis_per_s", "lat_p50_us", "lat_p99_us",
                                                      "host_blocked_us_per_event")})
        a["host_staged"]["note"] = "input in pinned host memory: a PCIe copy of 8 B/digi per event, never in value"
        fh = bench_async(px, torch, args, evsets["async"], SUB_STEPS["async"], shape=shape, fused_hits=True)
        a["with_fused_hits"] = _round({k: fh[k] for k in ("value", "digis_per_s", "lat_p50_us", "lat_p99_us")})
        a["with_fused_hits"]["kernel_mean_us"] = fh["roofline"]["kernel_mean_us"]
        a["with_fused_hits"]["note"] = ("every event asks for its hits (charge-weighted centroids), computed inside the "
                                        "clustering and compaction kernels and collected through the hits call")
        u = bench_async(px, torch, args, shuffled(evsets["async"]), SUB_STEPS["async"], shape=shape, any_order=True)
        a["any_order"] = _round({k: u[k] for k in ("value", "digis_per_s", "lat_p50_us", "lat_p99_us")})
        a["any_order"]["kernel_mean_us"] = u["roofline"]["kernel_mean_us"]
        a["any_order"]["note"] = ("the same events with their digis shuffled, grouped by module on the device "
                                  "(counting sort: count, table, scatter) in the segment slot")
        subs["async"] = sub_record(a, evsets["async"], args)
        print("bench: plain", file=sys.stderr, flush=True)
        p = bench_plain(px, torch, args, evsets["plain"], SUB_STEPS["plain"])
        pd = bench_plain(px, torch, args, evsets["plain"], SUB_STEPS["plain"], defer=True,
                         shape=tuple(p["config"]["kernel_config"]))
        p["with_deferred_big_kernels"] = _round({k: pd[k] for k in ("value", "digis_per_s", "lat_p50_us",
                                                                     "lat_p99_us")})
        p["with_deferred_big_kernels"]["note"] = ("the big-module kernels queued in a second launch only when the "
                                                  "small kernel lists a module for them (none in these events)")
        subs["plain"] = sub_record(p, evsets["plain"], args)
        line["workloads"] = subs
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(evsets[kinds[0]], args.cpu_seconds, head)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
