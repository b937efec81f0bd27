#!/usr/bin/env python3
"""Benchmark of the pixel-clustering path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload async|plain|batch|serve|stress]

Default workload ("async"): full-size events (1,856 modules of 160x416 pixels,
~50k digis each) through the non-blocking acquire/produce boundary, 4 host threads
each with one event in flight and synthetic CPU tasks filling the wait.  A step is
one event per host thread (4 events).  Inputs are resident in HBM before the timed
region starts.  One JSON line is printed; ``roofline`` describes the dominant kernel
(algorithmic bytes per launch / its mean duration, from hipEvents recorded on the
launch stream in a second run of the same workload right after the timed region, so
that the timed region carries no timing events) and ``cpu_baseline`` the plain CPU
oracle on a bounded sample of the same events.
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


def event_bytes(n_digis: int, n_kept: int) -> int:
    """Algorithmic HBM bytes of one event: read the 8 B/digi SoA, write a 4 B per-digi
    id, 12 B per kept cluster and a 4 B count."""
    return 8 * n_digis + 4 * n_digis + 12 * n_kept + 4


def kernel_src_sha() -> str:
    p = os.path.join(ROOT, "paper_2004_04334_amd", "csrc", "pxcl_kernels.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def load_traffic(workload: str, kernel: str):
    """HBM traffic per launch from the committed rocprofv3 counter summaries of the
    kernels behind a timing slot, if they were taken on the current kernel source
    (a kernel without a summary did not run in that workload)."""
    total, found = 0, False
    for sym in KERNEL_PARTS.get(kernel, [KERNEL_SYMBOLS[kernel]]):
        p = os.path.join(ROOT, "profiles", f"pmc_{sym}_{workload}.json")
        if not os.path.exists(p):
            continue
        d = json.load(open(p))
        if d.get("kernel_src_sha") != kernel_src_sha():
            return None
        total += d.get("traffic_bytes_per_launch", 0)
        found = True
    return total if found else None


def roofline(ctx, bytes_per_launch: float, workload: str):
    ms, cnt = ctx.timing(reset=True)
    avg = {k: (ms[i] / cnt[i] if cnt[i] else 0.0) for i, k in enumerate(KERNELS)}
    if not cnt[KERNELS.index("hits")]:
        del avg["hits"]
    tot = {k: ms[i] for i, k in enumerate(KERNELS)}
    dom = max(tot, key=tot.get)
    t = avg[dom] * 1e-3
    achieved = bytes_per_launch / t / 1e9 if t > 0 else 0.0
    pipe = sum(avg.values()) * 1e-3
    return {
        "bound": "hbm", "kernel": "+".join(KERNEL_PARTS.get(dom, [KERNEL_SYMBOLS[dom]])), "achieved": round(achieved, 2),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
        "traffic": load_traffic(workload, dom),
        "algorithmic_bytes_per_launch": int(bytes_per_launch),
        "kernel_mean_us": {k: round(v * 1e3, 3) for k, v in avg.items()},
        "timed_launches": int(max(cnt)),
        "pipeline_GBps": round(bytes_per_launch / pipe / 1e9, 2) if pipe > 0 else 0.0,
    }


COPY_BYTES = 1 << 30
SERVE_LOAD = 0.6           # serving: offered load as a fraction of the saturated rate
N_STREAMS = 4              # streams the batched workloads spread their launches over


def profile_commands(workload: str) -> dict:
    """The rocprofv3 commands whose output --summarize-profiles reads (run from the
    repository root with the output directory DIR)."""
    extra = "" if workload in ("async", "hits") else " --no-graph"
    steps = {"async": 100, "hits": 100, "batch": 20, "stress": 10}.get(workload, 20)
    b = f"python3 bench.py --workload {workload}{extra} --no-cpu-baseline"
    pmc = f"{b} --steps {steps} --warmup 2"
    return {
        "kt": f"rocprofv3 --kernel-trace --stats --output-format csv -d DIR/kt_{workload} -o run -- {b}",
        "fetch": f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR/fetch_{workload} -o run -- {pmc}",
        "write": f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d DIR/write_{workload} -o run -- {pmc}",
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


def cpu_baseline(events, seconds: float, unit_events: bool = True):
    """The oracle as it stands, single-threaded, over the workload's events for about
    `seconds` of CPU time."""
    import oracle
    oracle.build()
    t0 = time.perf_counter()
    n_ev = n_dg = 0
    i = 0
    while time.perf_counter() - t0 < seconds:
        ev = events[i % len(events)]
        oracle.cluster_event(ev, 2000)
        n_ev += 1
        n_dg += ev["module"].size
        i += 1
    dt = time.perf_counter() - t0
    return {"value": round(n_ev / dt, 2), "unit": "events/s", "cores": 1, "kind": "oracle",
            "digis_per_s": round(n_dg / dt, 1),
            "sample": f"{n_ev} events ({n_dg} digis) cycled from the workload's {len(events)} distinct "
                      f"events, one thread, {dt:.1f} s"}


def _read_csv(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _short(name: str) -> str:
    for k in ALL_SYMBOLS:
        if f"::{k}(" in name or f"::{k}<" in name:
            return k
    return name


def summarize_profiles(prof: str, workload: str, command: dict):
    """Turn rocprofv3 output of one workload into the committed summaries:
    profiles/kernels_<workload>.txt (kernel-trace statistics) and
    profiles/pmc_<kernel>_<workload>.json per kernel (FETCH_SIZE and WRITE_SIZE per
    dispatch, in KiB, scaled to bytes by the same counters on a device copy of
    COPY_BYTES, whose true traffic is COPY_BYTES read and COPY_BYTES written)."""
    out_dir = os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)
    stats = _read_csv(os.path.join(prof, f"kt_{workload}", "run_kernel_stats.csv"))
    lines = [f"rocprofv3 kernel-trace statistics, workload {workload}",
             f"command: {command['kt']}", "",
             f"{'kernel':<40}{'calls':>8}{'avg_us':>10}{'min_us':>10}{'max_us':>10}{'pct':>8}"]
    for r in stats:
        lines.append(f"{_short(r['Name'])[:39]:<40}{int(r['Calls']):>8}{float(r['AverageNs']) / 1e3:>10.2f}"
                     f"{float(r['MinNs']) / 1e3:>10.2f}{float(r['MaxNs']) / 1e3:>10.2f}{float(r['Percentage']):>8.2f}")
    open(os.path.join(out_dir, f"kernels_{workload}.txt"), "w").write("\n".join(lines) + "\n")

    def per_kernel(kind):
        rows = _read_csv(os.path.join(prof, f"{kind}_{workload}", "run_counter_collection.csv"))
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
        json.dump(d, open(os.path.join(out_dir, f"pmc_{k}_{workload}.json"), "w"), indent=1)
    print(json.dumps({"workload": workload, "fetch_scale": ff, "write_scale": fw,
                      "kernels": {k: [fetch.get(k), write.get(k)] for k in ALL_SYMBOLS}}))


def tune(px, ctx, args, events, digis, slots=None, batch=None):
    """Run the library's autotuner on one representative launch of the workload
    (every kernel shape, a few replays each) and keep the fastest shape; returns the
    table of mean microseconds per shape."""
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


def gen_events(maker, count, **kw):
    return [maker(i, **kw) for i in range(count)]


# ---------------------------------------------------------------------------
def bench_async(px, torch, args, synth, hits: bool = False):
    n_threads = 4
    evs = gen_events(synth.async_event, 32)
    ctx = px.Context(1856, 2000)
    pool = [px.Digis.from_numpy(e, "cuda") for e in evs]
    cap = max(e["module"].size for e in evs)
    slots = [px.Event(ctx, cap) for _ in range(n_threads)]
    streams = [torch.cuda.Stream() for _ in range(n_threads)]
    tuned = tune(px, ctx, args, evs[:1], pool[:1])
    if tuned:
        # one event alone does not show how shapes share the GPU across the streams:
        # the three fastest shapes are run briefly in the driver itself, the best kept
        best, best_rate = None, 0.0
        for shape in sorted(tuned, key=tuned.get)[:3]:
            ctx.set_kernel_config(*map(int, shape.split("x")))
            px.run_async(ctx, slots, streams, pool, 25, cpu_task_ns=args.cpu_task_ns, hits=hits)
            st = px.run_async(ctx, slots, streams, pool, 150, cpu_task_ns=args.cpu_task_ns, hits=hits)
            rate = st["events"] / st["wall_s"]
            if rate > best_rate:
                best, best_rate = shape, rate
        ctx.set_kernel_config(*map(int, best.split("x")))
    kept = []
    for d in pool:                       # one pass for the kept-cluster counts (bytes per event)
        px.acquire(slots[0], d)
        px.wait(slots[0])
        kept.append(px.produce(slots[0]).n_clusters)
    px.run_async(ctx, slots, streams, pool, max(1, args.warmup), cpu_task_ns=args.cpu_task_ns, hits=hits)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = px.run_async(ctx, slots, streams, pool, args.steps, cpu_task_ns=args.cpu_task_ns, hits=hits)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # kernel times from a second run of the same workload with timing events (so that
    # the throughput above carries no timing overhead)
    ctx.timing(reset=True)
    ctx.set_timing(True, args.timing_period)
    px.run_async(ctx, slots, streams, pool, max(200, args.steps // 2), cpu_task_ns=args.cpu_task_ns, hits=hits)
    torch.cuda.synchronize()
    ctx.set_timing(False)
    n_ev = st["events"]
    b_mean = float(np.mean([event_bytes(e["module"].size, k) for e, k in zip(evs, kept)]))
    rl = roofline(ctx, b_mean, "hits" if hits else "async")
    rl["kernel_times_from"] = "a second run of the same workload with timing events"
    if hits and rl["kernel_mean_us"].get("hits"):
        # hits kernel: reads row, col, adc and the per-digi id (10 B/digi), the kept ids
        # and charges (8 B/cluster), writes x and y (8 B/cluster)
        hb = float(np.mean([10 * e["module"].size + 16 * k for e, k in zip(evs, kept)]))
        gbs = hb / (rl["kernel_mean_us"]["hits"] * 1e-6) / 1e9
        rl["hits_kernel"] = {"algorithmic_bytes_per_launch": int(hb), "achieved": round(gbs, 2),
                             "frac": round(gbs / HBM_PEAK_GBS, 5)}
    out = {
        "value": n_ev / wall, "ms_per_step": wall * 1e3 / args.steps,
        "digis_per_s": st["digis"] / wall,
        "lat_p50_us": st["lat_p50_us"], "lat_p99_us": st["lat_p99_us"],
        "host_blocked_us_per_event": st["blocked_us_per_event"],
        "cpu_tasks_per_s": st["cpu_tasks_per_s"], "errors": st["errors"],
        "config": {"workload": "async: 1856 modules x 160x416, ~50k digis/event, 4 host threads x 1 event "
                               "in flight, synthetic CPU tasks while waiting" +
                               (", hits queued behind every event" if hits else ""),
                   "n_modules": 1856, "mean_digis": int(np.mean([e["module"].size for e in evs])),
                   "host_threads": n_threads, "cpu_task_ns": args.cpu_task_ns, "distinct_events": len(evs),
                   "kernel_config": list(ctx.kernel_config()), "autotune_us": tuned},
        "roofline": rl, "events": evs,
    }
    for s in slots:
        s.close()
    ctx.close()
    return out


def bench_hits(px, torch, args, synth):
    """The asynchronous workload with every event's hits queued behind it on the
    same stream (a consumer of the clusters) and produced with it."""
    return bench_async(px, torch, args, synth, hits=True)


def bench_plain(px, torch, args, synth):
    evs = gen_events(synth.plain_event, 32)
    ctx = px.Context(64, 2000)
    pool = [px.Digis.from_numpy(e, "cuda") for e in evs]
    slot = px.Event(ctx, max(e["module"].size for e in evs))
    stream = torch.cuda.Stream()
    tuned = tune(px, ctx, args, evs[:1], pool[:1])
    kept = []
    for d in pool:
        px.acquire(slot, d)
        px.wait(slot)
        kept.append(px.produce(slot).n_clusters)
    px.run_async(ctx, [slot], [stream], pool, max(1, args.warmup), blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = px.run_async(ctx, [slot], [stream], pool, args.steps, blocking=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.timing(reset=True)              # kernel times: a second run with timing events
    ctx.set_timing(True, args.timing_period)
    px.run_async(ctx, [slot], [stream], pool, max(200, args.steps // 2), blocking=True)
    torch.cuda.synchronize()
    ctx.set_timing(False)
    b_mean = float(np.mean([event_bytes(e["module"].size, k) for e, k in zip(evs, kept)]))
    out = {
        "value": st["events"] / wall, "ms_per_step": wall * 1e3 / args.steps, "digis_per_s": st["digis"] / wall,
        "lat_p50_us": st["lat_p50_us"], "lat_p99_us": st["lat_p99_us"],
        "host_blocked_us_per_event": st["blocked_us_per_event"], "errors": st["errors"],
        "config": {"workload": "plain: 64 modules x 160x416, 46,912 digis/event, one event per synchronous launch",
                   "n_modules": 64, "mean_digis": 46912, "distinct_events": len(evs),
                   "kernel_config": list(ctx.kernel_config()), "autotune_us": tuned},
        "roofline": roofline(ctx, b_mean, "plain"), "events": evs,
    }
    slot.close()
    ctx.close()
    return out


def _batched(px, torch, args, evs, n_copies, per_batch, workload, desc, n_modules=1856):
    """Graph-replayed batches over `n_copies` device-resident copies of the events (a
    working set larger than the 256 MB Infinity Cache); each copy has its own batch
    object and event slots, so the host only waits when it wraps around."""
    ctx = px.Context(n_modules, 2000)
    # consecutive launches go to different streams, so that one batch's completion
    # callback (a device -> host -> device round trip on its stream) overlaps the next
    # batch's kernels
    streams = [torch.cuda.Stream() for _ in range(N_STREAMS)]
    cap = max(e["module"].size for e in evs)
    groups = []
    for c in range(n_copies):
        digis = [px.Digis.from_numpy(e, "cuda") for e in evs]
        slots = [px.Event(ctx, cap) for _ in range(per_batch)]
        groups.append((px.Batch(ctx, per_batch), slots, digis, px.BatchInputs(slots, digis)))
    flags = [px.Flag() for _ in range(n_copies)]
    tuned = tune(px, ctx, args, evs, groups[0][2], slots=groups[0][1], batch=groups[0][0])

    def launch(i, graph, stream=None):
        b, _, _, prepared = groups[i % n_copies]
        while px.batch_query(b) == px.E_NOT_READY:     # this copy's previous launch
            time.sleep(0)
        px.acquire_batch(b, prepared, None, stream or streams[i % N_STREAMS], flag=flags[i % n_copies], graph=graph)

    def drain():
        torch.cuda.synchronize()
        for g in groups:
            while px.batch_query(g[0]) == px.E_NOT_READY:
                time.sleep(0)

    graph = not args.no_graph
    for i in range(max(args.warmup, n_copies)):          # also captures every graph
        launch(i, graph)
    drain()
    res = [px.produce(s).n_clusters for s in groups[0][1]]
    b_batch = float(sum(event_bytes(e["module"].size, k) for e, k in zip(evs, res)))
    if not graph:
        ctx.set_timing(True, args.timing_period)
    ctx.timing(reset=True)
    t0 = time.perf_counter()
    host = 0.0
    for i in range(args.steps):
        h0 = time.perf_counter()
        launch(i, graph)
        host += time.perf_counter() - h0
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    drain()
    if graph:
        # hipEvents recorded inside a captured graph cannot be timed: the kernel times
        # come from the same batches launched without a graph
        # (on one stream, so that concurrent batches do not stretch each other's kernels)
        ctx.set_timing(True)
        for i in range(min(args.steps, 8 * n_copies)):
            launch(i, False, streams[0])
        drain()
    for b, slots, _, _ in groups:
        b.close()
        for s in slots:
            s.close()
    rl = roofline(ctx, b_batch, workload)
    rl["kernel_times_from"] = "graph-free launches of the same batches" if graph else "the timed launches"
    ctx.set_timing(False)
    n_dg = sum(e["module"].size for e in evs)
    out = {
        "value": per_batch * args.steps / wall, "ms_per_step": wall * 1e3 / args.steps,
        "digis_per_s": n_dg * args.steps / wall,
        "host_us_per_launch": host * 1e6 / args.steps,
        "config": {"workload": desc, "n_modules": n_modules, "events_per_launch": per_batch,
                   "mean_digis": int(n_dg / len(evs)), "device_copies": n_copies, "streams": N_STREAMS,
                   "kernel_config": list(ctx.kernel_config()), "autotune_us": tuned},
        "roofline": rl, "events": evs,
    }
    ctx.close()
    return out


def bench_batch(px, torch, args, synth):
    evs = gen_events(synth.batch_event, 64)
    return _batched(px, torch, args, evs, 8, 64, "batch",
                    "batch: 64 events/launch (persistent kernels, captured graph), 1856 modules, "
                    "10k-120k digis/event, log-normal module occupancy")


def bench_stress(px, torch, args, synth):
    evs = gen_events(synth.stress_event, 16)
    return _batched(px, torch, args, evs, 4, 16, "stress",
                    "stress: 16 events/launch of ~320k digis, 16 modules at 20% occupancy with "
                    "mean-40 clusters, a full-column track and a serpentine per event")


def bench_serve(px, torch, args, synth):
    evs = gen_events(synth.serve_event, 32)
    ctx = px.Context(1856, 2000)
    pool = [px.Digis.from_numpy(e, "cuda") for e in evs]
    arena = torch.empty(16 << 30, dtype=torch.uint8, device="cuda")
    n_slots, n_b, max_batch = 512, 8, 64
    pinned = torch.empty(n_slots * 64, dtype=torch.uint8, pin_memory=True)
    batches = [px.Batch(ctx, max_batch) for _ in range(n_b)]
    streams = [torch.cuda.Stream() for _ in range(n_b)]
    tuned = tune(px, ctx, args, evs[:16], pool[:16])      # a typical continuous batch
    common = dict(budget_bytes=16 << 30, n_slots=n_slots, max_batch=max_batch, n_cpu_threads=16,
                  cpu_task_ns=args.cpu_task_ns, graph=True)
    # calibration: saturated throughput (all requests arrive at once, the largest
    # batches); Poisson arrivals form smaller batches, so the offered load is 0.6 of it
    cal, _, _ = px.serve(ctx, arena, pinned, batches, streams, pool, rate_hz=1e9, n_requests=10000, seed=7, **common)
    sat = cal["events"] / cal["wall_s"]
    rate = SERVE_LOAD * sat
    torch.cuda.synchronize()
    st, status, ncl = px.serve(ctx, arena, pinned, batches, streams, pool, rate_hz=rate,
                               n_requests=args.steps, seed=11, **common)
    torch.cuda.synchronize()
    # kernel times: hipEvents cannot be timed inside captured graphs, so a shorter run
    # of the same request stream launches its batches without a graph
    n_t = min(args.steps, 2000)
    ctx.timing(reset=True)
    ctx.set_timing(True)
    st_t, _, ncl_t = px.serve(ctx, arena, pinned, batches, streams, pool, rate_hz=rate, n_requests=n_t,
                              seed=11, **dict(common, graph=False))
    torch.cuda.synchronize()
    for b in batches:
        b.close()
    b_mean = float(np.mean([event_bytes(evs[r % len(evs)]["module"].size, ncl_t[r]) for r in range(n_t)]))
    rl = roofline(ctx, b_mean * n_t / max(1, st_t["batches"]), "serve")
    rl["kernel_times_from"] = f"graph-free launches of the first {n_t} requests"
    ctx.set_timing(False)
    n_batches = max(1, st["batches"])
    out = {
        "value": st["events"] / st["wall_s"], "ms_per_step": st["wall_s"] * 1e3 / args.steps,
        "digis_per_s": st["digis"] / st["wall_s"],
        "lat_p50_us": st["lat_p50_us"], "lat_p99_us": st["lat_p99_us"],
        "host_blocked_us_per_event": st["blocked_us_per_event"], "cpu_tasks_per_s": st["cpu_tasks_per_s"],
        "errors": st["errors"], "saturated_events_per_s": sat, "arrival_rate_hz": rate,
        "config": {"workload": f"serve: Poisson arrivals at {SERVE_LOAD}x saturated rate, 10k-200k digis/event, "
                               "16 GB admission budget, continuous batching over 8 streams, 16 CPU threads",
                   "n_modules": 1856, "mean_digis": int(np.mean([e["module"].size for e in evs])),
                   "requests": args.steps, "mean_events_per_launch": round(args.steps / n_batches, 2),
                   "kernel_config": list(ctx.kernel_config()), "autotune_us": tuned,
                   "peak_resident_bytes": st["peak_resident_bytes"]},
        "roofline": rl, "events": evs,
    }
    ctx.close()
    return out


WORKLOADS = {"async": (bench_async, 2000, 100), "hits": (bench_hits, 2000, 100), "plain": (bench_plain, 2000, 100),
             "batch": (bench_batch, 200, 10), "stress": (bench_stress, 100, 5),
             "serve": (bench_serve, 20000, 0)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="async")
    ap.add_argument("--cpu-task-ns", type=int, default=20000)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="batched workloads: plain launches, no captured graph")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default kernel shape instead of tuning it on the workload first")
    ap.add_argument("--timing-period", type=int, default=8,
                    help="time the kernels of every N-th launch of each event object in the timed region")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="REPS",
                    help="only run REPS device copies of 1 GiB (counter calibration) and exit")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="write profiles/ summaries of the workload from rocprofv3 output in DIR and exit")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles, args.workload, profile_commands(args.workload))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs on a single MI355X "
              "(events shard across GPUs with no exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)
    fn, d_steps, d_warm = WORKLOADS[args.workload]
    args.steps = args.steps or d_steps
    args.warmup = d_warm if args.warmup is None else args.warmup

    import torch
    from paper_2004_04334_amd import pxcl as px
    from paper_2004_04334_amd import synth
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(torch, args.copy_calibration)
        return
    px.lib()
    copy_gbs = copy_bandwidth(torch)
    r = fn(px, torch, args, synth)
    r["roofline"]["copy_GBps"] = copy_gbs
    r["roofline"]["frac_of_copy"] = round(r["roofline"]["achieved"] / copy_gbs, 5) if copy_gbs else None
    evs = r.pop("events")
    line = {
        "metric": "events/s + digis/s clustered (frac HBM peak); p50/p99 event latency; host block time",
        "value": round(r.pop("value"), 2), "unit": "events/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(r.pop("ms_per_step"), 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u16/i32", "data": "synthetic",
    }
    line.update({k: (round(v, 3) if isinstance(v, float) else v) for k, v in r.items()})
    line["device"] = torch.cuda.get_device_name(0)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(evs, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
