"""Boundary semantics and the systems forms on the device: non-blocking acquire,
exactly-once callbacks, synchronous error codes, batches and captured graphs, the
asynchronous driver, serving with continuous batching, the autotuner.  Every result
is checked bit-exactly against the oracle, alone / in a batch / in the serving mix."""
from __future__ import annotations

import json
import threading
import time

import numpy as np
import pytest

import oracle
from paper_2004_04334_amd import synth
from tests.gpu_util import compare, run_events

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def px():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_04334_amd import pxcl
    pxcl.lib()
    oracle.build()
    return pxcl


@pytest.fixture(scope="module")
def batch_events():
    return [synth.batch_event(i) for i in range(8)]


def test_acquire_returns_before_completion(px):
    import torch
    ev = synth.stress_event(2)
    ctx = px.Context(1856)
    slot = px.Event(ctx, ev["module"].size)
    d = px.Digis.from_numpy(ev, "cuda")
    s = torch.cuda.Stream()
    calls = []
    done = threading.Event()

    def cb(status):
        calls.append(status)
        done.set()

    with torch.cuda.stream(s):
        torch.cuda._sleep(200_000_000)          # keep the stream busy (~0.1 s)
    t0 = time.perf_counter()
    px.acquire(slot, d, s, done_cb=cb)
    t_acq = time.perf_counter() - t0
    assert px.query(slot) == px.E_NOT_READY
    with pytest.raises(px.PxclError) as ei:
        px.produce(slot)
    assert ei.value.code == px.E_NOT_READY
    with pytest.raises(px.PxclError) as ei:      # one event in flight per slot
        px.acquire(slot, d, s)
    assert ei.value.code == px.E_BUSY
    assert done.wait(30)
    px.wait(slot)
    time.sleep(0.05)
    assert calls == [0], "done_cb fires exactly once, with the status"
    assert t_acq < 0.02, f"acquire blocked for {t_acq * 1e3:.2f} ms"
    compare(px.produce(slot).numpy(), oracle.cluster_event(ev, 2000), "stress after sleep")
    slot.close()
    ctx.close()


def test_callback_may_acquire_again_not_destroy(px):
    """Completion callbacks run on the context's completion thread: one may produce and
    acquire the event again (that launch completes normally) but may not destroy the
    context (E_BUSY, the context stays usable)."""
    ev = synth.plain_event(5)
    ref = oracle.cluster_event(ev, 2000)
    ctx = px.Context(ev["n_modules"], 2000)
    slot = px.Event(ctx, ev["module"].size)
    d = px.Digis.from_numpy(ev, "cuda")
    seen = {}
    again = px.Flag()

    def cb(st):
        seen["status"] = st
        try:
            ctx.close()
        except px.PxclError as e:
            seen["close"] = e.code
        seen["n"] = px.produce(slot).n_clusters
        px.acquire(slot, d, flag=again)

    px.acquire(slot, d, done_cb=cb)
    t0 = time.time()
    while again.fired == 0:
        assert time.time() - t0 < 30, "the second launch did not complete"
        time.sleep(0.001)
    px.wait(slot)
    assert seen == {"status": 0, "close": px.E_BUSY, "n": ref["n_clusters"]}
    compare(px.produce(slot).numpy(), ref, "acquired in the callback")
    slot.close()
    ctx.close()


def test_synchronous_errors(px):
    ctx = px.Context(64)
    slot = px.Event(ctx, 100)
    ev = synth.plain_event(0)
    d = px.Digis.from_numpy(ev, "cuda")
    with pytest.raises(px.PxclError) as ei:
        px.acquire(slot, d)
    assert ei.value.code == px.E_CAPACITY
    with pytest.raises(px.PxclError) as ei:
        px.produce(slot)                       # never acquired
    assert ei.value.code == px.E_INVAL
    with pytest.raises(px.PxclError) as ei:
        ctx.close()                            # a slot is still bound
    assert ei.value.code == px.E_BUSY
    slot.close()
    ctx.close()


def test_two_streams_overlap(px):
    import torch
    evs = [synth.async_event(20), synth.async_event(21)]
    ctx = px.Context(1856)
    slots = [px.Event(ctx, e["module"].size) for e in evs]
    ds = [px.Digis.from_numpy(e, "cuda") for e in evs]
    ss = [torch.cuda.Stream(), torch.cuda.Stream()]
    flags = [px.Flag(), px.Flag()]
    for sl, d, s, f in zip(slots, ds, ss, flags):
        px.acquire(sl, d, s, flag=f)
    for sl in slots:
        px.wait(sl)
    for i, (sl, e) in enumerate(zip(slots, evs)):
        compare(px.produce(sl).numpy(), oracle.cluster_event(e, 2000), f"stream {i}")
        sl.close()
    ctx.close()


def test_batch_identity_alone_batch_graph(px, batch_events):
    import torch
    ctx = px.Context(1856)
    alone = run_events(px, ctx, batch_events)
    refs = [oracle.cluster_event(e, 2000) for e in batch_events]
    for i, (a, r) in enumerate(zip(alone, refs)):
        compare(a, r, f"alone {i}")
    b = px.Batch(ctx, 16)
    slots = [px.Event(ctx, max(e["module"].size for e in batch_events)) for _ in range(8)]
    res = run_events(px, ctx, batch_events, batch=b, slots=slots)
    for i, (x, a) in enumerate(zip(res, alone)):
        compare(x, a, f"batch vs alone {i}")
    # graph replays: different subsets and orders, eager work in between
    for rep, order in enumerate([[0, 1, 2, 3, 4, 5, 6, 7], [7, 2, 5], [3], [6, 5, 4, 3, 2, 1, 0, 7]]):
        sub = [batch_events[j] for j in order]
        res = run_events(px, ctx, sub, batch=b, graph=True, slots=[slots[j] for j in range(len(order))])
        torch.ones(1000, device="cuda").sum().item()
        for j, x in zip(order, res):
            compare(x, alone[j], f"graph replay {rep} event {j}")
    for s in slots:
        s.close()
    b.close()
    ctx.close()


def test_graph_per_flag_combination(px):
    """One batch object replayed with launches whose flags alternate (size hints that
    skip the big-module kernels, none, a bound that skips only the scratch kernel, and
    a module above 16,384 digis): each combination has a captured graph of its own, and
    every replay matches the oracle."""
    import torch
    lin = (np.arange(20000) * 37) % (160 * 416)
    huge = synth.from_pixels(np.concatenate([np.zeros(50, np.int64), np.full(20000, 2)]),
                             np.concatenate([np.arange(50) * 3 % 160, lin % 160]),
                             np.concatenate([np.arange(50) * 7 % 416, lin // 160]), n_modules=1856, seed=6)
    small = [synth.batch_event(70 + i) for i in range(3)]      # largest module 3,328 digis
    plains = [synth.plain_event(80 + i) for i in range(3)]     # 733 digis per module
    # flags: NO_SCRATCH; none; NO_BIG | NO_SCRATCH; none (a module of 20,000 digis); ...
    cases = [(small, True), (small, False), (plains, True), (small + [huge], True), (plains, True),
             (small, True), (small + [huge], False), (small, False)]
    refs = {id(e): oracle.cluster_event(e, 2000) for e in small + plains + [huge]}
    ctx = px.Context(1856, 2000)
    ctx.set_kernel_config(256, 1)
    b = px.Batch(ctx, 4)
    cap = max(e["module"].size for e in small + plains + [huge])
    slots = [px.Event(ctx, cap) for _ in range(4)]
    for rep, (evs, hint) in enumerate(cases):
        print(f"graph flags case {rep}", flush=True)
        digis = [px.Digis.from_numpy(e, "cuda", hint=hint) for e in evs]
        px.acquire_batch(b, slots[:len(evs)], digis, graph=True)
        for s in slots[:len(evs)]:
            px.wait(s)
        torch.ones(1000, device="cuda").sum().item()
        for i, (s, e) in enumerate(zip(slots, evs)):
            compare(px.produce(s).numpy(), refs[id(e)], f"case {rep} event {i}")
    for s in slots:
        s.close()
    b.close()
    ctx.close()


def test_full_batch_of_64(px):
    """Batching configuration at full size: 64 events, one captured-graph launch."""
    evs = [synth.batch_event(100 + i) for i in range(64)]
    ctx = px.Context(1856)
    b = px.Batch(ctx, 64)
    res = run_events(px, ctx, evs, batch=b, graph=True)
    for i, (r, e) in enumerate(zip(res, evs)):
        compare(r, oracle.cluster_event(e, 2000), f"batch64 ev {i}")
    b.close()
    ctx.close()


def test_full_stress_batch_of_16(px):
    """Stress configuration at full size: 16 events of ~320k digis in one launch."""
    evs = [synth.stress_event(i) for i in range(16)]
    ctx = px.Context(1856)
    b = px.Batch(ctx, 16)
    res = run_events(px, ctx, evs, batch=b, graph=True)
    for i, (r, e) in enumerate(zip(res, evs)):
        compare(r, oracle.cluster_event(e, 2000), f"stress ev {i}")
    b.close()
    ctx.close()


def test_async_driver(px):
    import torch
    pool_np = [synth.async_event(30 + i) for i in range(6)]
    ctx = px.Context(1856)
    pool = [px.Digis.from_numpy(e, "cuda") for e in pool_np]
    slots = [px.Event(ctx, 60000) for _ in range(4)]
    streams = [torch.cuda.Stream() for _ in range(4)]
    st = px.run_async(ctx, slots, streams, pool, events_per_thread=25, cpu_task_ns=20000)
    assert st["events"] == 100 and st["errors"] == 0
    assert st["cpu_tasks"] > 0
    assert st["blocked_us_per_event"] < st["lat_p50_us"]
    # every event of a run, copied out as it is produced (verification mode)
    refs = [oracle.cluster_event(e, 2000) for e in pool_np]
    sizes = [pool_np[r % len(pool_np)]["module"].size for r in range(100)]
    offs = np.concatenate([[0], np.cumsum([16 * n for n in sizes])]).astype(np.int64)
    results = torch.full((int(offs[-1]),), 0xFF, dtype=torch.uint8, device="cuda")
    ver = px.run_async(ctx, slots, streams, pool, events_per_thread=25, cpu_task_ns=20000, results=results,
                       result_offsets=offs[:-1].tolist())
    assert ver["events"] == 100 and ver["errors"] == 0
    host = results.cpu().numpy()
    for r in range(100):
        ref, n = refs[r % len(pool_np)], sizes[r]
        k = ref["n_clusters"]
        blob = host[offs[r]: offs[r] + 16 * n].view(np.int32)
        got = {"status": 0, "n_clusters": k, "digi": blob[:n], "id": blob[n:n + k],
               "charge": blob[2 * n:2 * n + k], "size": blob[3 * n:3 * n + k]}
        compare(got, ref, f"async event {r} (thread {r % 4})")
    blk = px.run_async(ctx, slots, streams, pool, events_per_thread=10, blocking=True)
    assert blk["errors"] == 0 and blk["cpu_tasks"] == 0
    # each thread's last event is still readable and exact
    for t, sl in enumerate(slots):
        idx = (t + 9 * 4) % len(pool_np)
        compare(px.produce(sl).numpy(), oracle.cluster_event(pool_np[idx], 2000), f"thread {t}")
    for s in slots:
        s.close()
    ctx.close()


def test_serving_mix_identical_to_alone(px):
    import torch
    pool_np = [synth.serve_event(i) for i in range(12)]
    # half the pool in any order (grouped on the device), mixed into the same batches
    for i in range(0, 12, 2):
        p = np.random.default_rng(40 + i).permutation(pool_np[i]["module"].size)
        pool_np[i] = {k: (v[p] if isinstance(v, np.ndarray) else v) for k, v in pool_np[i].items()}
    refs = [oracle.cluster_event(e, 2000, any_order=(i % 2 == 0)) for i, e in enumerate(pool_np)]
    ctx = px.Context(1856)
    pool = [px.Digis.from_numpy(e, "cuda", any_order=(i % 2 == 0)) for i, e in enumerate(pool_np)]
    n_req = 240
    budget = 64 << 20                                 # small, so that admission binds
    arena = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    pinned = torch.empty(32 * 64, dtype=torch.uint8, pin_memory=True)
    batches = [px.Batch(ctx, 16) for _ in range(3)]
    streams = [torch.cuda.Stream() for _ in range(3)]
    sizes = [pool_np[r % len(pool_np)]["module"].size for r in range(n_req)]
    offs = np.concatenate([[0], np.cumsum([16 * n for n in sizes])]).astype(np.int64)
    results = torch.empty(int(offs[-1]), dtype=torch.uint8, device="cuda")
    st, status, ncl = px.serve(ctx, arena, pinned, batches, streams, pool, rate_hz=20000.0, n_requests=n_req,
                               budget_bytes=budget, n_slots=32, max_batch=16, n_cpu_threads=4,
                               cpu_task_ns=10000, graph=True, seed=3, results=results,
                               result_offsets=offs[:-1].tolist(), max_inflight=2)
    assert st["errors"] == 0 and st["events"] == n_req
    assert st["peak_resident_bytes"] <= budget
    assert st["max_inflight"] > 1, "requests overlap on the device"
    host = results.cpu().numpy()
    for r in range(n_req):
        ref = refs[r % len(pool_np)]
        n, k = sizes[r], int(ncl[r])
        assert status[r] == 0 and k == ref["n_clusters"]
        blob = host[offs[r]: offs[r] + 16 * n].view(np.int32)
        got = {"status": 0, "n_clusters": k, "digi": blob[:n], "id": blob[n:n + k],
               "charge": blob[2 * n:2 * n + k], "size": blob[3 * n:3 * n + k]}
        compare(got, ref, f"served request {r}")
    for b in batches:
        b.close()
    ctx.close()


def test_autotune_and_cache(px, batch_events, tmp_path):
    ctx = px.Context(1856)
    b = px.Batch(ctx, 8)
    slots = [px.Event(ctx, max(e["module"].size for e in batch_events)) for _ in batch_events]
    digis = [px.Digis.from_numpy(e, "cuda") for e in batch_events]
    path = str(tmp_path / "tune.json")
    times = px.autotune(ctx, b, slots, digis, reps=2, cache_path=path)
    assert len(times) == 9 and all(t > 0 for t in times.values())
    best = min(times, key=times.get)
    assert ctx.kernel_config() == best
    data = json.load(open(path))
    assert list(data.values()) == [list(best)]
    ctx.set_kernel_config(64, 1)
    mean = int(np.mean([e["module"].size for e in batch_events]))
    assert px.autotune_load(ctx, path, mean)
    assert ctx.kernel_config() == best
    res = run_events(px, ctx, batch_events, batch=b, slots=slots)
    for i, (r, e) in enumerate(zip(res, batch_events)):
        compare(r, oracle.cluster_event(e, 2000), f"tuned {i}")
    for s in slots:
        s.close()
    b.close()
    ctx.close()


def _mutated(ev, **kw):
    out = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in ev.items()}
    for k, (i, val) in kw.items():
        out[k][i] = val
    return out


@pytest.mark.parametrize("graph", [False, True])
def test_batch_error_isolation(px, batch_events, graph):
    """Errors travel with their own event: a batch holding one event with a pixel out
    of range, one whose module ids decrease and one with a pixel fired twice, between
    valid events.  Each bad event reports the oracle's status; every other event of the
    batch is bit-exact; the batch callback reports the first event error."""
    import torch
    good = batch_events[:3]
    n0 = batch_events[3]["module"].size
    bad_range = _mutated(batch_events[3], row=(n0 // 2, 160))
    n1 = batch_events[4]["module"].size
    bad_order = _mutated(batch_events[4], module=(0, int(batch_events[4]["module"][-1])))
    e5 = batch_events[5]
    bad_dup = _mutated(e5, row=(1, int(e5["row"][0])), col=(1, int(e5["col"][0])), module=(1, int(e5["module"][0])))
    evs = [good[0], bad_range, good[1], bad_order, bad_dup, good[2]]
    refs = [oracle.cluster_event(e, 2000) for e in evs]
    assert [r["status"] for r in refs] == [0, px.E_RANGE, 0, px.E_ORDER, px.E_DUP_PIXEL, 0], \
        [r["status"] for r in refs]
    ctx = px.Context(1856)
    b = px.Batch(ctx, 8)
    slots = [px.Event(ctx, max(e["module"].size for e in evs)) for _ in evs]
    for rep in range(2):                                 # a second launch of the same slots
        print(f"error isolation graph={graph} rep {rep}", flush=True)
        f = px.Flag()
        digis = [px.Digis.from_numpy(e, "cuda", hint=False) for e in evs]
        px.acquire_batch(b, slots, digis, flag=f, graph=graph)
        for s in slots:
            px.wait(s)
        t0 = time.time()
        while f.fired == 0:
            assert time.time() - t0 < 30
        assert f.status == px.E_RANGE, "the batch reports the first event error"
        for i, (s, r) in enumerate(zip(slots, refs)):
            compare(px.produce(s).numpy(), r, f"graph={graph} rep {rep} event {i}")
        torch.ones(1000, device="cuda").sum().item()
    # the same slots with valid events afterwards
    res = run_events(px, ctx, batch_events[:6], batch=b, graph=graph, slots=slots)
    for i, (r, e) in enumerate(zip(res, batch_events[:6])):
        compare(r, oracle.cluster_event(e, 2000), f"after errors, event {i}")
    for s in slots:
        s.close()
    b.close()
    ctx.close()
