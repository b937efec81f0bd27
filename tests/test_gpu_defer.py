"""Deferred big-module kernels (PXCL_DIGIS_DEFER_BIG) on the device: one-event
launches without the big-module kernels, finished by a second launch that the
completion thread queues only when the small kernel listed modules for them;
bit-exact against the oracle for events with and without such modules (register and
scratch mode), in any order, with fused hits, alternating with ordinary launches and
errors on one slot, through the asynchronous driver; and the calls that must wait for
the callback."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2004_04334_amd import synth
from tests.gpu_util import compare

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


def _shuffled(ev, seed):
    p = np.random.default_rng(seed).permutation(ev["module"].size)
    return {k: (v[p] if isinstance(v, np.ndarray) else v) for k, v in ev.items()}


def _run(px, ctx, ev, slot=None, **kw):
    import torch
    own = slot is None
    slot = slot or px.Event(ctx, max(1, ev["module"].size))
    d = px.Digis.from_numpy(ev, "cuda", **kw)
    f = px.Flag()
    px.acquire(slot, d, torch.cuda.current_stream(), flag=f)
    px.wait(slot)
    assert f.fired == 1
    r = px.produce(slot).numpy()
    if own:
        slot.close()
    return r


@pytest.mark.parametrize("wg,mpw", [(64, 1), (512, 1)])
def test_deferred_single_events(px, wg, mpw):
    print(f"deferred big-module kernels, shape {wg}x{mpw}", flush=True)
    ctx = px.Context(1856, 2000, 0)
    ctx.set_kernel_config(wg, mpw)
    evs = [synth.async_event(3), dict(synth.plain_event(5), n_modules=1856), synth.stress_event(0),
           synth.stress_event(1)]
    for i, e in enumerate(evs):
        compare(_run(px, ctx, e, defer_big=True), oracle.cluster_event(e, 2000), f"event {i}")
        sh = _shuffled(e, 30 + i)
        compare(_run(px, ctx, sh, defer_big=True, any_order=True), oracle.cluster_event(sh, 2000, any_order=True),
                f"event {i}, any order")
    ctx.close()


def test_deferred_fused_hits(px):
    import torch
    ctx = px.Context(1856, 2000, 0)
    for i, e in enumerate([synth.async_event(4), synth.stress_event(2)]):
        slot = px.Event(ctx, e["module"].size)
        d = px.Digis.from_numpy(e, "cuda", defer_big=True, hits=True)
        px.acquire(slot, d, torch.cuda.current_stream())
        px.wait(slot)
        px.hits_enqueue(slot, torch.cuda.current_stream())
        px.hits_wait(slot)
        ref = oracle.hits(e, 2000)
        compare(px.produce(slot).numpy(), ref, f"event {i}")
        h = px.hits_produce(slot).numpy()
        assert np.array_equal(h["x"], ref["x"]) and np.array_equal(h["y"], ref["y"]), f"hits of event {i}"
        slot.close()
    ctx.close()


def test_deferred_alternating_on_one_slot(px):
    """One slot: deferred and ordinary launches, events with and without modules for
    the big kernels, and a deferred event with an input error and such a module (the
    first launch ends it with the error; the next launch starts clean)."""
    ctx = px.Context(1856, 2000, 0)
    st = synth.stress_event(3)
    bad = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    bad["row"][5] = 200
    seq = [(st, True), (synth.async_event(5), False), (bad, True), (synth.async_event(6), True), (st, False),
           (st, True)]
    slot = px.Event(ctx, max(e["module"].size for e, _ in seq))
    for i, (e, dfr) in enumerate(seq):
        compare(_run(px, ctx, e, slot=slot, defer_big=dfr), oracle.cluster_event(e, 2000), f"step {i}")
    slot.close()
    ctx.close()


def test_deferred_calls_wait_for_the_callback(px):
    import torch
    ctx = px.Context(1856, 2000, 0)
    st = synth.stress_all_event(1)                         # long enough to be in flight below
    slot = px.Event(ctx, st["module"].size)
    d = px.Digis.from_numpy(st, "cuda", defer_big=True)
    px.acquire(slot, d, torch.cuda.current_stream())
    if px.query(slot) == px.E_NOT_READY:
        with pytest.raises(px.PxclError) as e:
            px.hits_enqueue(slot, torch.cuda.current_stream())
        assert e.value.code == px.E_BUSY
    px.wait(slot)
    compare(px.produce(slot).numpy(), oracle.cluster_event(st, 2000), "event")
    b = px.Batch(ctx, 1)
    with pytest.raises(px.PxclError) as e:
        px.acquire_batch(b, [slot], [d], torch.cuda.current_stream())
    assert e.value.code == px.E_INVAL
    b.close()
    slot.close()
    ctx.close()


def test_deferred_async_driver(px):
    import torch
    pool_np = [synth.async_event(40 + i) for i in range(5)] + [synth.stress_event(4)]
    ctx = px.Context(1856, 2000, 0)
    pool = [px.Digis.from_numpy(e, "cuda", defer_big=True) for e in pool_np]
    slots = [px.Event(ctx, max(e["module"].size for e in pool_np)) for _ in range(4)]
    streams = [torch.cuda.Stream() for _ in range(4)]
    refs = [oracle.cluster_event(e, 2000) for e in pool_np]
    n_ev = 4 * 12
    sizes = [pool_np[r % len(pool_np)]["module"].size for r in range(n_ev)]
    offs = np.concatenate([[0], np.cumsum([16 * n for n in sizes])]).astype(np.int64)
    results = torch.full((int(offs[-1]),), 0xFF, dtype=torch.uint8, device="cuda")
    st = px.run_async(ctx, slots, streams, pool, events_per_thread=12, cpu_task_ns=20000, results=results,
                      result_offsets=offs[:-1].tolist())
    assert st["events"] == n_ev and st["errors"] == 0
    host = results.cpu().numpy()
    for r in range(n_ev):
        ref, n = refs[r % len(pool_np)], sizes[r]
        k = ref["n_clusters"]
        blob = host[offs[r]: offs[r] + 16 * n].view(np.int32)
        got = {"status": 0, "n_clusters": k, "digi": blob[:n], "id": blob[n:n + k],
               "charge": blob[2 * n:2 * n + k], "size": blob[3 * n:3 * n + k]}
        compare(got, ref, f"async event {r}")
    for s in slots:
        s.close()
    ctx.close()


@pytest.mark.parametrize("graph", [False, True])
def test_deferred_batches(px, graph):
    """Batches with their big-module kernels deferred: one whose events need none
    (finished in one launch) and one mixing stress events (register and scratch mode)
    with sparse ones, some in any order, some with fused hits."""
    import torch
    print(f"deferred batch, graph={graph}", flush=True)
    ctx = px.Context(1856, 2000, 0)
    mixes = [[synth.async_event(50 + i) for i in range(4)],
             [synth.stress_event(5), synth.async_event(55), _shuffled(synth.batch_event(56), 3), synth.stress_event(6),
              synth.batch_event(57)]]
    for j, evs in enumerate(mixes):
        anyo = [i == 2 for i in range(len(evs))]
        hits = [i % 2 == 1 for i in range(len(evs))]
        slots = [px.Event(ctx, e["module"].size) for e in evs]
        digis = [px.Digis.from_numpy(e, "cuda", any_order=a, hits=h) for e, a, h in zip(evs, anyo, hits)]
        b = px.Batch(ctx, len(evs))
        for rep in range(2):                           # the second replays the captured graph
            f = px.Flag()
            px.acquire_batch(b, slots, digis, torch.cuda.current_stream(), flag=f, graph=graph, defer_big=True)
            for s in slots:
                px.wait(s)
            while f.fired == 0:
                pass
            for i, (s, e, a, h) in enumerate(zip(slots, evs, anyo, hits)):
                ref = oracle.hits(e, 2000, any_order=a) if h else oracle.cluster_event(e, 2000, any_order=a)
                compare(px.produce(s).numpy(), ref, f"mix {j}, event {i}, launch {rep}")
                if h:
                    px.hits_enqueue(s, torch.cuda.current_stream())
                    px.hits_wait(s)
                    hh = px.hits_produce(s).numpy()
                    assert np.array_equal(hh["x"], ref["x"]) and np.array_equal(hh["y"], ref["y"]), f"hits {j} {i}"
        b.close()
        for s in slots:
            s.close()
    ctx.close()


def test_deferred_serving(px):
    import torch
    pool_np = [synth.serve_event(i) for i in range(8)] + [synth.stress_event(7)]
    refs = [oracle.cluster_event(e, 2000) for e in pool_np]
    ctx = px.Context(1856)
    pool = [px.Digis.from_numpy(e, "cuda") for e in pool_np]
    n_req = 90
    arena = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    pinned = torch.empty(64 * 64, dtype=torch.uint8, pin_memory=True)
    batches = [px.Batch(ctx, 16) for _ in range(3)]
    streams = [torch.cuda.Stream() for _ in range(3)]
    sizes = [pool_np[r % len(pool_np)]["module"].size for r in range(n_req)]
    offs = np.concatenate([[0], np.cumsum([16 * n for n in sizes])]).astype(np.int64)
    results = torch.empty(int(offs[-1]), dtype=torch.uint8, device="cuda")
    st, status, ncl = px.serve(ctx, arena, pinned, batches, streams, pool, rate_hz=20000.0, n_requests=n_req,
                               budget_bytes=400 << 20, n_slots=64, max_batch=16, n_cpu_threads=4,
                               cpu_task_ns=10000, graph=True, seed=4, results=results,
                               result_offsets=offs[:-1].tolist(), max_inflight=2, defer_big=True)
    assert st["errors"] == 0 and st["events"] == n_req
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
