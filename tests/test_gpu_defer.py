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
