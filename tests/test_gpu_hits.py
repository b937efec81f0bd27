"""Hits (the charge-weighted centroid of every kept cluster) as a consumer of an
event's clusters: on the event's own stream, on another stream while the event is
still in flight (the consumer waits for the event's completion event), after a
batch launch; bit-exact against the oracle's hits."""
from __future__ import annotations

import time

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


def _check_hits(px, slot, ev, what):
    ref = oracle.hits(ev, 2000)
    compare(px.produce(slot).numpy(), ref, what)
    h = px.hits_produce(slot)
    assert h.status == 0 and h.n_hits == ref["n_clusters"], what
    hn = h.numpy()
    assert np.array_equal(hn["x"], ref["x"]) and np.array_equal(hn["y"], ref["y"]), f"{what}: hits differ"


def test_hits_same_stream(px):
    import torch
    evs = [synth.plain_event(0), synth.async_event(7), synth.stress_event(3)]
    for i, ev in enumerate(evs):
        print(f"hits same stream, event {i}", flush=True)
        ctx = px.Context(ev["n_modules"], 2000)
        slot = px.Event(ctx, ev["module"].size)
        s = torch.cuda.Stream()
        d = px.Digis.from_numpy(ev, "cuda")
        px.acquire(slot, d, s)
        px.hits_enqueue(slot, s)                   # queued behind the clusters, no wait needed
        px.hits_wait(slot)
        px.wait(slot)
        _check_hits(px, slot, ev, f"event {i}")
        slot.close()
        ctx.close()


def test_hits_on_another_stream_while_in_flight(px):
    import torch
    ev = synth.async_event(8)
    ctx = px.Context(1856, 2000)
    slot = px.Event(ctx, ev["module"].size)
    d = px.Digis.from_numpy(ev, "cuda")
    s_ev, s_hits = torch.cuda.Stream(), torch.cuda.Stream()
    calls = []
    with torch.cuda.stream(s_ev):
        torch.cuda._sleep(100_000_000)             # keep the event's stream busy (~50 ms)
    px.acquire(slot, d, s_ev)
    assert px.query(slot) == px.E_NOT_READY
    px.hits_enqueue(slot, s_hits, done_cb=lambda st: calls.append(st))
    assert px.hits_query(slot) == px.E_NOT_READY
    with pytest.raises(px.PxclError) as ei:
        px.hits_enqueue(slot, s_hits)              # one hits launch in flight per event
    assert ei.value.code == px.E_BUSY
    with pytest.raises(px.PxclError) as ei:
        px.acquire(slot, d, s_ev)                  # the slot is still read by the hits
    assert ei.value.code == px.E_BUSY
    px.hits_wait(slot)
    px.wait(slot)
    time.sleep(0.01)
    assert calls == [0]
    _check_hits(px, slot, ev, "chained")
    slot.close()
    ctx.close()


def test_hits_complete_after_their_event(px):
    """A hits launch on the event's stream finishes right after the event: its
    completion is still delivered after the event's own (the event reads complete in
    the hits callback), every time."""
    import torch
    ev = synth.async_event(12)
    ctx = px.Context(1856, 2000)
    slot = px.Event(ctx, ev["module"].size)
    d = px.Digis.from_numpy(ev, "cuda")
    s = torch.cuda.Stream()
    seen = []
    for i in range(200):
        px.acquire(slot, d, s)
        px.hits_enqueue(slot, s, done_cb=lambda st: seen.append((st, px.query(slot))))
        px.hits_wait(slot)
        px.wait(slot)
        px.produce(slot)
        px.hits_produce(slot)
    assert seen == [(0, px.OK)] * 200
    slot.close()
    ctx.close()


def test_hits_after_batch(px):
    import torch
    evs = [synth.batch_event(40 + i) for i in range(6)]
    ctx = px.Context(1856, 2000)
    b = px.Batch(ctx, 8)
    slots = [px.Event(ctx, max(e["module"].size for e in evs)) for _ in evs]
    digis = [px.Digis.from_numpy(e, "cuda") for e in evs]
    s = torch.cuda.Stream()
    f = px.Flag()
    px.acquire_batch(b, slots, digis, s, flag=f, graph=True)
    other = torch.cuda.Stream()
    for sl in slots:
        px.hits_enqueue(sl, other)                 # some may still be in flight
    for i, (sl, e) in enumerate(zip(slots, evs)):
        px.hits_wait(sl)
        px.wait(sl)
        _check_hits(px, sl, e, f"batch event {i}")
    for sl in slots:
        sl.close()
    b.close()
    ctx.close()


def test_hits_errors(px):
    ctx = px.Context(4, 2000)
    ev = synth.plain_event(1, n_modules=4)
    slot = px.Event(ctx, ev["module"].size)
    with pytest.raises(px.PxclError) as ei:
        px.hits_enqueue(slot)                      # nothing acquired
    assert ei.value.code == px.E_INVAL
    bad = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in ev.items()}
    bad["row"][3] = 200
    px.acquire(slot, px.Digis.from_numpy(bad, "cuda"))
    px.hits_enqueue(slot)
    px.hits_wait(slot)
    assert px.hits_produce(slot).status == px.E_RANGE
    px.acquire(slot, px.Digis.from_numpy(ev, "cuda"))   # the slot is reusable
    px.hits_enqueue(slot)
    px.hits_wait(slot)
    px.wait(slot)
    _check_hits(px, slot, ev, "after error")
    slot.close()
    ctx.close()


def _wait_flag(f, timeout=30.0):
    t0 = time.time()
    while f.fired == 0:
        assert time.time() - t0 < timeout, "callback did not fire"
        time.sleep(0.0005)


def test_copy_to_host_on_demand(px):
    """Results and hits reach pinned host memory only when asked: after completion
    (exact sizes), and while the event is still in flight on another stream (a bound
    on the sizes, the count filled in by the callback)."""
    import torch
    ev = synth.async_event(9)
    n = ev["module"].size
    ref = oracle.hits(ev, 2000)
    ctx = px.Context(1856, 2000)
    slot = px.Event(ctx, n)
    d = px.Digis.from_numpy(ev, "cuda")
    # 1. after completion, same stream
    px.acquire(slot, d)
    px.wait(slot)
    px.hits_enqueue(slot)
    px.hits_wait(slot)
    dst = px.HostCopy(ref["n_clusters"], n_digis=n, hits=True)
    f = px.Flag()
    px.copy_to_host(slot, dst, flag=f)
    _wait_flag(f)
    got = dst.numpy(n)
    assert f.status == 0 and got["status"] == 0
    compare(got, ref, "copy after completion")
    assert np.array_equal(got["x"], ref["x"]) and np.array_equal(got["y"], ref["y"])
    small = px.HostCopy(ref["n_clusters"] - 1)
    with pytest.raises(px.PxclError) as ei:
        px.copy_to_host(slot, small)
    assert ei.value.code == px.E_CAPACITY
    # 2. while in flight, on another stream
    s_ev, s_cp = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s_ev):
        torch.cuda._sleep(100_000_000)
    px.acquire(slot, d, s_ev)
    px.hits_enqueue(slot, s_ev)
    dst2 = px.HostCopy(n, n_digis=n, hits=True)
    f2 = px.Flag()
    px.copy_to_host(slot, dst2, s_cp, flag=f2)
    assert px.copy_query(slot) == px.E_NOT_READY
    with pytest.raises(px.PxclError) as ei:
        px.acquire(slot, d, s_ev)
    assert ei.value.code == px.E_BUSY
    _wait_flag(f2)
    got2 = dst2.numpy(n)
    compare(got2, ref, "copy while in flight")
    assert np.array_equal(got2["x"], ref["x"]) and np.array_equal(got2["y"], ref["y"])
    px.wait(slot)
    px.hits_wait(slot)
    slot.close()
    ctx.close()


# ---------------------------------------------------------------------------
# hits fused into the clustering (PXCL_DIGIS_HITS): no hits kernel; the same values
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("wg,mpw", [(64, 1), (256, 4), (512, 1)])
def test_fused_hits_single_events(px, wg, mpw):
    import torch
    evs = [dict(synth.plain_event(2), n_modules=1856), synth.async_event(9), synth.stress_event(5)]
    ctx = px.Context(1856, 2000)
    ctx.set_kernel_config(wg, mpw)
    for i, ev in enumerate(evs):
        print(f"fused hits, shape {wg}x{mpw}, event {i}", flush=True)
        slot = px.Event(ctx, ev["module"].size)
        s, other = torch.cuda.Stream(), torch.cuda.Stream()
        px.acquire(slot, px.Digis.from_numpy(ev, "cuda", hits=True), s)
        px.hits_enqueue(slot, other)               # another stream: waits, queues no kernel
        px.hits_wait(slot)
        px.wait(slot)
        _check_hits(px, slot, ev, f"fused, event {i}")
        slot.close()
    ctx.close()


@pytest.mark.parametrize("graph", [False, True])
def test_fused_hits_batch_mixed(px, graph):
    """A batch mixing events with fused hits, events without them and shuffled events
    with fused hits; then the hits of every event with fused hits."""
    import torch
    base = [synth.batch_event(50 + i) for i in range(8)]
    flags = [(i % 2 == 0, i % 4 == 2) for i in range(8)]          # (fused hits, any order)
    evs = []
    for i, (e, (h, a)) in enumerate(zip(base, flags)):
        if a:
            p = np.random.default_rng(80 + i).permutation(e["module"].size)
            e = {k: (v[p] if isinstance(v, np.ndarray) else v) for k, v in e.items()}
        evs.append(e)
    ctx = px.Context(1856, 2000)
    cap = max(e["module"].size for e in evs)
    slots = [px.Event(ctx, cap) for _ in evs]
    b = px.Batch(ctx, len(evs))
    digis = [px.Digis.from_numpy(e, "cuda", hits=h, any_order=a) for e, (h, a) in zip(evs, flags)]
    f = px.Flag()
    px.acquire_batch(b, slots, digis, torch.cuda.current_stream(), flag=f, graph=graph)
    for s in slots:
        px.wait(s)
    for i, (slot, e, (h, a)) in enumerate(zip(slots, evs, flags)):
        ref = oracle.hits(e, 2000, any_order=a)
        compare(px.produce(slot).numpy(), ref, f"batch event {i}")
        if h:
            px.hits_enqueue(slot, torch.cuda.current_stream())
            px.hits_wait(slot)
            hn = px.hits_produce(slot).numpy()
            assert np.array_equal(hn["x"], ref["x"]) and np.array_equal(hn["y"], ref["y"]), f"hits of event {i}"
    for s in slots:
        s.close()
    b.close()
    ctx.close()


def test_fused_hits_repeated_on_one_slot(px):
    """The hit sums are zero between launches (the compaction clears what it read, the
    host clears the slot after an error): one slot runs several events with fused hits
    in turn, one of them with an input error, and every event's hits are exact."""
    import torch
    evs = [synth.async_event(20), synth.batch_event(21), synth.async_event(22)]
    bad = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in evs[1].items()}
    bad["row"][3] = 170
    seq = [evs[0], evs[1], bad, evs[0], evs[2], evs[1]]
    ctx = px.Context(1856, 2000)
    slot = px.Event(ctx, max(e["module"].size for e in evs))
    s = torch.cuda.current_stream()
    for i, ev in enumerate(seq):
        px.acquire(slot, px.Digis.from_numpy(ev, "cuda", hits=True), s)
        px.hits_enqueue(slot, s)
        px.hits_wait(slot)
        px.wait(slot)
        ref = oracle.hits(ev, 2000)
        compare(px.produce(slot).numpy(), ref, f"step {i}")
        if ref["status"] == 0:
            hn = px.hits_produce(slot).numpy()
            assert np.array_equal(hn["x"], ref["x"]) and np.array_equal(hn["y"], ref["y"]), f"hits at step {i}"
    slot.close()
    ctx.close()
