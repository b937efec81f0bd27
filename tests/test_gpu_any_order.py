"""Digis in any order (PXCL_DIGIS_ANY_ORDER) on the device: the grouping kernels'
counting sort by module ahead of the clustering, against the oracle's any-order
entry point (which groups on the host and returns per-digi ids at the input
positions), bit-exact, for fully shuffled events of every configuration, through
single-event launches and batches (plain and graph-replayed, mixed with grouped
events), with errors, with hits, and alternating with grouped launches of the same
slots."""
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


def _run_alone(px, ctx, ev, where="cuda", any_order=True, slot=None):
    import torch
    own = slot is None
    slot = slot or px.Event(ctx, max(1, ev["module"].size))
    d = px.Digis.from_numpy(ev, where, any_order=any_order)
    f = px.Flag()
    px.acquire(slot, d, torch.cuda.current_stream(), flag=f)
    px.wait(slot)
    assert f.fired == 1
    r = px.produce(slot).numpy()
    if own:
        slot.close()
    return r


def _run_batch(px, ctx, evs, flags, graph, cap=None):
    import torch
    slots = [px.Event(ctx, cap or max(1, e["module"].size)) for e in evs]
    b = px.Batch(ctx, len(evs))
    digis = [px.Digis.from_numpy(e, "cuda", any_order=a) for e, a in zip(evs, flags)]
    f = px.Flag()
    px.acquire_batch(b, slots, digis, torch.cuda.current_stream(), flag=f, graph=graph)
    for s in slots:
        px.wait(s)
    while f.fired == 0:
        pass
    out = [px.produce(s).numpy() for s in slots]
    for s in slots:
        s.close()
    b.close()
    return out


@pytest.mark.parametrize("wg,mpw", [(64, 1), (256, 4), (512, 1)])
def test_shuffled_single_events(px, wg, mpw):
    print(f"any order, single events, shape {wg}x{mpw}", flush=True)
    ctx = px.Context(1856, 2000, 0)
    ctx.set_kernel_config(wg, mpw)
    evs = [dict(synth.plain_event(7), n_modules=1856), synth.async_event(4), synth.batch_event(5)]
    for i, e in enumerate(evs):
        sh = _shuffled(e, 10 + i)
        compare(_run_alone(px, ctx, sh), oracle.cluster_event(sh, 2000, any_order=True), f"event {i}")
    ctx.close()


def test_shuffled_host_pinned_input(px):
    ctx = px.Context(1856, 2000, 0)
    sh = _shuffled(synth.async_event(6), 3)
    compare(_run_alone(px, ctx, sh, where="pinned"), oracle.cluster_event(sh, 2000, any_order=True), "pinned")
    ctx.close()


def test_grouped_input_flagged_any_order_is_unchanged(px):
    ctx = px.Context(1856, 2000, 0)
    ev = synth.async_event(8)
    a = _run_alone(px, ctx, ev, any_order=True)
    b = _run_alone(px, ctx, ev, any_order=False)
    compare(a, b, "same digis, with and without the flag")
    compare(a, oracle.cluster_event(ev, 2000), "oracle")
    ctx.close()


@pytest.mark.parametrize("graph", [False, True])
def test_shuffled_batches_mixed_with_grouped(px, graph):
    print(f"any order, batch, graph={graph}", flush=True)
    ctx = px.Context(1856, 2000, 0)
    base = [synth.batch_event(i) for i in range(12)]
    flags = [i % 3 != 0 for i in range(12)]             # every third event stays grouped
    evs = [_shuffled(e, 20 + i) if a else e for i, (e, a) in enumerate(zip(base, flags))]
    res = _run_batch(px, ctx, evs, flags, graph, cap=max(e["module"].size for e in evs))
    for i, (r, e, a) in enumerate(zip(res, evs, flags)):
        compare(r, oracle.cluster_event(e, 2000, any_order=a), f"batch event {i} (any order {a})")
    # every event in any order: no segmentation kernel at all
    res = _run_batch(px, ctx, [_shuffled(e, 40 + i) for i, e in enumerate(base[:6])], [True] * 6, graph)
    for i, (r, e) in enumerate(zip(res, base[:6])):
        compare(r, oracle.cluster_event(_shuffled(e, 40 + i), 2000, any_order=True), f"all-shuffled event {i}")
    ctx.close()


def test_shuffled_stress_batch(px):
    print("any order, stress batch", flush=True)
    ctx = px.Context(1856, 2000, 0)
    evs = [_shuffled(synth.stress_event(i), 60 + i) for i in range(4)]
    res = _run_batch(px, ctx, evs, [True] * 4, True)
    for i, (r, e) in enumerate(zip(res, evs)):
        compare(r, oracle.cluster_event(e, 2000, any_order=True), f"stress event {i}")
    ctx.close()


def test_shuffled_errors_isolated_in_a_batch(px):
    ctx = px.Context(1856, 2000, 0)
    good = [_shuffled(synth.batch_event(30 + i), 70 + i) for i in range(3)]
    bad_range = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in good[0].items()}
    bad_range["module"][17] = 1856
    dup = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in good[1].items()}
    j = int(np.nonzero(dup["module"] == dup["module"][0])[0][1])
    dup["row"][j], dup["col"][j] = dup["row"][0], dup["col"][0]
    evs = [bad_range, good[2], dup, good[0]]
    for graph in (False, True):
        res = _run_batch(px, ctx, evs, [True] * 4, graph, cap=max(e["module"].size for e in evs))
        st = [r["status"] for r in res]
        assert st == [px.E_RANGE, 0, px.E_DUP_PIXEL, 0], st
        for i, (r, e) in enumerate(zip(res, evs)):
            compare(r, oracle.cluster_event(e, 2000, any_order=True), f"event {i}, graph {graph}")
    ctx.close()


def test_shuffled_hits(px):
    import torch
    ctx = px.Context(1856, 2000, 0)
    sh = _shuffled(synth.async_event(9), 11)
    slot = px.Event(ctx, sh["module"].size)
    d = px.Digis.from_numpy(sh, "cuda", any_order=True)
    px.acquire(slot, d, torch.cuda.current_stream())
    px.hits_enqueue(slot, torch.cuda.current_stream())
    px.hits_wait(slot)
    ref = oracle.hits(sh, 2000, any_order=True)
    compare(px.produce(slot).numpy(), ref, "clusters")
    h = px.hits_produce(slot).numpy()
    assert h["n_hits"] == ref["n_clusters"]
    assert np.array_equal(h["x"], ref["x"]) and np.array_equal(h["y"], ref["y"])
    slot.close()
    ctx.close()


def test_slot_alternates_grouped_and_shuffled(px):
    """The same slots used for grouped, shuffled, empty and shuffled-with-error events
    in turn: what one launch leaves in the workspace does not reach the next."""
    ctx = px.Context(1856, 2000, 0)
    evs = [synth.async_event(i) for i in range(3)]
    slot = px.Event(ctx, max(e["module"].size for e in evs))
    empty = {k: evs[0][k][:0] for k in ("module", "row", "col", "adc")}
    empty["n_modules"] = 1856
    bad = _shuffled(evs[2], 5)
    bad["module"] = bad["module"].copy()
    bad["module"][3] = 4000
    seq = [(evs[0], False), (_shuffled(evs[1], 1), True), (empty, True), (bad, True), (evs[2], False),
           (_shuffled(evs[0], 2), True)]
    for i, (e, a) in enumerate(seq):
        compare(_run_alone(px, ctx, e, any_order=a, slot=slot), oracle.cluster_event(e, 2000, any_order=a),
                f"step {i}")
    slot.close()
    ctx.close()


def test_all_modules_hot_stress_event(px):
    """Maximum-size case: the stress configuration read literally (186 of 1,856 modules
    hot at 20 % occupancy, ~2.5 million digis in one event) through the single-event
    kernels, as a one-event batch replayed from a graph (segmentation kernel), and
    shuffled (grouping kernels), bit-exact against the oracle."""
    print("stress event with 10 % of all modules hot", flush=True)
    ev = synth.stress_all_event(0)
    assert ev["module"].size > 2_400_000
    ref = oracle.cluster_event(ev, 2000)
    assert ref["status"] == 0
    ctx = px.Context(1856, 2000, 0)
    compare(_run_alone(px, ctx, ev, any_order=False), ref, "alone")
    compare(_run_batch(px, ctx, [ev], [False], True)[0], ref, "one-event batch, graph")
    sh = _shuffled(ev, 90)
    compare(_run_alone(px, ctx, sh), oracle.cluster_event(sh, 2000, any_order=True), "shuffled")
    ctx.close()
