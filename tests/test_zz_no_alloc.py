"""The allocation-free entry point (pxcl_cluster_noalloc: scratch in the library's
fixed per-device array, caller-owned outputs) against pxcl_acquire on the same
events, and both against the oracle: bit-exact, over calls in a row whose inputs
shrink, so that every call must work from what the previous one left in the shared
array."""
from __future__ import annotations

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


def _subset(ev, keep_modules):
    """The digis of the listed modules (still grouped by ascending module)."""
    m = np.isin(ev["module"], np.asarray(sorted(keep_modules)))
    out = {k: ev[k][m] for k in ("module", "row", "col", "adc")}
    out["n_modules"] = ev["n_modules"]
    return out


def _dense_event(limit):
    """Modules of a high-pileup event, largest first, up to `limit` digis: the
    serpentine (scratch mode), the hot modules (register mode) and sparse ones."""
    ev = synth.stress_event(0)
    ids, cnt = np.unique(ev["module"], return_counts=True)
    keep, tot = [], 0
    for i in np.argsort(-cnt, kind="stable"):
        if tot + cnt[i] <= limit:
            keep.append(int(ids[i]))
            tot += int(cnt[i])
    sub = _subset(ev, keep)
    assert np.bincount(sub["module"]).max() > 16384      # a scratch-mode module is in it
    return sub


def test_noalloc_matches_acquire_on_shrinking_calls(px):
    import torch
    ctx = px.Context(1856, 2000, 0)
    evs = [_dense_event(px.NOALLOC_MAX_DIGIS), synth.async_event(3), synth.plain_event(1, n_modules=8)]
    evs[2]["n_modules"] = 1856
    sizes = [e["module"].size for e in evs]
    assert sizes[0] > sizes[1] > sizes[2] and sizes[0] <= px.NOALLOC_MAX_DIGIS
    ref_acq = run_events(px, ctx, evs)
    out = px.NoAllocOutputs(max(sizes))
    stream = torch.cuda.current_stream()
    for rep in range(2):
        for i, e in enumerate(evs):
            print(f"noalloc call rep {rep} event {i}: {e['module'].size} digis", flush=True)
            d = px.Digis.from_numpy(e, "cuda")
            out.digi.fill_(-7)                     # every per-digi entry must be rewritten
            tag = px.cluster_noalloc(ctx, d, out, stream)
            stream.synchronize()
            res = out.numpy(e["module"].size, tag)
            compare(res, ref_acq[i], f"noalloc vs acquire, rep {rep} event {i}")
            compare(res, oracle.cluster_event(e, 2000), f"noalloc vs oracle, rep {rep} event {i}")
    ctx.close()


def test_noalloc_empty_then_event_and_limits(px):
    import torch
    ctx = px.Context(64, 2000, 0)
    out = px.NoAllocOutputs(64)
    stream = torch.cuda.current_stream()
    ev = synth.plain_event(2)
    empty = {k: ev[k][:0] for k in ("module", "row", "col", "adc")}
    empty["n_modules"] = 64
    tag = px.cluster_noalloc(ctx, px.Digis.from_numpy(empty, "cuda"), out, stream)
    stream.synchronize()
    r = out.numpy(0, tag)
    assert r["status"] == 0 and r["n_clusters"] == 0
    # an input error travels in the status words; the next call is clean again
    bad = {k: ev[k].copy() for k in ("module", "row", "col", "adc")}
    bad["n_modules"] = 64
    bad["row"][5] = 200
    out2 = px.NoAllocOutputs(ev["module"].size)
    tag = px.cluster_noalloc(ctx, px.Digis.from_numpy(bad, "cuda"), out2, stream)
    stream.synchronize()
    assert out2.numpy(ev["module"].size, tag)["status"] == oracle.cluster_event(bad, 2000)["status"] == px.E_RANGE
    tag = px.cluster_noalloc(ctx, px.Digis.from_numpy(ev, "cuda"), out2, stream)
    stream.synchronize()
    compare(out2.numpy(ev["module"].size, tag), oracle.cluster_event(ev, 2000), "after an input error")
    # sizes beyond the fixed array are refused before anything is queued
    n = px.NOALLOC_MAX_DIGIS + 1
    z = torch.zeros(n, dtype=torch.uint16, device="cuda")
    with pytest.raises(px.PxclError) as ei:
        px.cluster_noalloc(ctx, px.Digis(z, z, z, z), px.NoAllocOutputs(n), stream)
    assert ei.value.code == px.E_CAPACITY
    ctx.close()
