"""Helpers for the device tests: run events through the C ABI and compare with the
oracle, element by element (integer results: bit-exact)."""
from __future__ import annotations

import numpy as np


def compare(res: dict, ref: dict, what: str = ""):
    assert res["status"] == ref["status"], f"{what}: status {res['status']} != {ref['status']}"
    if ref["status"] != 0:
        return
    assert res["n_clusters"] == ref["n_clusters"], f"{what}: n_clusters {res['n_clusters']} != {ref['n_clusters']}"
    for k in ("id", "charge", "size", "digi"):
        a, b = np.asarray(res[k]), np.asarray(ref[k])
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0] if a.shape == b.shape else np.array([-1])
            raise AssertionError(f"{what}: {k} differs at {bad[:10]} (of {bad.size}); "
                                 f"gpu {a[bad[:5]] if bad[0] >= 0 else a.shape} ref {b[bad[:5]] if bad[0] >= 0 else b.shape}")


def run_events(px, ctx, events, where="cuda", stream=None, batch=None, graph=False, slots=None):
    """Cluster each numpy event; alone (one acquire per event) unless ``batch`` is
    given (then all in one acquire_batch).  Returns a list of numpy result dicts."""
    import torch
    stream = stream or torch.cuda.current_stream()
    own = slots is None
    if own:
        slots = [px.Event(ctx, max(1, e["module"].size)) for e in events]
    digis = [px.Digis.from_numpy(e, where) for e in events]
    out = []
    if batch is None:
        for s, d in zip(slots, digis):
            f = px.Flag()
            px.acquire(s, d, stream, flag=f)
            px.wait(s)
            assert f.fired == 1
            out.append(px.produce(s).numpy())
    else:
        f = px.Flag()
        px.acquire_batch(batch, slots, digis, stream, flag=f, graph=graph)
        for s in slots:
            px.wait(s)
        while f.fired == 0:
            pass
        assert f.fired == 1
        out = [px.produce(s).numpy() for s in slots]
    if own:
        for s in slots:
            s.close()
    return out
