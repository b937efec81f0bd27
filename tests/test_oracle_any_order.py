"""Pins of the oracle's any-order entry point (digis not grouped by module: the raw
data the producer of the paper's Figure 1 reads, Sec. 3).  The definition of the
clustering does not depend on the order of the digis, so the expected values come
from order-free references: the pairwise brute force, min-label propagation on
binary patterns, and scipy's labeller, all run on digis shuffled across modules.
A per-digi id must stay with its digi wherever the shuffle put it."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2004_04334_amd import synth
from tests import brute

PIX, ROWS, COLS = 66560, 160, 416


def _shuffled(ev, seed):
    p = np.random.default_rng(seed).permutation(ev["module"].size)
    return {k: (v[p] if isinstance(v, np.ndarray) else v) for k, v in ev.items()}, p


def test_patterns_shuffled_across_modules(oracle_mod):
    """Every 4x4 pattern (one per module), its digis shuffled across all modules:
    against min-label propagation to a fixed point."""
    rng = np.random.default_rng(3)
    codes = np.arange(1 << 12) * 16 + 5
    ev, fired = brute.patterns_event(codes, 4, 4, 77, 300, rng)
    lab = brute.propagate_labels(fired)
    digi, cid, chg, siz = brute.expected_from_labels(ev, fired, lab, 4, 77, 300, 2000)
    sh, p = _shuffled(ev, 4)
    assert np.any(np.diff(sh["module"].astype(np.int64)) < 0)
    res = oracle_mod.cluster_event(sh, 2000, any_order=True)
    assert res["status"] == 0
    np.testing.assert_array_equal(res["digi"], digi[p])
    np.testing.assert_array_equal(res["id"], cid)
    np.testing.assert_array_equal(res["charge"], chg)
    np.testing.assert_array_equal(res["size"], siz)


def test_random_small_shuffled_vs_pairwise(oracle_mod):
    """Small random events over a few modules, shuffled: against the all-pairs
    labeller, which never looks at the order of the digis."""
    rng = np.random.default_rng(9)
    for t in range(60):
        n_modules = int(rng.integers(1, 5))
        n = int(rng.integers(0, 40))
        lin = rng.choice(n_modules * 12 * 12, size=n, replace=False)
        m, rest = np.divmod(lin, 144)
        r, c = 70 + rest % 12, 200 + rest // 12
        order = rng.permutation(n)
        ev = {"module": m[order].astype(np.uint16), "row": r[order].astype(np.uint16),
              "col": c[order].astype(np.uint16), "adc": rng.integers(0, 4001, n).astype(np.uint16),
              "n_modules": n_modules}
        cut = int(rng.choice([0, 2000, 5000]))
        ids, kept = brute.pairwise_components(ev["module"], ev["row"], ev["col"], ev["adc"], cut)
        res = oracle_mod.cluster_event(ev, cut, any_order=True)
        assert res["status"] == 0, t
        np.testing.assert_array_equal(res["digi"], ids)
        assert [tuple(x) for x in zip(res["id"], res["charge"], res["size"])] == kept, t


def test_full_modules_shuffled_vs_scipy(oracle_mod):
    """Three full modules at 5 % occupancy, digis shuffled across them: against
    scipy.ndimage.label with a 3x3 structure, id = smallest linear index."""
    ndimage = pytest.importorskip("scipy.ndimage")
    rng = np.random.default_rng(21)
    fired = rng.random((3, ROWS, COLS)) < 0.05
    m, r, c = np.nonzero(fired)
    ev, p = _shuffled(synth.from_pixels(m, r, c, n_modules=3, seed=22), 23)
    res = oracle_mod.cluster_event(ev, 0, any_order=True)
    assert res["status"] == 0
    em, er, ec = (ev[k].astype(np.int64) for k in ("module", "row", "col"))
    exp = np.empty(em.size, np.int64)
    lin = np.arange(COLS)[None, :] * ROWS + np.arange(ROWS)[:, None]
    for mm in range(3):
        lab, nlab = ndimage.label(fired[mm], structure=np.ones((3, 3), dtype=int))
        mins = np.full(nlab + 1, np.iinfo(np.int64).max)
        np.minimum.at(mins, lab[fired[mm]], lin[fired[mm]])
        sel = em == mm
        exp[sel] = mm * PIX + mins[lab[er[sel], ec[sel]]]
    np.testing.assert_array_equal(res["digi"], exp)
    uid, inv = np.unique(exp, return_inverse=True)
    np.testing.assert_array_equal(res["id"], uid)
    np.testing.assert_array_equal(res["size"], np.bincount(inv))


@pytest.mark.parametrize("maker", ["plain_event", "batch_event", "stress_event"])
def test_workload_events_any_order_invariant(oracle_mod, maker):
    """Workload events, grouped and shuffled: identical clusters, and each digi's id
    follows the digi (the grouped input is the shuffle's special case)."""
    ev = getattr(synth, maker)(1)
    ref = oracle_mod.cluster_event(ev, 2000)
    same = oracle_mod.cluster_event(ev, 2000, any_order=True)
    sh, p = _shuffled(ev, 5)
    res = oracle_mod.cluster_event(sh, 2000, any_order=True)
    for r in (same, res):
        assert r["status"] == 0 and r["n_clusters"] == ref["n_clusters"]
        for k in ("id", "charge", "size"):
            np.testing.assert_array_equal(r[k], ref[k])
    np.testing.assert_array_equal(same["digi"], ref["digi"])
    np.testing.assert_array_equal(res["digi"], ref["digi"][p])


def test_any_order_errors(oracle_mod):
    """Out of range: -6 (before anything else); the same pixel twice, far apart in the
    input and with other modules between: -5; decreasing module ids are no error."""
    base = synth.plain_event(2, n_modules=6)
    sh, _ = _shuffled(base, 6)
    assert oracle_mod.cluster_event(sh, 2000)["status"] == -7          # the grouped entry point
    assert oracle_mod.cluster_event(sh, 2000, any_order=True)["status"] == 0
    dup = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in sh.items()}
    i, j = 3, dup["module"].size - 2
    for k in ("module", "row", "col"):
        dup[k][j] = dup[k][i]
    assert oracle_mod.cluster_event(dup, 2000, any_order=True)["status"] == -5
    rng_bad = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in dup.items()}
    rng_bad["col"][7] = 416
    assert oracle_mod.cluster_event(rng_bad, 2000, any_order=True)["status"] == -6
    rng_bad["col"][7] = 3
    rng_bad["module"][9] = 6
    assert oracle_mod.cluster_event(rng_bad, 2000, any_order=True)["status"] == -6
    empty = {k: np.zeros(0, np.uint16) for k in ("module", "row", "col", "adc")}
    r = oracle_mod.cluster_event(dict(empty, n_modules=4), 2000, any_order=True)
    assert r["status"] == 0 and r["n_clusters"] == 0
