"""Pins of the CPU oracle against things other than itself: exhaustive brute force on
tiny grids, scipy's textbook labeller, closed forms and invariants.

The paper prints no worked example for the clustering its Figure 1 names
("ClusterProducer", Sec. 3), so nothing here is pinned to a printed value; every
expected value is derived from the definition (8-connectivity, id = smallest
linear index module*66560 + col*160 + row, charge cut) by an independent route.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_2004_04334_amd import synth
from tests import brute

PIX, ROWS, COLS = 66560, 160, 416


def _check_patterns(oracle_mod, codes, R, C, r0, c0, seed, cut):
    rng = np.random.default_rng(seed)
    ev, fired = brute.patterns_event(codes, R, C, r0, c0, rng)
    lab = brute.propagate_labels(fired)
    digi, cid, chg, siz = brute.expected_from_labels(ev, fired, lab, R, r0, c0, cut)
    res = oracle_mod.cluster_event(ev, charge_cut=cut)
    assert res["status"] == 0
    np.testing.assert_array_equal(res["digi"], digi)
    np.testing.assert_array_equal(res["id"], cid)
    np.testing.assert_array_equal(res["charge"], chg)
    np.testing.assert_array_equal(res["size"], siz)


@pytest.mark.parametrize("r0,c0", [(0, 0), (156, 412), (78, 200)])
def test_exhaustive_4x4(oracle_mod, r0, c0):
    codes = np.arange(1 << 16)
    for k in range(0, codes.size, 16384):
        _check_patterns(oracle_mod, codes[k:k + 16384], 4, 4, r0, c0, seed=k + r0, cut=0)
        _check_patterns(oracle_mod, codes[k:k + 16384], 4, 4, r0, c0, seed=k + 1, cut=3000)


@pytest.mark.parametrize("R,C,r0,c0", [(4, 5, 0, 0), (5, 4, 155, 412)])
def test_exhaustive_4x5_5x4(oracle_mod, R, C, r0, c0):
    codes = np.arange(1 << 20)
    for k in range(0, codes.size, 16384):
        _check_patterns(oracle_mod, codes[k:k + 16384], R, C, r0, c0, seed=k, cut=2000)


@pytest.mark.parametrize("occ", [0.005, 0.05, 0.5])
def test_full_module_vs_scipy(oracle_mod, occ):
    ndimage = pytest.importorskip("scipy.ndimage")
    rng = np.random.default_rng(int(occ * 1e4))
    for m_count in (1, 3):
        fired = rng.random((m_count, ROWS, COLS)) < occ
        m, r, c = np.nonzero(fired)
        ev = synth.from_pixels(m, r, c, n_modules=m_count, seed=int(occ * 1e3) + m_count)
        res = oracle_mod.components(ev)
        assert res["status"] == 0
        exp = np.empty(ev["module"].size, dtype=np.int64)
        em, er, ec = (ev[k].astype(np.int64) for k in ("module", "row", "col"))
        for mm in range(m_count):
            lab, nlab = ndimage.label(fired[mm], structure=np.ones((3, 3), dtype=int))
            lin = np.arange(COLS)[None, :] * ROWS + np.arange(ROWS)[:, None]
            mins = np.full(nlab + 1, np.iinfo(np.int64).max)
            np.minimum.at(mins, lab[fired[mm]], lin[fired[mm]])
            sel = em == mm
            exp[sel] = mm * PIX + mins[lab[er[sel], ec[sel]]]
        np.testing.assert_array_equal(res["digi"], exp)
        uid, inv = np.unique(exp, return_inverse=True)
        np.testing.assert_array_equal(res["id"], uid)
        np.testing.assert_array_equal(res["size"], np.bincount(inv))
        np.testing.assert_array_equal(res["charge"], np.bincount(inv, weights=ev["adc"].astype(np.int64)).astype(np.int64))


def _single_module(oracle_mod, r, c, m=0, n_modules=None, adc=None, cut=0, seed=0):
    r = np.asarray(r)
    ev = synth.from_pixels(np.full(r.size, m), r, c, adc=adc,
                           n_modules=n_modules or m + 1, seed=seed)
    return ev, oracle_mod.cluster_event(ev, charge_cut=cut)


def test_closed_form_single_pixel(oracle_mod):
    ev, res = _single_module(oracle_mod, [17], [301], m=5, adc=[1234])
    assert res["n_clusters"] == 1
    assert res["id"][0] == 5 * PIX + 301 * ROWS + 17
    assert res["size"][0] == 1 and res["charge"][0] == 1234


@pytest.mark.parametrize("col", [0, 207, 415])
def test_closed_form_column_track(oracle_mod, col):
    r, c = synth.column_track(col)
    ev, res = _single_module(oracle_mod, r, c, m=3)
    assert res["n_clusters"] == 1
    assert res["size"][0] == ROWS
    assert res["id"][0] == 3 * PIX + col * ROWS
    assert res["charge"][0] == int(ev["adc"].astype(np.int64).sum())


def test_closed_form_diagonals(oracle_mod):
    k = np.arange(ROWS)
    for r, c in ((k, k), (k, 300 - k), (k, 415 - k)):
        ev, res = _single_module(oracle_mod, r, c)
        assert res["n_clusters"] == 1, "a diagonal line is one 8-connected cluster"
        assert res["size"][0] == ROWS
        assert res["id"][0] == int((c * ROWS + r).min())


def test_closed_form_checkerboard_and_lattice(oracle_mod):
    rr, cc = np.meshgrid(np.arange(ROWS), np.arange(COLS), indexing="ij")
    sel = (rr + cc) % 2 == 0
    ev, res = _single_module(oracle_mod, rr[sel], cc[sel], m=2)
    assert res["n_clusters"] == 1 and res["size"][0] == 33280 and res["id"][0] == 2 * PIX
    sel = (rr % 2 == 0) & (cc % 2 == 0)
    ev, res = _single_module(oracle_mod, rr[sel], cc[sel], m=1)
    assert res["n_clusters"] == 16640
    np.testing.assert_array_equal(res["size"], 1)
    np.testing.assert_array_equal(res["id"], np.sort(PIX + cc[sel] * ROWS + rr[sel]))


@pytest.mark.parametrize("row_wise,size", [(True, 33359), (False, 33487)])
def test_closed_form_serpentine(oracle_mod, row_wise, size):
    r, c = synth.serpentine(row_wise)
    assert r.size == size
    ev, res = _single_module(oracle_mod, r, c, m=7)
    assert res["n_clusters"] == 1 and res["size"][0] == size and res["id"][0] == 7 * PIX


def test_closed_form_full_module(oracle_mod):
    rr, cc = np.meshgrid(np.arange(ROWS), np.arange(COLS), indexing="ij")
    ev, res = _single_module(oracle_mod, rr.ravel(), cc.ravel(), m=9, n_modules=12)
    assert res["n_clusters"] == 1 and res["size"][0] == PIX and res["id"][0] == 9 * PIX


def test_closed_form_no_wraparound(oracle_mod):
    # (r, 415) and (r+1, 0) are adjacent in no layout
    ev, res = _single_module(oracle_mod, [40, 41], [415, 0])
    assert res["n_clusters"] == 2
    # (159, c) in module m and (0, c) in module m+1 are separate
    ev = synth.from_pixels([4, 5], [159, 0], [33, 33], n_modules=6)
    res = oracle_mod.components(ev)
    assert res["n_clusters"] == 2
    # a knight's move is not adjacent, a diagonal step is
    ev, res = _single_module(oracle_mod, [10, 11], [10, 12])
    assert res["n_clusters"] == 2
    ev, res = _single_module(oracle_mod, [10, 11], [10, 11])
    assert res["n_clusters"] == 1


def test_closed_form_cut_boundary(oracle_mod):
    # three isolated clusters with charges 1999 / 2000 / 2001
    r = [5, 6, 50, 51, 100]
    c = [5, 5, 60, 60, 300]
    adc = [999, 1000, 1000, 1000, 2001]
    ev, res = _single_module(oracle_mod, r, c, adc=adc, cut=2000)
    assert res["n_clusters"] == 2
    np.testing.assert_array_equal(res["charge"], [2000, 2001])
    np.testing.assert_array_equal(res["id"], [60 * ROWS + 50, 300 * ROWS + 100])
    kept = {60 * ROWS + 50, 300 * ROWS + 100}
    for i in range(5):
        lin = int(ev["col"][i]) * ROWS + int(ev["row"][i])
        exp = -1 if lin in (5 * ROWS + 5, 5 * ROWS + 6) else (60 * ROWS + 50 if lin < 300 * ROWS else 300 * ROWS + 100)
        assert res["digi"][i] == exp
        assert (exp == -1) or exp in kept


def test_closed_form_adc_zero_and_empty(oracle_mod):
    ev, res = _single_module(oracle_mod, [0, 1], [0, 0], adc=[0, 0], cut=0)
    assert res["n_clusters"] == 1 and res["charge"][0] == 0 and res["size"][0] == 2
    ev, res = _single_module(oracle_mod, [0, 1], [0, 0], adc=[0, 0], cut=1)
    assert res["n_clusters"] == 0
    np.testing.assert_array_equal(res["digi"], [-1, -1])
    empty = synth.from_pixels([], [], [], n_modules=10)
    res = oracle_mod.cluster_event(empty)
    assert res["status"] == 0 and res["n_clusters"] == 0


def test_errors_and_precedence(oracle_mod):
    base = synth.from_pixels([0, 0, 1], [1, 2, 3], [1, 1, 1], n_modules=2)

    def mut(**kw):
        ev = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in base.items()}
        for k, (i, val) in kw.items():
            ev[k][i] = val
        return ev

    assert oracle_mod.cluster_event(base)["status"] == 0
    assert oracle_mod.cluster_event(mut(row=(0, 160)))["status"] == oracle_mod.E_RANGE
    assert oracle_mod.cluster_event(mut(col=(2, 416)))["status"] == oracle_mod.E_RANGE
    assert oracle_mod.cluster_event(mut(module=(2, 2)))["status"] == oracle_mod.E_RANGE
    assert oracle_mod.cluster_event(mut(module=(0, 1)))["status"] == oracle_mod.E_ORDER
    dup = mut(row=(1, int(base["row"][0])), col=(1, int(base["col"][0])))
    assert oracle_mod.cluster_event(dup)["status"] == oracle_mod.E_DUP
    both = mut(module=(0, 1), row=(2, 170))
    assert oracle_mod.cluster_event(both)["status"] == oracle_mod.E_RANGE


def _invariants(ev, comp, cut_res, cut):
    m, r, c = (ev[k].astype(np.int64) for k in ("module", "row", "col"))
    adc = ev["adc"].astype(np.int64)
    lin = m * PIX + c * ROWS + r
    ids = comp["digi"].astype(np.int64)
    assert (ids >= 0).all(), "every digi is labelled"
    pos = {int(x): i for i, x in enumerate(lin)}
    for i in range(lin.size):
        for dr in (-1, 0, 1):
            for dc in (-1, 0, 1):
                rr, cc = r[i] + dr, c[i] + dc
                if 0 <= rr < ROWS and 0 <= cc < COLS:
                    j = pos.get(int(m[i] * PIX + cc * ROWS + rr))
                    if j is not None:
                        assert ids[j] == ids[i], "8-neighbours share a label"
    assert (ids <= lin).all()
    assert set(ids.tolist()) <= set(lin.tolist()), "each id is a member's linear index"
    assert int(comp["size"].sum()) == lin.size
    assert int(comp["charge"].astype(np.int64).sum()) == int(adc.sum())
    kept = cut_res["charge"].astype(np.int64)
    assert (kept >= cut).all()
    lost = adc[cut_res["digi"] < 0].sum()
    assert int(kept.sum()) + int(lost) == int(adc.sum())
    assert np.all(np.diff(cut_res["id"].astype(np.int64)) > 0), "ascending ids"


@pytest.mark.parametrize("maker,idx", [(synth.plain_event, 0), (synth.async_event, 0),
                                       (synth.batch_event, 1)])
def test_invariants_synthetic(oracle_mod, maker, idx):
    ev = maker(idx)
    comp = oracle_mod.components(ev)
    res = oracle_mod.cluster_event(ev, 2000)
    assert comp["status"] == 0 and res["status"] == 0
    _invariants(ev, comp, res, 2000)


def test_permutation_and_translation(oracle_mod):
    ev = synth.plain_event(3, n_modules=8)
    res = oracle_mod.cluster_event(ev)
    rng = np.random.default_rng(5)
    # shuffle within modules: per-digi ids follow their digis, cluster arrays unchanged
    m = ev["module"].astype(np.int64)
    perm = np.argsort(m * 10**7 + rng.permutation(m.size), kind="stable")
    ev2 = {k: (v[perm] if isinstance(v, np.ndarray) else v) for k, v in ev.items()}
    res2 = oracle_mod.cluster_event(ev2)
    np.testing.assert_array_equal(res2["digi"], res["digi"][perm])
    for k in ("id", "charge", "size"):
        np.testing.assert_array_equal(res2[k], res[k])
    # translation without clipping shifts ids by dc*160 + dr
    r, c = ev["row"].astype(np.int64), ev["col"].astype(np.int64)
    sel = (r < ROWS - 3) & (c < COLS - 2)
    sub = {k: (v[sel] if isinstance(v, np.ndarray) else v) for k, v in ev.items()}
    a = oracle_mod.components(sub)
    moved = dict(sub)
    moved["row"] = (sub["row"] + 3).astype(np.uint16)
    moved["col"] = (sub["col"] + 2).astype(np.uint16)
    b = oracle_mod.components(moved)
    np.testing.assert_array_equal(b["digi"], a["digi"] + 2 * ROWS + 3)


def test_random_small_vs_pairwise(oracle_mod):
    rng = np.random.default_rng(11)
    for trial in range(60):
        nm = int(rng.integers(1, 4))
        n = int(rng.integers(0, 60))
        # a small window so that clusters touch often; unique pixels
        m = rng.integers(0, nm, n)
        r = rng.integers(0, 8, n) + (0 if trial % 2 else 152)
        c = rng.integers(0, 8, n) + (0 if trial % 3 else 408)
        key = np.unique((m * ROWS + r) * COLS + c)
        m, r, c = key // (ROWS * COLS), (key // COLS) % ROWS, key % COLS
        ev = synth.from_pixels(m, r, c, n_modules=nm, seed=trial)
        cut = int(rng.integers(0, 6000))
        ids, kept = brute.pairwise_components(ev["module"], ev["row"], ev["col"], ev["adc"], cut)
        res = oracle_mod.cluster_event(ev, cut)
        np.testing.assert_array_equal(res["digi"], ids)
        assert [tuple(x) for x in zip(res["id"].tolist(), res["charge"].tolist(), res["size"].tolist())] == kept


def test_golden_hand_derived(oracle_mod):
    from tests import golden_cases
    cases = golden_cases.load()
    assert len(cases) == 4
    for name, ev, cut, digi, kept in cases:
        res = oracle_mod.cluster_event(ev, cut)
        assert res["status"] == 0, name
        np.testing.assert_array_equal(res["digi"], digi, err_msg=name)
        np.testing.assert_array_equal(res["id"], kept[:, 0], err_msg=name)
        np.testing.assert_array_equal(res["charge"], kept[:, 1], err_msg=name)
        np.testing.assert_array_equal(res["size"], kept[:, 2], err_msg=name)
