"""Pins of the oracle's hits (the charge-weighted centroid of every kept cluster):
closed forms evaluated with exact rationals, and an independent implementation from
scipy.ndimage.label with numpy weighted sums on whole modules.  Expected floats are
the exact quotient rounded to double and then to float32, the same two roundings the
definition prescribes, so comparisons are bit-exact."""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest
from scipy import ndimage

from paper_2004_04334_amd import synth

ROWS, COLS = 160, 416


def _f32(q: Fraction) -> np.float32:
    return np.float32(float(q))           # float(Fraction) is the correctly rounded double


def _event(pix, adc, n_modules=1):
    m = np.array([p[0] for p in pix])
    r = np.array([p[1] for p in pix])
    c = np.array([p[2] for p in pix])
    return synth.from_pixels(m, r, c, adc=np.array(adc), n_modules=n_modules, seed=1)


def test_single_pixel_is_its_own_hit(oracle_mod):
    for (r, c) in [(0, 0), (159, 415), (37, 201)]:
        h = oracle_mod.hits(_event([(0, r, c)], [2500]), 2000)
        assert h["n_clusters"] == 1 and h["x"][0] == np.float32(c) and h["y"][0] == np.float32(r)


def test_two_pixels_weighted(oracle_mod):
    # (r, c) with adc a and (r+1, c+1) with adc b: x = c + b/(a+b), y = r + b/(a+b)
    for (r, c, a, b) in [(10, 20, 1000, 3000), (100, 7, 1234, 999), (0, 414, 4000, 100)]:
        h = oracle_mod.hits(_event([(0, r, c), (0, r + 1, c + 1)], [a, b]), 2000)
        assert h["n_clusters"] == 1
        assert h["x"][0] == _f32(Fraction(a * c + b * (c + 1), a + b))
        assert h["y"][0] == _f32(Fraction(a * r + b * (r + 1), a + b))
        assert h["x"][0] != h["y"][0]        # a swap of the axes would show


def test_cut_clusters_have_no_hit_and_zero_charge_is_nan(oracle_mod):
    ev = _event([(0, 5, 5), (0, 50, 50), (0, 51, 50)], [3000, 0, 0])
    h = oracle_mod.hits(ev, 2000)
    assert h["n_clusters"] == 1 and h["x"][0] == 5.0
    h0 = oracle_mod.hits(ev, 0)
    assert h0["n_clusters"] == 2 and np.isnan(h0["x"][1]) and np.isnan(h0["y"][1])


@pytest.mark.parametrize("occ", [0.005, 0.05, 0.5])
def test_against_scipy_label(oracle_mod, occ):
    rng = np.random.default_rng(int(occ * 1000))
    fired = rng.random((ROWS, COLS)) < occ
    r, c = np.nonzero(fired)
    adc = rng.integers(100, 4001, r.size)
    ev = synth.from_pixels(np.full(r.size, 2), r, c, adc=adc, n_modules=3, seed=2)
    lab, nlab = ndimage.label(fired, structure=np.ones((3, 3), dtype=int))
    grid_adc = np.zeros((ROWS, COLS), dtype=np.int64)
    grid_adc[r, c] = adc
    rr, cc = np.nonzero(fired)
    ll = lab[rr, cc]
    w = grid_adc[rr, cc]
    charge = np.bincount(ll, weights=w, minlength=nlab + 1).astype(np.int64)
    # exact integer sums (well below 2**53, so float64 bincount sums are exact)
    sx = np.bincount(ll, weights=w * cc, minlength=nlab + 1).astype(np.int64)
    sy = np.bincount(ll, weights=w * rr, minlength=nlab + 1).astype(np.int64)
    lin = 2 * ROWS * COLS + cc * ROWS + rr
    minlin = np.full(nlab + 1, np.iinfo(np.int64).max)
    np.minimum.at(minlin, ll, lin)
    keep = [k for k in range(1, nlab + 1) if charge[k] >= 2000]
    keep.sort(key=lambda k: minlin[k])
    ex = np.array([np.float32(sx[k] / charge[k]) for k in keep], dtype=np.float32)
    ey = np.array([np.float32(sy[k] / charge[k]) for k in keep], dtype=np.float32)
    h = oracle_mod.hits(ev, 2000)
    assert h["status"] == 0 and h["n_clusters"] == len(keep)
    assert np.array_equal(h["id"], minlin[keep].astype(np.int32))
    assert np.array_equal(h["x"], ex) and np.array_equal(h["y"], ey)


def test_hits_on_synthetic_events(oracle_mod):
    """Every hit lies inside its cluster's bounding box, and the clustering part is
    the plain oracle's."""
    ev = synth.async_event(3)
    h = oracle_mod.hits(ev, 2000)
    base = oracle_mod.cluster_event(ev, 2000)
    for k in ("id", "charge", "size", "digi"):
        assert np.array_equal(h[k], base[k])
    col = ev["col"].astype(np.int64)
    row = ev["row"].astype(np.int64)
    for i, cid in enumerate(h["id"][:200]):
        sel = h["digi"] == cid
        assert col[sel].min() <= h["x"][i] <= col[sel].max()
        assert row[sel].min() <= h["y"][i] <= row[sel].max()


def test_large_clusters_exact(oracle_mod):
    """Fully fired modules (one cluster of 66,560 pixels, sums near 3e10): the hit is
    the exact quotient rounded to double and then to float, which a division in
    single precision would miss."""
    rr, cc = np.meshgrid(np.arange(ROWS), np.arange(COLS), indexing="ij")
    rr, cc = rr.ravel(), cc.ravel()
    for seed in range(6):
        adc = np.random.default_rng(seed).integers(100, 4001, rr.size)
        ev = synth.from_pixels(np.zeros(rr.size, np.int64), rr, cc, adc=adc, n_modules=1, seed=seed)
        h = oracle_mod.hits(ev, 2000)
        a = ev["adc"].astype(np.int64)
        q = int(a.sum())
        assert h["n_clusters"] == 1
        assert h["x"][0] == _f32(Fraction(int((a * ev["col"].astype(np.int64)).sum()), q))
        assert h["y"][0] == _f32(Fraction(int((a * ev["row"].astype(np.int64)).sum()), q))
