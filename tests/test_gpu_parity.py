"""Device path vs the CPU oracle, bit-exact (integer work: ids, charges, sizes,
per-digi ids, counts and status must all be identical)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2004_04334_amd import synth
from tests import brute
from tests.gpu_util import compare, run_events

pytestmark = pytest.mark.gpu

CONFIGS = [(64, 1), (128, 1), (128, 2), (256, 1), (256, 2), (256, 4), (512, 1), (512, 2), (512, 4)]


@pytest.fixture(scope="module")
def px():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_04334_amd import pxcl
    pxcl.lib()
    oracle.build()
    return pxcl


def _ctx(px, n_modules, cut=2000):
    return px.Context(n_modules, cut, 0)


def test_plain_events(px):
    evs = [synth.plain_event(i) for i in range(3)]
    ctx = _ctx(px, 64)
    for i, (e, r) in enumerate(zip(evs, run_events(px, ctx, evs))):
        compare(r, oracle.cluster_event(e, 2000), f"plain {i}")
    ctx.close()


@pytest.mark.parametrize("wg,mpw", CONFIGS)
def test_kernel_configs(px, wg, mpw):
    print(f"config wg={wg} mpw={mpw}", flush=True)
    evs = [synth.plain_event(5), synth.async_event(2), synth.batch_event(3)]
    ctx = _ctx(px, 1856)
    ctx.set_kernel_config(wg, mpw)
    evs[0]["n_modules"] = 1856
    for i, (e, r) in enumerate(zip(evs, run_events(px, ctx, evs))):
        compare(r, oracle.cluster_event(e, 2000), f"cfg {wg}x{mpw} ev {i}")
    ctx.close()


def _pattern_events(R, C, r0, c0, chunk=16384, seed=0, total=None):
    codes = np.arange(total if total is not None else 1 << (R * C))
    rng = np.random.default_rng(seed)
    return [brute.patterns_event(codes[k:k + chunk], R, C, r0, c0, rng)[0] for k in range(0, codes.size, chunk)]


@pytest.mark.parametrize("r0,c0", [(0, 0), (156, 412), (0, 412), (156, 0), (78, 200), (30, 31)])
def test_exhaustive_4x4_embedded(px, r0, c0):
    print(f"4x4 at ({r0},{c0})", flush=True)
    evs = _pattern_events(4, 4, r0, c0, seed=r0 * 1000 + c0)
    ctx = _ctx(px, 16384, cut=3000)
    for i, (e, r) in enumerate(zip(evs, run_events(px, ctx, evs))):
        compare(r, oracle.cluster_event(e, 3000), f"4x4 ({r0},{c0}) chunk {i}")
    ctx.close()


@pytest.mark.parametrize("R,C,r0,c0", [(4, 5, 0, 0), (5, 4, 155, 412), (4, 5, 61, 207)])
def test_exhaustive_4x5_5x4_embedded(px, R, C, r0, c0):
    print(f"{R}x{C} at ({r0},{c0})", flush=True)
    evs = _pattern_events(R, C, r0, c0, seed=R * 7 + c0)
    ctx = _ctx(px, 16384, cut=2000)
    ctx.set_kernel_config(64, 1)
    for i, e in enumerate(evs):
        (r,) = run_events(px, ctx, [e])
        compare(r, oracle.cluster_event(e, 2000), f"{R}x{C} chunk {i}")
    ctx.close()


def _closed_form_event():
    rr, cc = np.meshgrid(np.arange(160), np.arange(416), indexing="ij")
    mods, rows, cols = [], [], []

    def add(m, r, c):
        mods.append(np.full(np.size(r), m)); rows.append(np.ravel(r)); cols.append(np.ravel(c))

    add(0, *synth.column_track(0))
    add(1, *synth.column_track(415))
    k = np.arange(160)
    add(2, k, k)
    add(3, k, 415 - k)
    sel = (rr + cc) % 2 == 0
    add(4, rr[sel], cc[sel])                       # checkerboard: one cluster of 33,280
    sel = (rr % 2 == 0) & (cc % 2 == 0)
    add(5, rr[sel], cc[sel])                       # lattice: 16,640 singletons
    add(6, *synth.serpentine(True))
    add(7, *synth.serpentine(False))
    add(8, rr.ravel(), cc.ravel())                 # fully fired module
    add(9, np.array([40, 41]), np.array([415, 0]))
    add(10, np.array([159]), np.array([33]))
    add(11, np.array([0]), np.array([33]))
    add(12, np.array([10, 11, 50]), np.array([10, 12, 60]))
    return synth.from_pixels(np.concatenate(mods), np.concatenate(rows), np.concatenate(cols),
                             n_modules=13, seed=4)


@pytest.mark.parametrize("wg,mpw", [(256, 1), (64, 1), (512, 4)])
def test_closed_forms(px, wg, mpw):
    ev = _closed_form_event()
    ctx = _ctx(px, 13, cut=0)
    ctx.set_kernel_config(wg, mpw)
    (r,) = run_events(px, ctx, [ev])
    ref = oracle.cluster_event(ev, 0)
    compare(r, ref, "closed forms")
    # spot-check the closed forms themselves
    ids = set(r["id"].tolist())
    assert 4 * 66560 in ids and 6 * 66560 in ids and 7 * 66560 in ids and 8 * 66560 in ids
    sizes = dict(zip(r["id"].tolist(), r["size"].tolist()))
    assert sizes[4 * 66560] == 33280 and sizes[6 * 66560] == 33359
    assert sizes[7 * 66560] == 33487 and sizes[8 * 66560] == 66560
    ctx.close()


def test_cut_boundary_and_adc_zero(px):
    ev = synth.from_pixels([0, 0, 0, 0, 0, 1, 1], [5, 6, 50, 51, 100, 3, 4], [5, 5, 60, 60, 300, 9, 9],
                           adc=[999, 1000, 1000, 1000, 2001, 0, 0], n_modules=2)
    ctx = _ctx(px, 2, cut=2000)
    (r,) = run_events(px, ctx, [ev])
    compare(r, oracle.cluster_event(ev, 2000), "cut boundary")
    assert r["charge"].tolist() == [2000, 2001]
    ctx.close()
    ctx = _ctx(px, 2, cut=0)
    (r,) = run_events(px, ctx, [ev])
    compare(r, oracle.cluster_event(ev, 0), "adc zero")
    ctx.close()


def test_golden_hand_derived(px):
    from tests import golden_cases
    for name, ev, cut, digi, kept in golden_cases.load():
        ctx = _ctx(px, ev["n_modules"], cut=cut)
        (r,) = run_events(px, ctx, [ev])
        assert r["status"] == 0
        np.testing.assert_array_equal(r["digi"], digi, err_msg=name)
        np.testing.assert_array_equal(r["id"], kept[:, 0], err_msg=name)
        np.testing.assert_array_equal(r["charge"], kept[:, 1], err_msg=name)
        np.testing.assert_array_equal(r["size"], kept[:, 2], err_msg=name)
        ctx.close()


def test_empty_event(px):
    ctx = _ctx(px, 10)
    ev = synth.from_pixels([], [], [], n_modules=10)
    (r,) = run_events(px, ctx, [ev])
    assert r["status"] == 0 and r["n_clusters"] == 0
    ctx.close()


def test_host_pinned_input(px):
    evs = [synth.async_event(7), synth.plain_event(2)]
    evs[1]["n_modules"] = 1856
    ctx = _ctx(px, 1856)
    for i, (e, r) in enumerate(zip(evs, run_events(px, ctx, evs, where="pinned"))):
        compare(r, oracle.cluster_event(e, 2000), f"pinned {i}")
    ctx.close()


def test_errors(px):
    base = synth.plain_event(1, n_modules=4)

    def mut(**kw):
        ev = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in base.items()}
        for k, (i, val) in kw.items():
            ev[k][i] = val
        return ev

    n = base["module"].size
    cases = {
        "row": mut(row=(5, 160)),
        "col": mut(col=(n - 1, 416)),
        "module": mut(module=(n - 1, 4)),
        "order": mut(module=(0, 1)),
        "dup": mut(row=(1, int(base["row"][0])), col=(1, int(base["col"][0]))),
        "both": mut(module=(0, 1), row=(7, 300)),
    }
    ctx = _ctx(px, 4)
    slot = px.Event(ctx, n)
    for name, ev in cases.items():
        print(f"error case {name}", flush=True)
        (r,) = run_events(px, ctx, [ev], slots=[slot])
        ref = oracle.cluster_event(ev, 2000)
        assert ref["status"] != 0
        assert r["status"] == ref["status"], name
        # the next valid event on the same slot is unaffected
        (r2,) = run_events(px, ctx, [base], slots=[slot])
        compare(r2, oracle.cluster_event(base, 2000), f"after {name}")
    slot.close()
    ctx.close()


def test_size_hint(px):
    """max_module_digis: a bound at most the small kernel's capacity (2,048 digis for
    256-thread groups) skips the big-module kernel.  Results are exact when the bound
    holds or is absent; a module above a wrong bound fails the event with E_HINT
    rather than losing clusters silently, and the slot stays usable."""
    lin = (np.arange(3000) * 37) % (160 * 416)
    big = synth.from_pixels(np.concatenate([np.zeros(40, np.int64), np.full(3000, 3)]),
                            np.concatenate([np.arange(40) * 3 % 160, lin % 160]),
                            np.concatenate([np.arange(40) * 5 % 416, lin // 160]), n_modules=8, seed=4)
    small = synth.plain_event(3, n_modules=8)
    ctx = _ctx(px, 8)
    ctx.set_kernel_config(256, 1)
    slot = px.Event(ctx, max(big["module"].size, small["module"].size))

    def run(ev, digis):
        px.acquire(slot, digis)
        px.wait(slot)
        return px.produce(slot).numpy()

    d = px.Digis.from_numpy(big, "cuda", hint=True)
    assert d.max_module_digis == 3000
    compare(run(big, d), oracle.cluster_event(big, 2000), "hint above capacity")
    compare(run(big, px.Digis.from_numpy(big, "cuda", hint=False)), oracle.cluster_event(big, 2000), "no hint")
    d.max_module_digis = 100
    r = run(big, d)
    assert r["status"] == px.E_HINT and r["n_clusters"] <= big["module"].size
    ds = px.Digis.from_numpy(small, "cuda", hint=True)
    assert 0 < ds.max_module_digis <= 2048
    compare(run(small, ds), oracle.cluster_event(small, 2000), "hint within capacity")
    slot.close()
    ctx.close()


def test_size_hint_scratch_mode(px):
    """A bound of at most 16,384 digis skips the scratch-mode kernel; a module above a
    wrong bound (20,000 digis under a bound of 16,384) fails the event with E_HINT, and
    with a right bound or none the scratch kernel clusters it exactly."""
    lin = (np.arange(20000) * 37) % (160 * 416)
    ev = synth.from_pixels(np.concatenate([np.zeros(50, np.int64), np.full(20000, 2)]),
                           np.concatenate([np.arange(50) * 3 % 160, lin % 160]),
                           np.concatenate([np.arange(50) * 7 % 416, lin // 160]), n_modules=4, seed=6)
    ref = oracle.cluster_event(ev, 2000)
    ctx = _ctx(px, 4)
    slot = px.Event(ctx, ev["module"].size)
    for name, hint in [("right bound", 20000), ("no bound", None), ("wrong bound", 16384)]:
        d = px.Digis.from_numpy(ev, "cuda", hint=hint is not None)
        if hint is not None:
            d.max_module_digis = hint
        print(f"scratch hint: {name}", flush=True)
        px.acquire(slot, d)
        px.wait(slot)
        r = px.produce(slot).numpy()
        if name == "wrong bound":
            assert r["status"] == px.E_HINT and r["n_clusters"] <= ev["module"].size
        else:
            compare(r, ref, name)
    slot.close()
    ctx.close()


def test_full_size_async_and_stress(px):
    """Full-size events of the asynchronous and the stress configurations."""
    ctx = _ctx(px, 1856)
    evs = [synth.async_event(11), synth.stress_event(0), synth.stress_event(1)]
    for i, (e, r) in enumerate(zip(evs, run_events(px, ctx, evs))):
        compare(r, oracle.cluster_event(e, 2000), f"full {i}")
    ctx.close()
