"""The seeded generators produce the workloads they claim (shape, uniqueness, order)."""
import numpy as np
import pytest

from paper_2004_04334_amd import synth


def _valid(ev):
    m, r, c = (ev[k].astype(np.int64) for k in ("module", "row", "col"))
    assert (np.diff(m) >= 0).all()
    assert (m < ev["n_modules"]).all() and (r < 160).all() and (c < 416).all()
    key = (m * 160 + r) * 416 + c
    assert np.unique(key).size == key.size
    a = ev["adc"]
    assert a.min() >= 100 and a.max() <= 4000


def test_reproducible():
    a, b = synth.async_event(4), synth.async_event(4)
    for k in ("module", "row", "col", "adc"):
        np.testing.assert_array_equal(a[k], b[k])
    c = synth.async_event(5)
    assert a["module"].size != c["module"].size or not np.array_equal(a["row"], c["row"])


def test_plain_shape():
    ev = synth.plain_event(0)
    _valid(ev)
    assert ev["module"].size == 46912 and ev["n_modules"] == 64
    assert (np.bincount(ev["module"]) == 733).all()


def test_async_shape():
    ev = synth.async_event(0)
    _valid(ev)
    assert 48000 < ev["module"].size < 52000 and ev["n_modules"] == 1856


@pytest.mark.parametrize("i", [0, 1, 2])
def test_batch_and_serve_sizes(i):
    ev = synth.batch_event(i)
    _valid(ev)
    assert 10_000 <= ev["module"].size <= 120_000
    ev = synth.serve_event(i)
    _valid(ev)
    assert 10_000 <= ev["module"].size <= 200_000


def test_stress_shape():
    ev = synth.stress_event(0)
    _valid(ev)
    assert np.unique(ev["module"]).size == 160
    assert 290_000 < ev["module"].size < 340_000
    counts = np.bincount(ev["module"])
    assert (counts == 13312).sum() == 16
    assert 33359 in counts.tolist() and 160 in counts.tolist()
    ev = synth.stress_event(1)
    assert 33487 in np.bincount(ev["module"]).tolist()


def test_stress_all_modules_hot_shape():
    """The literal reading of the stress configuration: 10 % of the 1,856 modules hot."""
    ev = synth.stress_all_event(0)
    _valid(ev)
    counts = np.bincount(ev["module"], minlength=1856)
    assert (counts == 13312).sum() == 186
    assert np.count_nonzero(counts) == 186 + 142 + 2
    assert 33359 in counts.tolist() and 160 in counts.tolist()
    assert 2_400_000 < ev["module"].size < 2_700_000


def test_elongated_along_columns():
    # row steps are 3x likelier than column steps, so clusters extend more in rows
    ev = synth.plain_event(1, n_modules=4)
    m, r, c = (ev[k].astype(np.int64) for k in ("module", "row", "col"))
    occ = {(a, b, d) for a, b, d in zip(m, r, c)}
    vert = sum(((a, b + 1, d) in occ) for a, b, d in occ)
    horiz = sum(((a, b, d + 1) in occ) for a, b, d in occ)
    assert vert > 1.5 * horiz
