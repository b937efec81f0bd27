"""The pins are strong enough: plausible mistakes planted in a *copy* of the C oracle
(built on the CPU into a temporary library) must each fail at least one pin."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests import test_oracle_any_order as apins
from tests import test_oracle_hits as hpins
from tests import test_oracle_pins as pins

MUTANTS = {
    "four_connectivity": ("if ((dr == 0 && dc == 0) ||", "if ((dr == 0 && dc == 0) || (dr != 0 && dc != 0) ||"),
    "row_major_id": ("(int64_t)col[d] * O_ROWS + row[d]", "(int64_t)row[d] * O_COLS + col[d]"),
    "strict_cut": ("(c->charge >= charge_cut)", "(c->charge > charge_cut)"),
    "dropped_charge_term": ("charge += adc[d];", "if (head > 1) charge += adc[d];"),
    "modules_not_separated": ("for (uint32_t i = s; i < e; ++i) grid[row[i] * O_COLS + col[i]] = -1;", ""),
    "descending_order": ("return (x > y) - (x < y);", "return (x < y) - (x > y);"),
    "max_instead_of_min_id": ("if (lin < min_lin) min_lin = lin;", "if (min_lin == INT64_MAX || lin > min_lin) min_lin = lin;"),
    # hits
    "unweighted_hit": ("sum_col += (uint64_t)adc[d] * col[d];", "sum_col += (uint64_t)col[d] * 3000u;"),
    "hit_axes_swapped": ("sum_row += (uint64_t)adc[d] * row[d];", "sum_row += (uint64_t)adc[d] * col[d];"),
    "hit_in_float": ("(float)((double)cls[j].sum_col / (double)cls[j].charge)",
                     "((float)cls[j].sum_col / (float)cls[j].charge)"),
    # digis in any order
    "any_order_ids_not_returned_to_input_positions": ("digi_cluster[pos[j]] = gd[j];", "digi_cluster[j] = gd[j];"),
    "any_order_rows_not_gathered": ("gr[j] = row[pos[j]];", "gr[j] = row[j];"),
}


class _Fake:
    """Stands in for the ``oracle`` module with a mutant library loaded."""

    def __init__(self, lib):
        self._lib = lib
        self.E_DUP, self.E_RANGE, self.E_ORDER = oracle.E_DUP, oracle.E_RANGE, oracle.E_ORDER

    def cluster_event(self, ev, charge_cut=2000, any_order=False):
        saved = oracle._lib
        oracle._lib = self._lib
        try:
            return oracle.cluster_event(ev, charge_cut, any_order=any_order)
        finally:
            oracle._lib = saved

    def components(self, ev):
        return self.cluster_event(ev, 0)

    def hits(self, ev, charge_cut=2000):
        saved = oracle._lib
        oracle._lib = self._lib
        try:
            return oracle.hits(ev, charge_cut)
        finally:
            oracle._lib = saved


def _build_mutant(tmp_path, name, old, new):
    src = open(oracle._SRC).read()
    assert old in src, name
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", str(so), str(path)])
    lib = ctypes.CDLL(str(so))
    u16p, i32p, u32p = (ctypes.POINTER(t) for t in (ctypes.c_uint16, ctypes.c_int32, ctypes.c_uint32))
    lib.pxo_cluster_event.restype = ctypes.c_int
    lib.pxo_cluster_event.argtypes = [u16p, u16p, u16p, u16p, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_uint32, i32p, i32p, i32p, i32p, u32p, u32p]
    lib.pxo_cluster_event_hits.restype = ctypes.c_int
    lib.pxo_cluster_event_hits.argtypes = lib.pxo_cluster_event.argtypes + [ctypes.POINTER(ctypes.c_float)] * 2
    lib.pxo_cluster_event_any_order.restype = ctypes.c_int
    lib.pxo_cluster_event_any_order.argtypes = lib.pxo_cluster_event_hits.argtypes
    return lib


def _caught(fake):
    checks = [
        lambda: pins._check_patterns(fake, np.arange(4096), 4, 4, 0, 0, 1, 0),
        lambda: pins._check_patterns(fake, np.arange(4096), 4, 4, 156, 412, 2, 3000),
        lambda: pins.test_closed_form_cut_boundary(fake),
        lambda: pins.test_closed_form_no_wraparound(fake),
        lambda: pins.test_closed_form_column_track(fake, 207),
        lambda: pins.test_random_small_vs_pairwise(fake),
        lambda: hpins.test_two_pixels_weighted(fake),
        lambda: hpins.test_against_scipy_label(fake, 0.05),
        lambda: hpins.test_against_scipy_label(fake, 0.5),
        lambda: hpins.test_large_clusters_exact(fake),          # sums above 2**24
        lambda: apins.test_patterns_shuffled_across_modules(fake),
        lambda: apins.test_random_small_shuffled_vs_pairwise(fake),
    ]
    for chk in checks:
        try:
            chk()
        except AssertionError:
            return True
    return False


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    fake = _Fake(_build_mutant(tmp_path, name, old, new))
    assert _caught(fake), f"mutant {name} survived the pins"


def test_unmutated_passes(tmp_path):
    fake = _Fake(_build_mutant(tmp_path, "identity", "#include <stdint.h>", "#include <stdint.h>"))
    assert not _caught(fake)
