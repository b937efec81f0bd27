"""CPU oracle for per-event pixel clustering -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the device library: the C oracle
(``ccl_oracle.c``, a breadth-first search over a dense per-module grid) is built
with ``gcc`` into ``liboracle.so`` beside it and called through ctypes.

The definition it implements (8-connected components per module, id = smallest
linear pixel index ``module*66560 + col*160 + row``, charge = sum of adc, size,
keep iff charge >= cut, clusters in ascending id, per-digi id or -1) fills the role
of the "ClusterProducer" of the paper's Figure 1 (Sec. 3); the paper gives no
formula, so the definition is the textbook one stated in ``ccl_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ccl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_DUP, E_RANGE, E_ORDER = 0, -5, -6, -7
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle (plain gcc -O2, no vectorisation flags)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        u16p = ctypes.POINTER(ctypes.c_uint16)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lib.pxo_cluster_event.restype = ctypes.c_int
        lib.pxo_cluster_event.argtypes = [u16p, u16p, u16p, u16p, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_uint32, i32p, i32p, i32p, i32p, u32p, u32p]
        f32p = ctypes.POINTER(ctypes.c_float)
        lib.pxo_cluster_event_hits.restype = ctypes.c_int
        lib.pxo_cluster_event_hits.argtypes = lib.pxo_cluster_event.argtypes + [f32p, f32p]
        lib.pxo_cluster_event_any_order.restype = ctypes.c_int
        lib.pxo_cluster_event_any_order.argtypes = lib.pxo_cluster_event_hits.argtypes
        _lib = lib
    return _lib


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def cluster_event(ev, charge_cut: int = 2000, any_order: bool = False):
    """Run the oracle on one event (dict of uint16 arrays + ``n_modules``).

    Returns a dict: ``status``, ``err_bits``, ``n_clusters``, ``id``, ``charge``,
    ``size`` (int32 arrays of the kept clusters, ascending id) and ``digi`` (int32
    per digi: kept cluster id or -1).  With ``any_order`` the digis need not be
    grouped by module (``pxo_cluster_event_any_order``).
    """
    if any_order:
        r = hits(ev, charge_cut, any_order=True)
        del r["x"], r["y"]
        return r
    lib = _load()
    mod = np.ascontiguousarray(ev["module"], dtype=np.uint16)
    row = np.ascontiguousarray(ev["row"], dtype=np.uint16)
    col = np.ascontiguousarray(ev["col"], dtype=np.uint16)
    adc = np.ascontiguousarray(ev["adc"], dtype=np.uint16)
    n = mod.size
    cap = max(n, 1)
    digi = np.full(cap, -1, dtype=np.int32)
    cid = np.zeros(cap, dtype=np.int32)
    chg = np.zeros(cap, dtype=np.int32)
    siz = np.zeros(cap, dtype=np.int32)
    ncl = np.zeros(1, dtype=np.uint32)
    bits = np.zeros(1, dtype=np.uint32)
    st = lib.pxo_cluster_event(_p(mod, ctypes.c_uint16), _p(row, ctypes.c_uint16),
                               _p(col, ctypes.c_uint16), _p(adc, ctypes.c_uint16),
                               n, int(ev["n_modules"]), int(charge_cut) & 0xFFFFFFFF,
                               _p(digi, ctypes.c_int32), _p(cid, ctypes.c_int32),
                               _p(chg, ctypes.c_int32), _p(siz, ctypes.c_int32),
                               _p(ncl, ctypes.c_uint32), _p(bits, ctypes.c_uint32))
    k = int(ncl[0])
    return {"status": int(st), "err_bits": int(bits[0]), "n_clusters": k,
            "id": cid[:k].copy(), "charge": chg[:k].copy(), "size": siz[:k].copy(),
            "digi": digi[:n].copy()}


def hits(ev, charge_cut: int = 2000, any_order: bool = False):
    """The clustering result plus, per kept cluster, its hit: the charge-weighted
    centroid x = sum(adc*col)/charge, y = sum(adc*row)/charge (exact 64-bit sums,
    divided in double, rounded to float32; NaN for zero charge).  With ``any_order``
    the digis need not be grouped by module."""
    lib = _load()
    mod = np.ascontiguousarray(ev["module"], dtype=np.uint16)
    row = np.ascontiguousarray(ev["row"], dtype=np.uint16)
    col = np.ascontiguousarray(ev["col"], dtype=np.uint16)
    adc = np.ascontiguousarray(ev["adc"], dtype=np.uint16)
    n = mod.size
    cap = max(n, 1)
    digi = np.full(cap, -1, dtype=np.int32)
    cid, chg, siz = (np.zeros(cap, dtype=np.int32) for _ in range(3))
    hx, hy = np.zeros(cap, dtype=np.float32), np.zeros(cap, dtype=np.float32)
    ncl = np.zeros(1, dtype=np.uint32)
    bits = np.zeros(1, dtype=np.uint32)
    fn = lib.pxo_cluster_event_any_order if any_order else lib.pxo_cluster_event_hits
    st = fn(_p(mod, ctypes.c_uint16), _p(row, ctypes.c_uint16),
                                    _p(col, ctypes.c_uint16), _p(adc, ctypes.c_uint16),
                                    n, int(ev["n_modules"]), int(charge_cut) & 0xFFFFFFFF,
                                    _p(digi, ctypes.c_int32), _p(cid, ctypes.c_int32),
                                    _p(chg, ctypes.c_int32), _p(siz, ctypes.c_int32),
                                    _p(ncl, ctypes.c_uint32), _p(bits, ctypes.c_uint32),
                                    _p(hx, ctypes.c_float), _p(hy, ctypes.c_float))
    k = int(ncl[0])
    return {"status": int(st), "err_bits": int(bits[0]), "n_clusters": k,
            "id": cid[:k].copy(), "charge": chg[:k].copy(), "size": siz[:k].copy(),
            "digi": digi[:n].copy(), "x": hx[:k].copy(), "y": hy[:k].copy()}


def components(ev):
    """All components before the cut (cut = 0 keeps every cluster)."""
    return cluster_event(ev, charge_cut=0)


def event_bytes(ev, result) -> int:
    """Algorithmic HBM bytes of one event: read 8 B/digi, write 4 B/digi,
    12 B/kept cluster, 4 B count."""
    return 8 * ev["module"].size + 4 * ev["module"].size + 12 * result["n_clusters"] + 4
