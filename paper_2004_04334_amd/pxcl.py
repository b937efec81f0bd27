"""Python binding of the HIP pixel-clustering library (``libpxcl.so``, C ABI in
``include/pxcl.h``).

Argument marshalling only: every step of the clustering runs in the library's
kernels.  PyTorch provides device memory (its caching allocator plays the role of
the memory pool the paper describes in Sec. 4.1) and streams.  The names follow the
External Worker split of the paper (Sec. 2): ``acquire(event, digis, stream,
done_cb)`` enqueues the device work and returns at once; ``done_cb(status)`` fires
once on completion; ``produce(event)`` returns the clusters as tensors that view the
event's workspace (valid until the next acquire on that event).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Callable, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpxcl.so")

OK, E_INVAL, E_CAPACITY, E_BUSY, E_NOT_READY = 0, -1, -2, -3, -4
E_DUP_PIXEL, E_RANGE, E_ORDER, E_HIP, E_INTERNAL, E_NOTFOUND, E_HINT = -5, -6, -7, -8, -10, -11, -12
WHERE_HOST, WHERE_DEVICE = 0, 1
DIGIS_ANY_ORDER, DIGIS_HITS, DIGIS_DEFER_BIG = 1, 2, 4
BATCH_GRAPH = 1
BATCH_DEFER_BIG = 2
MAX_BATCH = 128
ROWS, COLS, PIXELS_PER_MODULE = 160, 416, 66560


class PxclError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})" if what else f"{strerror(code)} ({code})")


class _Config(ctypes.Structure):
    _fields_ = [("n_modules", ctypes.c_uint32), ("charge_cut", ctypes.c_uint32)]


class _Digis(ctypes.Structure):
    _fields_ = [("module", ctypes.c_void_p), ("row", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("adc", ctypes.c_void_p), ("n", ctypes.c_uint32), ("where", ctypes.c_int32),
                ("max_module_digis", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class _Hits(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_hits", ctypes.c_uint32), ("x", ctypes.c_void_p),
                ("y", ctypes.c_void_p), ("stream", ctypes.c_void_p), ("done_event", ctypes.c_void_p),
                ("device", ctypes.c_int32)]


class _HostClusters(ctypes.Structure):
    _fields_ = [("id", ctypes.c_void_p), ("charge", ctypes.c_void_p), ("size", ctypes.c_void_p),
                ("digi_cluster", ctypes.c_void_p), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("capacity", ctypes.c_uint32), ("n_clusters", ctypes.c_uint32), ("status", ctypes.c_int32)]


class _Clusters(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("err_bits", ctypes.c_uint32), ("n_clusters", ctypes.c_uint32),
                ("n_digis", ctypes.c_uint32), ("id", ctypes.c_void_p), ("charge", ctypes.c_void_p),
                ("size", ctypes.c_void_p), ("digi_cluster", ctypes.c_void_p), ("stream", ctypes.c_void_p),
                ("done_event", ctypes.c_void_p), ("device", ctypes.c_int32)]


class _NoAllocOut(ctypes.Structure):
    _fields_ = [("digi_cluster", ctypes.c_void_p), ("id", ctypes.c_void_p), ("charge", ctypes.c_void_p),
                ("size", ctypes.c_void_p), ("status", ctypes.c_void_p)]


class Flag(ctypes.Structure):
    """Host word pair written by the library's ready-made callback ``pxcl_flag_cb``."""
    _fields_ = [("status", ctypes.c_int32), ("fired", ctypes.c_uint32)]


class RunStats(ctypes.Structure):
    _fields_ = [("wall_s", ctypes.c_double), ("events", ctypes.c_uint64), ("digis", ctypes.c_uint64),
                ("lat_p50_us", ctypes.c_double), ("lat_p99_us", ctypes.c_double), ("lat_max_us", ctypes.c_double),
                ("blocked_us_per_event", ctypes.c_double), ("cpu_tasks_per_s", ctypes.c_double),
                ("cpu_tasks", ctypes.c_uint64), ("errors", ctypes.c_uint32), ("max_inflight", ctypes.c_uint32),
                ("peak_resident_bytes", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("stage_p50_us", ctypes.c_double * 4), ("stage_p99_us", ctypes.c_double * 4),
                ("cpu_tasks_per_s_idle", ctypes.c_double), ("offered_per_s", ctypes.c_double)]

    def as_dict(self):
        out = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            out[k] = list(v) if isinstance(v, ctypes.Array) else v
        return out


class ServeOpts(ctypes.Structure):
    _fields_ = [("rate_hz", ctypes.c_double), ("n_requests", ctypes.c_uint32), ("budget_bytes", ctypes.c_uint64),
                ("n_slots", ctypes.c_uint32), ("max_batch", ctypes.c_uint32), ("n_cpu_threads", ctypes.c_uint32),
                ("cpu_task_ns", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("max_inflight", ctypes.c_uint32), ("batch_delay_us", ctypes.c_uint32)]


DONE_CB = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32)

_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "pxcl_ctx_create": (ctypes.c_int, [ctypes.POINTER(_Config), ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "pxcl_ctx_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "pxcl_set_kernel_config": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32]),
    "pxcl_get_kernel_config": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32),
                                              ctypes.POINTER(ctypes.c_uint32)]),
    "pxcl_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "pxcl_get_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_uint64), ctypes.c_int]),
    "pxcl_event_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_uint32]),
    "pxcl_event_pinned_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "pxcl_event_bind": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                       ctypes.c_size_t, ctypes.c_uint32, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_void_p)]),
    "pxcl_event_unbind": (ctypes.c_int, [ctypes.c_void_p]),
    "pxcl_event_capacity": (ctypes.c_uint32, [ctypes.c_void_p]),
    "pxcl_acquire": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Digis), ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]),
    "pxcl_query": (ctypes.c_int, [ctypes.c_void_p]),
    "pxcl_produce": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Clusters)]),
    "pxcl_wait": (ctypes.c_int, [ctypes.c_void_p]),
    "pxcl_flag_cb": (None, [ctypes.c_void_p, ctypes.c_int32]),
    "pxcl_hits_enqueue": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pxcl_hits_query": (ctypes.c_int, [ctypes.c_void_p]),
    "pxcl_hits_produce": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Hits)]),
    "pxcl_hits_wait": (ctypes.c_int, [ctypes.c_void_p]),
    "pxcl_copy_to_host": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_HostClusters),
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "pxcl_copy_query": (ctypes.c_int, [ctypes.c_void_p]),
    "pxcl_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_uint32]),
    "pxcl_batch_pinned_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_uint32]),
    "pxcl_batch_bind": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                       ctypes.c_size_t, ctypes.c_uint32, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_void_p)]),
    "pxcl_batch_unbind": (ctypes.c_int, [ctypes.c_void_p]),
    "pxcl_acquire_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(_Digis),
                                          ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_uint32]),
    "pxcl_batch_query": (ctypes.c_int, [ctypes.c_void_p]),
    "pxcl_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                     ctypes.POINTER(_Digis), ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint32,
                                     ctypes.c_char_p, ctypes.POINTER(ctypes.c_float)]),
    "pxcl_autotune_load": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_uint32]),
    "pxcl_run_async": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32, ctypes.POINTER(_Digis),
                                      ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                      ctypes.POINTER(RunStats), ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "pxcl_serve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                  ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                  ctypes.c_uint32, ctypes.POINTER(_Digis), ctypes.c_uint32,
                                  ctypes.POINTER(ServeOpts), ctypes.POINTER(RunStats),
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint32),
                                  ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "pxcl_cluster_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Digis), ctypes.POINTER(_NoAllocOut),
                                            ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32)]),
    "pxcl_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "pxcl_version": (ctypes.c_char_p, []),
}


def lib():
    """Load ``libpxcl.so``; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2004_04334_amd.build`")
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def strerror(code: int) -> str:
    return lib().pxcl_strerror(int(code)).decode()


def _check(code: int, what: str):
    if code != OK:
        raise PxclError(code, what)


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


FLAG_CB = None  # pxcl_flag_cb as a C function pointer, resolved on first use


def flag_cb_ptr() -> int:
    global FLAG_CB
    if FLAG_CB is None:
        FLAG_CB = ctypes.cast(lib().pxcl_flag_cb, ctypes.c_void_p).value
    return FLAG_CB


# ---------------------------------------------------------------------------
@dataclass
class Digis:
    """Digis of one event as four uint16 tensors (CUDA or pinned CPU), grouped by
    non-decreasing module, or in any order with ``any_order`` (the library then
    groups them on the device).  Keep the object alive until the done callback.
    max_module_digis: an upper bound on the digis of any one module, or 0 (unknown);
    a small bound lets the library skip its big-module kernel.  ``defer_big`` (single
    acquire only): the big-module kernels run in a second launch, queued by the
    library only if a module needs them; results are final at the callback."""
    module: torch.Tensor
    row: torch.Tensor
    col: torch.Tensor
    adc: torch.Tensor
    max_module_digis: int = 0
    any_order: bool = False
    hits: bool = False           # hits fused into the clustering
    defer_big: bool = False      # big-module kernels only when needed, in a second launch

    @property
    def n(self) -> int:
        return int(self.module.numel())

    @property
    def where(self) -> int:
        return WHERE_DEVICE if self.module.is_cuda else WHERE_HOST

    def struct(self) -> _Digis:
        ts = (self.module, self.row, self.col, self.adc)
        for t in ts:
            if t.dtype != torch.uint16 or not t.is_contiguous() or t.numel() != self.n:
                raise ValueError("digis must be contiguous uint16 tensors of equal length")
            if t.is_cuda != self.module.is_cuda or (not t.is_cuda and not t.is_pinned()):
                raise ValueError("digis must all be on the device or all in pinned host memory")
        return _Digis(*(t.data_ptr() if self.n else None for t in ts), self.n, self.where,
                      int(self.max_module_digis),
                      (DIGIS_ANY_ORDER if self.any_order else 0) | (DIGIS_HITS if self.hits else 0) |
                      (DIGIS_DEFER_BIG if self.defer_big else 0))

    @staticmethod
    def from_numpy(ev, device: str = "cuda", hint: bool = False, any_order: bool = False,
                   hits: bool = False, defer_big: bool = False) -> "Digis":
        """Copy a numpy event; with `hint`, the largest number of digis sharing a
        module id (a host-side count over the event) is passed as max_module_digis;
        with `any_order` the digis are flagged as being in any order."""
        ts = []
        for k in ("module", "row", "col", "adc"):
            t = torch.from_numpy(ev[k].astype("uint16", copy=True))
            if device == "cuda":
                t = t.to("cuda", non_blocking=False)
            elif device == "pinned":
                t = t.pin_memory()
            ts.append(t.contiguous())
        mx = int(np.bincount(ev["module"]).max()) if (hint and ev["module"].size) else 0
        return Digis(*ts, max_module_digis=mx, any_order=any_order, hits=hits, defer_big=defer_big)


@dataclass
class ClusterResult:
    status: int
    err_bits: int
    n_clusters: int
    id: torch.Tensor
    charge: torch.Tensor
    size: torch.Tensor
    digi_cluster: torch.Tensor
    stream: int
    done_event: int

    def numpy(self):
        return {"status": self.status, "err_bits": self.err_bits, "n_clusters": self.n_clusters,
                "id": self.id.cpu().numpy(), "charge": self.charge.cpu().numpy(),
                "size": self.size.cpu().numpy(), "digi": self.digi_cluster.cpu().numpy()}


class Context:
    def __init__(self, n_modules: int, charge_cut: int = 2000, device: int = 0):
        self._h = ctypes.c_void_p()
        cfg = _Config(int(n_modules), int(charge_cut))
        _check(lib().pxcl_ctx_create(ctypes.byref(cfg), int(device), ctypes.byref(self._h)), "ctx_create")
        self.n_modules, self.charge_cut, self.device = int(n_modules), int(charge_cut), int(device)

    @property
    def handle(self):
        return self._h

    def set_kernel_config(self, wg: int, mpw: int):
        _check(lib().pxcl_set_kernel_config(self._h, wg, mpw), "set_kernel_config")

    def kernel_config(self):
        a, b = ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().pxcl_get_kernel_config(self._h, ctypes.byref(a), ctypes.byref(b)), "get_kernel_config")
        return a.value, b.value

    def set_timing(self, enable, period: int = 1):
        """Time the kernels of every `period`-th launch (enable False: off)."""
        _check(lib().pxcl_set_timing(self._h, int(period) if enable else 0), "set_timing")

    def timing(self, reset: bool = False):
        """Summed milliseconds and timed launches of the kernels: segment, big,
        small, compact, hits."""
        ms = (ctypes.c_double * 5)()
        cnt = (ctypes.c_uint64 * 5)()
        _check(lib().pxcl_get_timing(self._h, ms, cnt, 1 if reset else 0), "get_timing")
        return list(ms), list(cnt)

    def workspace_bytes(self, max_digis: int) -> int:
        return int(lib().pxcl_event_workspace_bytes(self._h, int(max_digis)))

    def close(self):
        if self._h:
            _check(lib().pxcl_ctx_destroy(self._h), "ctx_destroy")
            self._h = ctypes.c_void_p()


class Event:
    """An event slot: a device workspace and a pinned status block, bound once."""

    def __init__(self, ctx: Context, max_digis: int, stream=None):
        self.ctx = ctx
        self.max_digis = int(max_digis)
        nb = ctx.workspace_bytes(self.max_digis)
        if nb == 0:
            raise PxclError(E_INVAL, "workspace size")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=f"cuda:{ctx.device}")
        pb = int(lib().pxcl_event_pinned_bytes(ctx.handle))
        self.pinned = torch.empty(max(pb, 64), dtype=torch.uint8, pin_memory=True)
        self._h = ctypes.c_void_p()
        _check(lib().pxcl_event_bind(ctx.handle, self.ws.data_ptr(), nb, self.pinned.data_ptr(), pb,
                                     self.max_digis, _stream_ptr(stream), ctypes.byref(self._h)), "event_bind")
        torch.cuda.synchronize(ctx.device)   # set-up time: the slot is clean before any stream uses it
        self._keep = None
        self._cb = None

    @property
    def handle(self):
        return self._h

    def _view(self, ptr: int, count: int) -> torch.Tensor:
        off = int(ptr) - self.ws.data_ptr()
        return self.ws[off: off + 4 * count].view(torch.int32)

    def close(self):
        if self._h:
            _check(lib().pxcl_event_unbind(self._h), "event_unbind")
            self._h = ctypes.c_void_p()


def acquire(event: Event, digis: Digis, stream=None, done_cb: Optional[Callable[[int], None]] = None,
            flag: Optional[Flag] = None) -> None:
    """Enqueue the clustering of one event; returns without waiting.  ``done_cb``
    (a Python callable, called with the status from the context's completion thread) or
    ``flag`` (filled by the library's own callback) signal completion."""
    d = digis.struct()
    cb_ptr, user = None, None
    if flag is not None:
        cb_ptr, user = flag_cb_ptr(), ctypes.addressof(flag)
    elif done_cb is not None:
        c = DONE_CB(lambda _u, st: done_cb(int(st)))
        event._cb = c
        cb_ptr = ctypes.cast(c, ctypes.c_void_p).value
    event._keep = (digis, d, flag)
    _check(lib().pxcl_acquire(event.handle, ctypes.byref(d), _stream_ptr(stream), cb_ptr, user), "acquire")


def query(event: Event) -> int:
    return int(lib().pxcl_query(event.handle))


def wait(event: Event) -> None:
    _check(lib().pxcl_wait(event.handle), "wait")


def produce(event: Event) -> ClusterResult:
    """Results of a completed event (E_NOT_READY raises).  Async input errors are
    reported in ``status`` rather than raised."""
    c = _Clusters()
    st = int(lib().pxcl_produce(event.handle, ctypes.byref(c)))
    if st in (E_NOT_READY, E_INVAL):
        raise PxclError(st, "produce")
    return ClusterResult(st, int(c.err_bits), int(c.n_clusters), event._view(c.id, c.n_clusters),
                         event._view(c.charge, c.n_clusters), event._view(c.size, c.n_clusters),
                         event._view(c.digi_cluster, c.n_digis), c.stream or 0, c.done_event or 0)


@dataclass
class HitsResult:
    status: int
    n_hits: int
    x: torch.Tensor      # float32 views into the event's workspace
    y: torch.Tensor
    stream: int
    done_event: int

    def numpy(self):
        return {"status": self.status, "n_hits": self.n_hits, "x": self.x.cpu().numpy(), "y": self.y.cpu().numpy()}


def hits_enqueue(event: Event, stream=None, done_cb: Optional[Callable[[int], None]] = None,
                 flag: Optional[Flag] = None) -> None:
    """Queue the hits of the event's last acquire on ``stream`` (a consumer of its
    clusters; another stream waits for the event's completion event)."""
    cb_ptr, user = None, None
    if flag is not None:
        cb_ptr, user = flag_cb_ptr(), ctypes.addressof(flag)
    elif done_cb is not None:
        c = DONE_CB(lambda _u, st: done_cb(int(st)))
        event._hcb = c
        cb_ptr = ctypes.cast(c, ctypes.c_void_p).value
    event._hkeep = flag
    _check(lib().pxcl_hits_enqueue(event.handle, _stream_ptr(stream), cb_ptr, user), "hits_enqueue")


def hits_query(event: Event) -> int:
    return int(lib().pxcl_hits_query(event.handle))


def hits_wait(event: Event) -> None:
    _check(lib().pxcl_hits_wait(event.handle), "hits_wait")


def hits_produce(event: Event) -> HitsResult:
    h = _Hits()
    st = int(lib().pxcl_hits_produce(event.handle, ctypes.byref(h)))
    if st in (E_NOT_READY, E_INVAL):
        raise PxclError(st, "hits_produce")
    n = int(h.n_hits)
    return HitsResult(st, n, event._view(h.x, n).view(torch.float32), event._view(h.y, n).view(torch.float32),
                      h.stream or 0, h.done_event or 0)


class HostCopy:
    """Pinned host buffers a copy to the host fills (cluster arrays of `capacity`,
    optionally per-digi ids and hits)."""

    def __init__(self, capacity: int, n_digis: int = 0, hits: bool = False):
        pin = dict(dtype=torch.int32, pin_memory=True)
        self.id, self.charge, self.size = (torch.zeros(max(1, capacity), **pin) for _ in range(3))
        self.digi = torch.zeros(max(1, n_digis), **pin) if n_digis else None
        fpin = dict(dtype=torch.float32, pin_memory=True)
        self.x = torch.zeros(max(1, capacity), **fpin) if hits else None
        self.y = torch.zeros(max(1, capacity), **fpin) if hits else None
        self.s = _HostClusters(self.id.data_ptr(), self.charge.data_ptr(), self.size.data_ptr(),
                               self.digi.data_ptr() if self.digi is not None else None,
                               self.x.data_ptr() if hits else None, self.y.data_ptr() if hits else None,
                               int(capacity), 0, E_NOT_READY)

    def numpy(self, n_digis: int = 0) -> dict:
        k = int(self.s.n_clusters)
        out = {"status": int(self.s.status), "n_clusters": k, "id": self.id[:k].numpy().copy(),
               "charge": self.charge[:k].numpy().copy(), "size": self.size[:k].numpy().copy()}
        if self.digi is not None:
            out["digi"] = self.digi[:n_digis].numpy().copy()
        if self.x is not None:
            out["x"], out["y"] = self.x[:k].numpy().copy(), self.y[:k].numpy().copy()
        return out


def copy_to_host(event: Event, dst: HostCopy, stream=None, flag: Optional[Flag] = None) -> None:
    """Queue the copy of the event's results (and hits, if `dst` has room for them)
    to pinned host memory; `flag` fires when the data is there."""
    cb_ptr, user = (flag_cb_ptr(), ctypes.addressof(flag)) if flag is not None else (None, None)
    event._ckeep = (dst, flag)
    _check(lib().pxcl_copy_to_host(event.handle, _stream_ptr(stream), ctypes.byref(dst.s), cb_ptr, user),
           "copy_to_host")


def copy_query(event: Event) -> int:
    return int(lib().pxcl_copy_query(event.handle))


class Batch:
    def __init__(self, ctx: Context, max_events: int, stream=None):
        self.ctx = ctx
        self.max_events = int(max_events)
        nb = int(lib().pxcl_batch_workspace_bytes(ctx.handle, self.max_events))
        pb = int(lib().pxcl_batch_pinned_bytes(ctx.handle, self.max_events))
        if nb == 0 or pb == 0:
            raise PxclError(E_INVAL, "batch size")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=f"cuda:{ctx.device}")
        self.pinned = torch.empty(pb, dtype=torch.uint8, pin_memory=True)
        self._h = ctypes.c_void_p()
        _check(lib().pxcl_batch_bind(ctx.handle, self.ws.data_ptr(), nb, self.pinned.data_ptr(), pb,
                                     self.max_events, _stream_ptr(stream), ctypes.byref(self._h)), "batch_bind")
        torch.cuda.synchronize(ctx.device)
        self._keep = None

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _check(lib().pxcl_batch_unbind(self._h), "batch_unbind")
            self._h = ctypes.c_void_p()


def _batch_arrays(events: Sequence[Event], digis: Sequence[Digis]):
    k = len(events)
    evs = (ctypes.c_void_p * k)(*[e.handle.value for e in events])
    ins = (_Digis * k)(*[d.struct() for d in digis])
    return k, evs, ins


class BatchInputs:
    """The argument arrays of one batch (event objects and their digis), marshalled
    once for repeated launches of the same inputs."""

    def __init__(self, events: Sequence[Event], digis: Sequence[Digis]):
        if len(events) != len(digis):
            raise ValueError("one Digis per event")
        self.k, self.evs, self.ins = _batch_arrays(events, digis)
        self._keep = (list(events), list(digis))


def acquire_batch(batch: Batch, events, digis: Optional[Sequence[Digis]] = None, stream=None,
                  flag: Optional[Flag] = None, graph: bool = False, defer_big: bool = False) -> None:
    """Launch a batch: `events` and `digis` are sequences of equal length, or `events`
    is a BatchInputs (and `digis` None); ``defer_big``: big-module kernels only in a
    second launch, when some event needs them (results final at the callback)."""
    prepared = events if isinstance(events, BatchInputs) else BatchInputs(events, digis)
    k, evs, ins = prepared.k, prepared.evs, prepared.ins
    cb_ptr, user = (flag_cb_ptr(), ctypes.addressof(flag)) if flag is not None else (None, None)
    batch._keep = (prepared, flag)
    _check(lib().pxcl_acquire_batch(batch.handle, evs, ins, k, _stream_ptr(stream), cb_ptr, user,
                                    (BATCH_GRAPH if graph else 0) | (BATCH_DEFER_BIG if defer_big else 0)),
           "acquire_batch")


def batch_query(batch: Batch) -> int:
    return int(lib().pxcl_batch_query(batch.handle))


def autotune(ctx: Context, batch: Batch, events: Sequence[Event], digis: Sequence[Digis], stream=None,
             reps: int = 5, cache_path: Optional[str] = None):
    """Time every (workgroup size, modules per workgroup) of the clustering kernel on
    this batch, keep the fastest; returns {(wg, mpw): microseconds}."""
    k, evs, ins = _batch_arrays(events, digis)
    us = (ctypes.c_float * 12)()
    _check(lib().pxcl_autotune(ctx.handle, batch.handle, evs, ins, k, _stream_ptr(stream), int(reps),
                               cache_path.encode() if cache_path else None, us), "autotune")
    out = {}
    for i, wg in enumerate((64, 128, 256, 512)):
        for j, mpw in enumerate((1, 2, 4)):
            if us[i * 3 + j] >= 0:
                out[(wg, mpw)] = float(us[i * 3 + j])
    return out


def autotune_load(ctx: Context, cache_path: str, mean_digis: int) -> bool:
    r = int(lib().pxcl_autotune_load(ctx.handle, cache_path.encode(), int(mean_digis)))
    if r == E_NOTFOUND:
        return False
    _check(r, "autotune_load")
    return True


def run_async(ctx: Context, events: Sequence[Event], streams, pool: Sequence[Digis], events_per_thread: int,
              cpu_task_ns: int = 0, blocking: bool = False, hits: bool = False,
              results: Optional[torch.Tensor] = None, result_offsets: Optional[Sequence[int]] = None) -> dict:
    """Asynchronous form.  With ``results`` (a device uint8 tensor) and
    ``result_offsets`` (one per event, request r = thread + i * threads) every event's
    outputs are copied there (verification mode)."""
    n = len(events)
    evs = (ctypes.c_void_p * n)(*[e.handle.value for e in events])
    sts = (ctypes.c_void_p * n)(*[int(s.cuda_stream) for s in streams])
    ins = (_Digis * len(pool))(*[d.struct() for d in pool])
    st = RunStats()
    n_req = n * int(events_per_thread)
    if result_offsets is not None and len(result_offsets) != n_req:
        raise ValueError(f"run_async: {len(result_offsets)} result offsets for {n_req} events")
    _check(lib().pxcl_run_async(ctx.handle, evs, sts, n, ins, len(pool), int(events_per_thread),
                                int(cpu_task_ns), (1 if blocking else 0) | (2 if hits else 0), ctypes.byref(st),
                                results.data_ptr() if results is not None else None,
                                (ctypes.c_uint64 * n_req)(*result_offsets) if result_offsets is not None
                                else None), "run_async")
    return st.as_dict()


def serve(ctx: Context, arena: torch.Tensor, pinned: torch.Tensor, batches: Sequence[Batch], streams,
          pool: Sequence[Digis], rate_hz: float, n_requests: int, budget_bytes: int, n_slots: int,
          max_batch: int, n_cpu_threads: int = 16, cpu_task_ns: int = 20000, graph: bool = True,
          seed: int = 1, results: Optional[torch.Tensor] = None, result_offsets: Optional[Sequence[int]] = None,
          max_inflight: int = 0, batch_delay_us: int = 0, defer_big: bool = False):
    """Serving form; returns (stats dict, per-request status, per-request n_clusters).
    With ``results`` (a device uint8 tensor) and ``result_offsets`` every request's
    outputs are copied there (verification mode)."""
    nb = len(batches)
    bh = (ctypes.c_void_p * nb)(*[b.handle.value for b in batches])
    sts = (ctypes.c_void_p * nb)(*[int(s.cuda_stream) for s in streams])
    ins = (_Digis * len(pool))(*[d.struct() for d in pool])
    o = ServeOpts(float(rate_hz), int(n_requests), int(budget_bytes), int(n_slots), int(max_batch),
                  int(n_cpu_threads), int(cpu_task_ns),
                  (BATCH_GRAPH if graph else 0) | (BATCH_DEFER_BIG if defer_big else 0), int(seed), int(max_inflight),
                  int(batch_delay_us))
    st = RunStats()
    rs = (ctypes.c_int32 * n_requests)()
    rn = (ctypes.c_uint32 * n_requests)()
    _check(lib().pxcl_serve(ctx.handle, arena.data_ptr(), arena.numel() * arena.element_size(),
                            pinned.data_ptr(), pinned.numel() * pinned.element_size(), bh, sts, nb, ins,
                            len(pool), ctypes.byref(o), ctypes.byref(st), rs, rn,
                            results.data_ptr() if results is not None else None,
                            (ctypes.c_uint64 * n_requests)(*result_offsets) if result_offsets is not None
                            else None), "serve")
    return st.as_dict(), list(rs), list(rn)


NOALLOC_MAX_DIGIS = 262144
ERRBIT_RANGE, ERRBIT_ORDER, ERRBIT_DUP, ERRBIT_INTERNAL, ERRBIT_HINT = 1, 2, 4, 8, 16


def status_from_bits(bits: int) -> int:
    """The status an event with these error bits reports (precedence RANGE, ORDER,
    HINT, DUP, INTERNAL)."""
    for bit, code in ((ERRBIT_RANGE, E_RANGE), (ERRBIT_ORDER, E_ORDER), (ERRBIT_HINT, E_HINT),
                      (ERRBIT_DUP, E_DUP_PIXEL), (ERRBIT_INTERNAL, E_INTERNAL)):
        if bits & bit:
            return code
    return OK


class NoAllocOutputs:
    """Caller-owned device outputs of ``cluster_noalloc`` for events of up to
    `max_digis` digis (allocated here, once, by torch; the call itself allocates
    nothing)."""

    def __init__(self, max_digis: int, device: int = 0):
        n = max(1, int(max_digis))
        dev = f"cuda:{device}"
        self.digi, self.id, self.charge, self.size = (torch.empty(n, dtype=torch.int32, device=dev) for _ in range(4))
        self.status = torch.zeros(16, dtype=torch.int32, device=dev)
        self.s = _NoAllocOut(self.digi.data_ptr(), self.id.data_ptr(), self.charge.data_ptr(),
                             self.size.data_ptr(), self.status.data_ptr())

    def numpy(self, n_digis: int, tag: int) -> dict:
        """Results once the stream has passed the call."""
        st = self.status.cpu().numpy().view(np.uint32)
        bits = int(st[1]) | (ERRBIT_INTERNAL if int(st[0]) != tag else 0)
        k = min(int(st[2]), n_digis)
        return {"status": status_from_bits(bits), "err_bits": bits, "n_clusters": k,
                "id": self.id[:k].cpu().numpy(), "charge": self.charge[:k].cpu().numpy(),
                "size": self.size[:k].cpu().numpy(), "digi": self.digi[:n_digis].cpu().numpy()}


def cluster_noalloc(ctx: Context, digis: Digis, out: NoAllocOutputs, stream=None) -> int:
    """Queue the clustering of one device-resident event on ``stream`` with the
    library's fixed per-device scratch (nothing allocated); returns the call's launch
    tag.  Results are in ``out`` once the stream has passed this point."""
    d = digis.struct()
    tag = ctypes.c_uint32()
    _check(lib().pxcl_cluster_noalloc(ctx.handle, ctypes.byref(d), ctypes.byref(out.s), _stream_ptr(stream),
                                      ctypes.byref(tag)), "cluster_noalloc")
    return int(tag.value)
