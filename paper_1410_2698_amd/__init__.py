"""Trajectory distance-threshold search on AMD MI355X (gfx950).

Thin Python front of ``libtds.so`` (C ABI in ``include/tds.h``).  Every step
of the search runs in the library's HIP kernels; this module only marshals
arguments.  PyTorch supplies device memory and the current stream.

Problem (Gowanlock & Casanova, arXiv:1410.2698, Sec. 3.1): for every query
segment and every entry segment of the indexed database that overlap in
time, report the interval during which the two linearly moving points are
within distance d.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional

import numpy as np

from . import _lib
from ._lib import (TDS_E_INVALID, TDS_E_OVERFLOW, TDS_OK, TDS_PREC_FP32_RECHECK, TDS_PREC_FP64, TdsError,
                   check, load)

RESULT_DTYPE = np.dtype([("q_seg", "<u4"), ("e_seg", "<u4"), ("q_traj", "<u4"),
                         ("e_traj", "<u4"), ("t_lo", "<f8"), ("t_hi", "<f8")])

TRAJ_DTYPE = np.dtype([("q_traj", "<u4"), ("e_traj", "<u4"), ("t_lo", "<f8"), ("t_hi", "<f8")])

PRECISIONS = {"fp64": TDS_PREC_FP64, "fp32": TDS_PREC_FP32_RECHECK,
              "fp32_recheck": TDS_PREC_FP32_RECHECK}

_FIELDS = ("xs", "ys", "zs", "ts", "xe", "ye", "ze", "te")


def _torch():
    import torch
    return torch


def _current_stream():
    torch = _torch()
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible: the search runs only on the GPU")
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class _SegHandle:
    """Keeps the arrays of one tds_segments view alive."""

    def __init__(self, S, keep):
        self.struct = S
        self.keep = keep


def prepare_segments(S) -> _SegHandle:
    """The C view of a segment set, built once (for callers that submit the
    same queries many times or want the marshalling out of a timed loop)."""
    return _segments(S)


def _segments(S) -> _SegHandle:
    if isinstance(S, _SegHandle):
        return S
    """Marshal a segment set: an object or dict with xs..te (+ traj), either
    NumPy arrays (host memory) or torch CUDA tensors (device memory)."""
    get = (lambda k: S[k]) if isinstance(S, dict) else (lambda k: getattr(S, k))
    arrs = [get(k) for k in _FIELDS]
    try:
        traj = get("traj")
    except (KeyError, AttributeError):
        traj = None
    st = _lib.tds_segments()
    first = arrs[0]
    keep = []
    if hasattr(first, "data_ptr"):  # torch tensors
        torch = _torch()
        for k, a in zip(_FIELDS, arrs):
            if not (a.is_cuda and a.dtype == torch.float64 and a.is_contiguous()):
                raise ValueError(f"{k}: expected a contiguous float64 CUDA tensor")
            setattr(st, k, a.data_ptr())
            keep.append(a)
        if traj is not None:
            if not (traj.is_cuda and traj.dtype in (torch.int32, torch.uint32) and traj.is_contiguous()):
                raise ValueError("traj: expected a contiguous int32/uint32 CUDA tensor")
            st.traj_id = traj.data_ptr()
            keep.append(traj)
        st.on_device = 1
        st.n = int(first.numel())
    else:
        for k, a in zip(_FIELDS, arrs):
            a = np.ascontiguousarray(a, dtype=np.float64)
            setattr(st, k, a.ctypes.data)
            keep.append(a)
        if traj is not None:
            t = np.ascontiguousarray(traj, dtype=np.uint32)
            st.traj_id = t.ctypes.data
            keep.append(t)
        st.on_device = 0
        st.n = int(np.asarray(arrs[0]).shape[0])
    return _SegHandle(st, keep)


LAYOUTS = {"default": _lib.TDS_LAYOUT_DEFAULT, "temporal": _lib.TDS_LAYOUT_TEMPORAL,
           "spatial": _lib.TDS_LAYOUT_SPATIAL}


class PendingSearch:
    """A search begun with Index.search_begin; end() waits for it (once)."""

    def __init__(self, lib, handle, segments):
        self._lib, self._h, self._segments = lib, handle, segments  # keep Q's arrays alive

    def end(self):
        if self._h is None:
            raise RuntimeError("tds_search_end: already ended")
        n = ctypes.c_uint64()
        st = _lib.tds_stats()
        status = self._lib.tds_search_end(self._h, ctypes.byref(n), ctypes.byref(st))
        self._h = None
        self._segments = None
        return status, int(n.value), st.as_dict()


class Index:
    """Temporal index of an entry-segment database, resident in HBM (Sec. 4.2.1);
    layout "spatial" (the default) also orders every bin by space and keeps a
    bounding box per 64-entry block (the subdivision idea of Sec. 4.3)."""

    def __init__(self, D, num_bins: int = 0, layout: str = "default"):
        lib = load()
        h = _segments(D)
        p = _lib.tds_build_params()
        p.num_bins = int(num_bins)
        p.layout = LAYOUTS[layout]
        out = ctypes.c_void_p()
        check(lib.tds_build_index(ctypes.byref(h.struct), ctypes.byref(p), _current_stream(),
                                  ctypes.byref(out)), "tds_build_index")
        self._h = out
        self._lib = lib
        self.last_stats: Optional[dict] = None

    def close(self):
        if getattr(self, "_h", None):
            self._lib.tds_index_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = _lib.tds_index_info()
        check(self._lib.tds_index_info_get(self._h, ctypes.byref(inf)), "tds_index_info_get")
        return {k: getattr(inf, k) for k, _ in inf._fields_}

    def export(self) -> dict:
        inf = self.info()
        n, m = inf["n"], inf["num_bins"]
        out = {"order": np.empty(n, np.uint32), "bin_first": np.empty(m + 1, np.uint32),
               "min_ts": np.empty(m), "max_te": np.empty(m), "cmax_te": np.empty(m)}
        check(self._lib.tds_index_export(self._h, *[out[k].ctypes.data for k in
                                                    ("order", "bin_first", "min_ts", "max_te", "cmax_te")]),
              "tds_index_export")
        return out

    def schedule(self, Q, t_start: float = -math.inf, t_end: float = math.inf):
        h = _segments(Q)
        n = h.struct.n
        lo, hi = np.empty(n, np.uint32), np.empty(n, np.uint32)
        check(self._lib.tds_schedule(self._h, ctypes.byref(h.struct), float(t_start), float(t_end),
                                     lo.ctypes.data, hi.ctypes.data, _current_stream()), "tds_schedule")
        return lo, hi

    def search_raw(self, Q, d: float, t_start: float = -math.inf, t_end: float = math.inf, *,
                   out_ptr: int, capacity: int, out_on_device: bool, precision: str = "fp32",
                   chunk: int = 0, grid_waves: int = 0, device_capacity: int = 0, tile: int = 0, refine: str = "default", deal: str = "default",
                   output: str = "default"):
        """One call of tds_search into caller memory; returns (status, n_total, stats)."""
        h = _segments(Q)
        p = _search_params(precision, chunk, grid_waves, tile, refine, deal, output)
        p.out_on_device = 1 if out_on_device else 0
        p.device_capacity = int(device_capacity)
        n = ctypes.c_uint64()
        st = _lib.tds_stats()
        status = self._lib.tds_search(self._h, ctypes.byref(h.struct), float(d), float(t_start),
                                      float(t_end), ctypes.c_void_p(out_ptr), ctypes.c_uint64(capacity),
                                      ctypes.byref(n), ctypes.byref(p), _current_stream(),
                                      ctypes.byref(st))
        self.last_stats = st.as_dict()
        return status, int(n.value), self.last_stats

    def search_begin(self, Q, d: float, t_start: float = -math.inf, t_end: float = math.inf, *,
                     out_ptr: int, capacity: int, precision: str = "fp32", chunk: int = 0,
                     grid_waves: int = 0, tile: int = 0, refine: str = "default",
                     deal: str = "default", output: str = "default"):
        """tds_search_begin into device memory at out_ptr: the search is ordered
        on the current stream and this returns at once.  Returns a
        PendingSearch; its end() waits and gives (status, n_total, stats)."""
        h = _segments(Q)
        p = _search_params(precision, chunk, grid_waves, tile, refine, deal, output)
        p.out_on_device = 1
        handle = ctypes.c_void_p()
        check(self._lib.tds_search_begin(self._h, ctypes.byref(h.struct), float(d),
                                         float(t_start), float(t_end), ctypes.c_void_p(out_ptr),
                                         ctypes.c_uint64(capacity), ctypes.byref(p),
                                         _current_stream(), ctypes.byref(handle)),
              "tds_search_begin")
        return PendingSearch(self._lib, handle, h)

    def search_noalloc_raw(self, Q, d: float, t_start: float = -math.inf,
                           t_end: float = math.inf, *, out_ptr: int, capacity: int,
                           precision: str = "fp32", chunk: int = 0, grid_waves: int = 0,
                           tile: int = 0, refine: str = "default", deal: str = "default",
                   output: str = "default"):
        """One call of tds_search_noalloc (Q and out in device memory); returns
        (status, n_total, stats)."""
        h = _segments(Q)
        p = _search_params(precision, chunk, grid_waves, tile, refine, deal, output)
        p.out_on_device = 1
        n = ctypes.c_uint64()
        st = _lib.tds_stats()
        status = self._lib.tds_search_noalloc(self._h, ctypes.byref(h.struct), float(d),
                                              float(t_start), float(t_end),
                                              ctypes.c_void_p(out_ptr), ctypes.c_uint64(capacity),
                                              ctypes.byref(n), ctypes.byref(p),
                                              _current_stream(), ctypes.byref(st))
        return status, int(n.value), st.as_dict()

    def search(self, Q, d: float, t_start: float = -math.inf, t_end: float = math.inf, *,
               capacity: Optional[int] = None, precision: str = "fp32", chunk: int = 0,
               grid_waves: int = 0, device_capacity: int = 0, tile: int = 0, refine: str = "default",
               deal: str = "default", output: str = "default") -> np.ndarray:
        """Search into host memory; grows the buffer and retries on overflow.
        Returns the records (unspecified order) as a NumPy structured array."""
        cap = 1 << 16 if capacity is None else int(capacity)
        while True:
            buf = np.empty(max(cap, 1), RESULT_DTYPE)
            status, n, _ = self.search_raw(Q, d, t_start, t_end, out_ptr=buf.ctypes.data,
                                           capacity=cap, out_on_device=False, precision=precision,
                                           chunk=chunk, grid_waves=grid_waves,
                                           device_capacity=device_capacity, tile=tile,
                                           refine=refine, deal=deal, output=output)
            if status == TDS_OK:
                return buf[:n].copy()
            if status == TDS_E_OVERFLOW and capacity is None:
                cap = n
                continue
            raise TdsError(status, "tds_search")


    def self_join_raw(self, d: float, t_start: float = -math.inf, t_end: float = math.inf, *,
                      out_ptr: int, capacity: int, out_on_device: bool, precision: str = "fp32",
                      chunk: int = 0, grid_waves: int = 0, device_capacity: int = 0,
                      tile: int = 0, refine: str = "default", deal: str = "default",
                   output: str = "default"):
        """One call of tds_self_join into caller memory; returns (status, n_total, stats)."""
        p = _search_params(precision, chunk, grid_waves, tile, refine, deal, output)
        p.out_on_device = 1 if out_on_device else 0
        p.device_capacity = int(device_capacity)
        n = ctypes.c_uint64()
        st = _lib.tds_stats()
        status = self._lib.tds_self_join(self._h, float(d), float(t_start), float(t_end),
                                         ctypes.c_void_p(out_ptr), ctypes.c_uint64(capacity),
                                         ctypes.byref(n), ctypes.byref(p), _current_stream(),
                                         ctypes.byref(st))
        self.last_stats = st.as_dict()
        return status, int(n.value), self.last_stats

    def self_join(self, d: float, t_start: float = -math.inf, t_end: float = math.inf, *,
                  capacity: Optional[int] = None, precision: str = "fp32",
                  device_capacity: int = 0) -> np.ndarray:
        """Self-join of the indexed segments (pairs of different trajectories,
        each once, lower segment id first) into host memory; grows the buffer
        on overflow."""
        cap = 1 << 16 if capacity is None else int(capacity)
        while True:
            buf = np.empty(max(cap, 1), RESULT_DTYPE)
            status, n, _ = self.self_join_raw(d, t_start, t_end, out_ptr=buf.ctypes.data,
                                              capacity=cap, out_on_device=False,
                                              precision=precision, device_capacity=device_capacity)
            if status == TDS_OK:
                return buf[:n].copy()
            if status == TDS_E_OVERFLOW and capacity is None:
                cap = n
                continue
            raise TdsError(status, "tds_self_join")

    def search_batch_raw(self, Q, requests, *, out_ptr: int, out_capacity: int,
                         out_on_device: bool, precision: str = "fp32", chunk: int = 0,
                         grid_waves: int = 0, tile: int = 0, refine: str = "default", deal: str = "default",
                   output: str = "default"):
        """One call of tds_search_batch into caller memory.  ``requests`` holds
        (q_begin, q_count, d, t_start, t_end, out_offset, out_capacity) tuples
        that tile Q in order.  Returns (status, counts, stats)."""
        h = _segments(Q)
        reqs = (_lib.tds_request * len(requests))()
        for r, (qb, qc, d, t0, t1, oo, oc) in zip(reqs, requests):
            r.q_begin, r.q_count, r.d, r.t_start, r.t_end = int(qb), int(qc), float(d), float(t0), float(t1)
            r.out_offset, r.out_capacity = int(oo), int(oc)
        counts = (ctypes.c_uint64 * len(requests))()
        p = _search_params(precision, chunk, grid_waves, tile, refine, deal, output)
        p.out_on_device = 1 if out_on_device else 0
        st = _lib.tds_stats()
        status = self._lib.tds_search_batch(self._h, ctypes.byref(h.struct), reqs, len(requests),
                                            ctypes.c_void_p(out_ptr), int(out_capacity), counts,
                                            ctypes.byref(p), _current_stream(), ctypes.byref(st))
        self.last_stats = st.as_dict()
        return status, [int(c) for c in counts], self.last_stats

    def search_batch(self, requests, *, precision: str = "fp32", chunk: int = 0,
                     grid_waves: int = 0, capacity: Optional[int] = None):
        """Batched search (tds_search_batch).  ``requests`` is a list of
        (Q, d, t_start, t_end); returns one record array per request.  Output
        slices start at ``capacity`` records each and grow on overflow."""
        Qcat, reqs = _concat_requests(requests, 1 << 12 if capacity is None else capacity)
        h = _segments(Qcat)
        while True:
            total = sum(r.out_capacity for r in reqs)
            buf = np.empty(max(total, 1), RESULT_DTYPE)
            counts = (ctypes.c_uint64 * len(reqs))()
            p = _search_params(precision, chunk, grid_waves)
            st = _lib.tds_stats()
            status = self._lib.tds_search_batch(self._h, ctypes.byref(h.struct), reqs, len(reqs),
                                                ctypes.c_void_p(buf.ctypes.data), total, counts,
                                                ctypes.byref(p), _current_stream(), ctypes.byref(st))
            self.last_stats = st.as_dict()
            if status == TDS_OK:
                return [buf[r.out_offset: r.out_offset + counts[i]].copy() for i, r in enumerate(reqs)]
            if status == TDS_E_OVERFLOW and capacity is None:
                _resize_slices(reqs, counts)
                continue
            raise TdsError(status, "tds_search_batch")


class FSG:
    """Fixed spatial grid over the entries of an Index (the spatial method of
    Sec. 4.1, Alg. 1); the Index must outlive the grid."""

    def __init__(self, index: "Index", gx: int = 0, gy: int = 0, gz: int = 0):
        lib = load()
        out = ctypes.c_void_p()
        check(lib.tds_fsg_build(index.handle, int(gx), int(gy), int(gz), _current_stream(),
                                ctypes.byref(out)), "tds_fsg_build")
        self._h = out
        self._lib = lib
        self._index = index  # keeps the entries alive
        self.last_stats: Optional[dict] = None

    def close(self):
        if getattr(self, "_h", None):
            self._lib.tds_fsg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def search_raw(self, Q, d: float, t_start: float = -math.inf, t_end: float = math.inf, *,
                   out_ptr: int, capacity: int, out_on_device: bool):
        """One call of tds_fsg_search into caller memory; returns (status, n_total, stats)."""
        h = _segments(Q)
        p = _search_params("fp64")
        p.out_on_device = 1 if out_on_device else 0
        n = ctypes.c_uint64()
        st = _lib.tds_stats()
        status = self._lib.tds_fsg_search(self._h, ctypes.byref(h.struct), float(d), float(t_start),
                                          float(t_end), ctypes.c_void_p(out_ptr),
                                          ctypes.c_uint64(capacity), ctypes.byref(n), ctypes.byref(p),
                                          _current_stream(), ctypes.byref(st))
        self.last_stats = st.as_dict()
        return status, int(n.value), self.last_stats

    def search(self, Q, d: float, t_start: float = -math.inf, t_end: float = math.inf, *,
               capacity: Optional[int] = None) -> np.ndarray:
        """Search into host memory; grows the buffer and retries on overflow."""
        cap = 1 << 16 if capacity is None else int(capacity)
        while True:
            buf = np.empty(max(cap, 1), RESULT_DTYPE)
            status, n, _ = self.search_raw(Q, d, t_start, t_end, out_ptr=buf.ctypes.data,
                                           capacity=cap, out_on_device=False)
            if status == TDS_OK:
                return buf[:n].copy()
            if status == TDS_E_OVERFLOW and capacity is None:
                cap = n
                continue
            raise TdsError(status, "tds_fsg_search")


REFINES = {"default": 0, "queued": 1, "inline": 2}
DEALS = {"default": 0, "dynamic": 1, "static": 2}
OUTPUTS = {"default": 0, "direct": 1, "staged": 2}


def _search_params(precision="fp32", chunk=0, grid_waves=0, tile=0, refine="default",
                   deal="default", output="default"):
    lib = load()
    p = _lib.tds_search_params()
    lib.tds_search_params_default(ctypes.byref(p))
    p.precision = PRECISIONS[precision]
    p.chunk = int(chunk)
    p.grid_waves = int(grid_waves)
    p.tile = int(tile)
    p.refine = REFINES[refine]
    p.deal = DEALS[deal]
    p.output = OUTPUTS[output]
    return p


def _concat_requests(requests, cap):
    """Concatenate the requests' query segments; one output slice each."""
    parts = [r[0] for r in requests]
    Qcat = {k: np.concatenate([np.asarray(getattr(q, k) if not isinstance(q, dict) else q[k],
                                          dtype=np.float64) for q in parts]) for k in _FIELDS}
    Qcat["traj"] = np.concatenate([np.asarray(getattr(q, "traj") if not isinstance(q, dict) else q["traj"],
                                              dtype=np.uint32) for q in parts])
    reqs = (_lib.tds_request * len(requests))()
    off = 0
    for i, (q, d, t0, t1) in enumerate(requests):
        n = len(np.asarray(getattr(q, "xs") if not isinstance(q, dict) else q["xs"]))
        reqs[i].q_begin = off
        reqs[i].q_count = n
        reqs[i].d = float(d)
        reqs[i].t_start = float(t0)
        reqs[i].t_end = float(t1)
        reqs[i].out_offset = i * cap
        reqs[i].out_capacity = cap
        off += n
    return Qcat, reqs


def _resize_slices(reqs, counts):
    off = 0
    for i in range(len(reqs)):
        reqs[i].out_offset = off
        reqs[i].out_capacity = max(int(counts[i]), int(reqs[i].out_capacity))
        off += reqs[i].out_capacity


class Batcher:
    """Fixed-capacity batched search replayed from a captured hipGraph."""

    def __init__(self, index: Index, max_segments: int, max_requests: int, result_capacity: int,
                 *, precision: str = "fp32", chunk: int = 0, grid_waves: int = 0):
        self._lib = load()
        self.index = index
        self.result_capacity = int(result_capacity)
        p = _search_params(precision, chunk, grid_waves)
        out = ctypes.c_void_p()
        check(self._lib.tds_batcher_create(index.handle, int(max_segments), int(max_requests),
                                           int(result_capacity), ctypes.byref(p), None,
                                           ctypes.byref(out)), "tds_batcher_create")
        self._h = out
        self.last_stats: Optional[dict] = None

    def run(self, requests, slice_capacity: Optional[int] = None):
        """``requests``: list of (Q, d, t_start, t_end).  Returns (records per
        request, status): every request gets an equal output slice."""
        cap = slice_capacity or max(1, self.result_capacity // len(requests))
        Qcat, reqs = _concat_requests(requests, cap)
        h = _segments(Qcat)
        buf = np.empty(self.result_capacity, RESULT_DTYPE)
        counts = (ctypes.c_uint64 * len(reqs))()
        st = _lib.tds_stats()
        status = self._lib.tds_batcher_run(self._h, ctypes.byref(h.struct), reqs, len(reqs),
                                           ctypes.c_void_p(buf.ctypes.data), counts, ctypes.byref(st))
        if status not in (TDS_OK, TDS_E_OVERFLOW):
            raise TdsError(status, "tds_batcher_run")
        self.last_stats = st.as_dict()
        out = [buf[r.out_offset: r.out_offset + min(counts[i], r.out_capacity)].copy()
               for i, r in enumerate(reqs)]
        return out, [int(c) for c in counts], status

    @property
    def replays(self) -> int:
        return int(self._lib.tds_batcher_replays(self._h))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.tds_batcher_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop with continuous batching over a resident index."""

    def __init__(self, index: Index, *, max_batch_segments: int = 0, max_batch_requests: int = 0,
                 slots: int = 0, result_capacity: int = 0, default_reserve: int = 0,
                 max_pending: int = 0, precision: str = "fp32", chunk: int = 0, grid_waves: int = 0,
                 tile: int = 0, refine: str = "default", deal: str = "default",
                   output: str = "default",
                 cpu_route_tests: int = 0):
        self._lib = load()
        self.index = index
        p = _lib.tds_server_params()
        p.max_batch_segments = max_batch_segments
        p.max_batch_requests = max_batch_requests
        p.slots = slots
        p.result_capacity = result_capacity
        p.default_reserve = default_reserve
        p.max_pending = max_pending
        p.cpu_route_tests = int(cpu_route_tests)
        p.search = _search_params(precision, chunk, grid_waves, tile, refine, deal, output)
        out = ctypes.c_void_p()
        check(self._lib.tds_server_create(index.handle, ctypes.byref(p), ctypes.byref(out)),
              "tds_server_create")
        self._h = out
        self._keep = {}

    def submit(self, Q, d: float, t_start: float = -math.inf, t_end: float = math.inf, *,
               reserve: int = 0, blocking: bool = True) -> int:
        h = _segments(Q)
        t = ctypes.c_uint64()
        check(self._lib.tds_server_submit(self._h, ctypes.byref(h.struct), float(d), float(t_start),
                                          float(t_end), int(reserve), 1 if blocking else 0,
                                          ctypes.byref(t)), "tds_server_submit")
        return int(t.value)

    def wait(self, ticket: int):
        """Returns (records, latency_ms)."""
        cap = 1024
        while True:
            buf = np.empty(cap, RESULT_DTYPE)
            n = ctypes.c_uint64()
            lat = ctypes.c_double()
            st = self._lib.tds_server_wait(self._h, ticket, ctypes.c_void_p(buf.ctypes.data), cap,
                                           ctypes.byref(n), ctypes.byref(lat))
            if st == TDS_OK:
                return buf[: n.value].copy(), lat.value
            if st == TDS_E_OVERFLOW:
                cap = int(n.value)
                continue
            raise TdsError(st, "tds_server_wait")

    def poll(self, ticket: int) -> bool:
        done = ctypes.c_int()
        check(self._lib.tds_server_poll(self._h, ticket, ctypes.byref(done)), "tds_server_poll")
        return bool(done.value)

    def stats(self) -> dict:
        s = _lib.tds_server_stats()
        check(self._lib.tds_server_stats_get(self._h, ctypes.byref(s)), "tds_server_stats_get")
        return s.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            self._lib.tds_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def abi_version() -> int:
    return int(load().tds_abi_version())


def sort_records(r: np.ndarray) -> np.ndarray:
    """Records in (q_seg, e_seg) order."""
    key = (r["q_seg"].astype(np.uint64) << np.uint64(32)) | r["e_seg"].astype(np.uint64)
    return r[np.argsort(key, kind="stable")]


def merge_trajectories_raw(recs_ptr: int, n: int, recs_on_device: bool, out_ptr: int,
                           capacity: int, out_on_device: bool):
    """One call of tds_merge_trajectories; returns (status, n_total)."""
    lib = load()
    n_out = ctypes.c_uint64()
    status = lib.tds_merge_trajectories(ctypes.c_void_p(recs_ptr), int(n), 1 if recs_on_device else 0,
                                        ctypes.c_void_p(out_ptr), int(capacity),
                                        1 if out_on_device else 0, ctypes.byref(n_out),
                                        _current_stream())
    return status, int(n_out.value)


def merge_trajectories(records: np.ndarray, capacity: Optional[int] = None) -> np.ndarray:
    """Trajectory-level intervals of host segment records (TRAJ_DTYPE array in
    (q_traj, e_traj, t_lo) order), merged on the GPU."""
    recs = np.ascontiguousarray(records, dtype=RESULT_DTYPE)
    cap = max(recs.size, 1) if capacity is None else int(capacity)
    while True:
        out = np.empty(max(cap, 1), TRAJ_DTYPE)
        status, n = merge_trajectories_raw(recs.ctypes.data, recs.size, False, out.ctypes.data,
                                           cap, False)
        if status == TDS_OK:
            return out[:n].copy()
        if status == TDS_E_OVERFLOW and capacity is None:
            cap = n
            continue
        raise TdsError(status, "tds_merge_trajectories")
