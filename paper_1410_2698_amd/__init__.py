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
from ._lib import (TDS_E_OVERFLOW, TDS_OK, TDS_PREC_FP32_RECHECK, TDS_PREC_FP64, TdsError,
                   check, load)

RESULT_DTYPE = np.dtype([("q_seg", "<u4"), ("e_seg", "<u4"), ("q_traj", "<u4"),
                         ("e_traj", "<u4"), ("t_lo", "<f8"), ("t_hi", "<f8")])

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


def _segments(S) -> _SegHandle:
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


class Index:
    """Temporal index of an entry-segment database, resident in HBM (Sec. 4.2.1)."""

    def __init__(self, D, num_bins: int = 0):
        lib = load()
        h = _segments(D)
        p = _lib.tds_build_params()
        p.num_bins = int(num_bins)
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
                   chunk: int = 0, grid_waves: int = 0, device_capacity: int = 0):
        """One call of tds_search into caller memory; returns (status, n_total, stats)."""
        h = _segments(Q)
        p = _lib.tds_search_params()
        self._lib.tds_search_params_default(ctypes.byref(p))
        p.precision = PRECISIONS[precision]
        p.out_on_device = 1 if out_on_device else 0
        p.chunk = int(chunk)
        p.grid_waves = int(grid_waves)
        p.device_capacity = int(device_capacity)
        n = ctypes.c_uint64()
        st = _lib.tds_stats()
        status = self._lib.tds_search(self._h, ctypes.byref(h.struct), float(d), float(t_start),
                                      float(t_end), ctypes.c_void_p(out_ptr), ctypes.c_uint64(capacity),
                                      ctypes.byref(n), ctypes.byref(p), _current_stream(),
                                      ctypes.byref(st))
        self.last_stats = st.as_dict()
        return status, int(n.value), self.last_stats

    def search(self, Q, d: float, t_start: float = -math.inf, t_end: float = math.inf, *,
               capacity: Optional[int] = None, precision: str = "fp32", chunk: int = 0,
               grid_waves: int = 0, device_capacity: int = 0) -> np.ndarray:
        """Search into host memory; grows the buffer and retries on overflow.
        Returns the records (unspecified order) as a NumPy structured array."""
        cap = 1 << 16 if capacity is None else int(capacity)
        while True:
            buf = np.empty(max(cap, 1), RESULT_DTYPE)
            status, n, _ = self.search_raw(Q, d, t_start, t_end, out_ptr=buf.ctypes.data,
                                           capacity=cap, out_on_device=False, precision=precision,
                                           chunk=chunk, grid_waves=grid_waves,
                                           device_capacity=device_capacity)
            if status == TDS_OK:
                return buf[:n].copy()
            if status == TDS_E_OVERFLOW and capacity is None:
                cap = n
                continue
            raise TdsError(status, "tds_search")


def abi_version() -> int:
    return int(load().tds_abi_version())


def sort_records(r: np.ndarray) -> np.ndarray:
    """Records in (q_seg, e_seg) order."""
    key = (r["q_seg"].astype(np.uint64) << np.uint64(32)) | r["e_seg"].astype(np.uint64)
    return r[np.argsort(key, kind="stable")]
