"""Python front of the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package; the product library
never does.  It shares no code with the GPU path; inputs come from
``trajgen`` (which holds no search arithmetic).

Each function cites the part of the paper it follows; the arithmetic itself
lives in ``oracle.c`` and is documented there.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

RESULT_DTYPE = np.dtype([("q_seg", "<u4"), ("e_seg", "<u4"), ("q_traj", "<u4"),
                         ("e_traj", "<u4"), ("t_lo", "<f8"), ("t_hi", "<f8")])
TRAJ_DTYPE = np.dtype([("q_traj", "<u4"), ("e_traj", "<u4"), ("t_lo", "<f8"), ("t_hi", "<f8")])

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: FP64, no FMA contraction, no fast-math."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
               "-o", _SO + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64, dbl = ctypes.c_int64, ctypes.c_double
        lib.orc_pair.argtypes = [P, P, dbl, dbl, dbl, P, P]
        lib.orc_pair.restype = ctypes.c_int
        lib.orc_search.argtypes = [i64] + [P] * 9 + [i64] + [P] * 9 + [dbl, dbl, dbl, ctypes.c_int, P]
        lib.orc_search.restype = i64
        lib.orc_free.argtypes = [P]
        lib.orc_velocity.argtypes = [i64] + [P] * 11
        lib.orc_bins.argtypes = [i64, P, P, i64] + [P] * 10
        lib.orc_bins.restype = ctypes.c_int
        lib.orc_schedule.argtypes = [i64, P, P, P, P, i64, P, P, dbl, dbl, P, P]
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def velocity(S):
    """Per-segment velocity (P_end - P_start) / (t_end - t_start) (Sec. 3.1:
    a segment is a linearly moving point between its two 4-D end points)."""
    lib = _load()
    n = len(S)
    arrs = [_f64(getattr(S, k)) for k in ("xs", "ys", "zs", "ts", "xe", "ye", "ze", "te")]
    v = [np.empty(n) for _ in range(3)]
    lib.orc_velocity(n, *[_ptr(a) for a in arrs], *[_ptr(a) for a in v])
    return np.stack(v, axis=1)


def pair(q, l, d: float, t_start: float = -np.inf, t_end: float = np.inf):
    """One interaction (Sec. 3.1): ``q`` and ``l`` are {xs,ys,zs,vx,vy,vz,ts,te}.
    Returns (t_lo, t_hi) or None."""
    lib = _load()
    qa, la = _f64(q), _f64(l)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    ok = lib.orc_pair(_ptr(qa), _ptr(la), d, t_start, t_end, ctypes.byref(lo), ctypes.byref(hi))
    return (lo.value, hi.value) if ok else None


def seg_record(xs, ys, zs, ts, xe, ye, ze, te):
    """Build the {xs,ys,zs,vx,vy,vz,ts,te} record of one segment (velocity as in
    ``velocity``)."""
    lib = _load()
    vals = [np.array([v], dtype=np.float64) for v in (xs, ys, zs, ts, xe, ye, ze, te)]
    v = [np.empty(1) for _ in range(3)]
    lib.orc_velocity(1, *[_ptr(a) for a in vals], *[_ptr(a) for a in v])
    return np.array([xs, ys, zs, v[0][0], v[1][0], v[2][0], ts, te], dtype=np.float64)


def search(Q, D, d: float, t_start: float = -np.inf, t_end: float = np.inf,
           threads: int = 0) -> np.ndarray:
    """Brute-force distance threshold search (Sec. 3.1): every (q, l) pair, strict
    time overlap, canonical FP64 evaluation.  Returns records sorted by
    (q_seg, e_seg)."""
    lib = _load()
    qa = [_f64(getattr(Q, k)) for k in ("xs", "ys", "zs", "ts", "xe", "ye", "ze", "te")]
    da = [_f64(getattr(D, k)) for k in ("xs", "ys", "zs", "ts", "xe", "ye", "ze", "te")]
    qt = np.ascontiguousarray(Q.traj, dtype=np.uint32)
    dt = np.ascontiguousarray(D.traj, dtype=np.uint32)
    out = ctypes.c_void_p()
    n = lib.orc_search(len(Q), *[_ptr(a) for a in qa], _ptr(qt),
                       len(D), *[_ptr(a) for a in da], _ptr(dt),
                       float(d), float(t_start), float(t_end), int(threads), ctypes.byref(out))
    if n < 0:
        raise MemoryError("oracle search failed to allocate")
    try:
        buf = (ctypes.c_char * (int(n) * RESULT_DTYPE.itemsize)).from_address(out.value) if n else b""
        res = np.frombuffer(bytes(buf), dtype=RESULT_DTYPE).copy() if n else np.zeros(0, RESULT_DTYPE)
    finally:
        lib.orc_free(out)
    return sort_results(res)


def sort_results(res: np.ndarray) -> np.ndarray:
    """Canonical order (q_seg, e_seg)."""
    key = (res["q_seg"].astype(np.uint64) << np.uint64(32)) | res["e_seg"].astype(np.uint64)
    return res[np.argsort(key, kind="stable")]


def bins(ts, te, m: int):
    """Temporal bins of Sec. 4.2.1 (see ``oracle.c``).  Returns a dict."""
    lib = _load()
    ts, te = _f64(ts), _f64(te)
    n = ts.shape[0]
    out = {
        "order": np.empty(n, np.int64), "bin": np.empty(n, np.int32),
        "first": np.empty(m, np.int64), "last": np.empty(m, np.int64),
        "bstart": np.empty(m), "bend": np.empty(m), "min_ts": np.empty(m),
        "max_te": np.empty(m), "cmax_te": np.empty(m), "t_range": np.empty(2),
    }
    rc = lib.orc_bins(n, _ptr(ts), _ptr(te), m, *[_ptr(out[k]) for k in
                      ("order", "bin", "first", "last", "bstart", "bend", "min_ts",
                       "max_te", "cmax_te", "t_range")])
    if rc != 0:
        raise ValueError("bad bin arguments")
    return out


def schedule(ts, te, m: int, qts, qte, t_start=-np.inf, t_end=np.inf, tables: Optional[dict] = None):
    """Candidate range [lo, hi) of every query segment (Sec. 4.2.2 schedule S)."""
    lib = _load()
    ts, te = _f64(ts), _f64(te)
    tb = tables if tables is not None else bins(ts, te, m)
    qts, qte = _f64(qts), _f64(qte)
    nq = qts.shape[0]
    lo, hi = np.empty(nq, np.int64), np.empty(nq, np.int64)
    lib.orc_schedule(m, _ptr(tb["first"]), _ptr(tb["last"]), _ptr(tb["min_ts"]), _ptr(tb["cmax_te"]),
                     nq, _ptr(qts), _ptr(qte), float(t_start), float(t_end), _ptr(lo), _ptr(hi))
    return lo, hi


def self_join(D, d: float, t_start: float = -np.inf, t_end: float = np.inf,
              threads: int = 0) -> np.ndarray:
    """Every pair of segments of D from different trajectories within d during
    the window (the all-against-all search that motivates the paper, Sec. 1),
    each unordered pair once, lower segment id first: the brute-force search
    of D against itself, keeping the records with q_seg < e_seg of different
    trajectories (the pair's interval does not depend on which side is the
    query: the evaluation is symmetric under exchanging the two segments)."""
    res = search(D, D, d, t_start, t_end, threads=threads)
    keep = (res["q_traj"] != res["e_traj"]) & (res["q_seg"] < res["e_seg"])
    return sort_results(res[keep])


def merge_trajectories(recs: np.ndarray) -> np.ndarray:
    """Trajectory-level intervals: per (q_traj, e_traj), the union of the
    records' [t_lo, t_hi] as maximal intervals, taking the records in t_lo
    order and extending the current interval while the next one starts no
    later than its end (touching intervals merge).  Sorted by
    (q_traj, e_traj, t_lo).  A plain loop over the records."""
    recs = np.asarray(recs)
    order = np.lexsort((recs["t_lo"], recs["e_traj"], recs["q_traj"]))
    out = []
    cur = None
    for i in order:
        key = (int(recs["q_traj"][i]), int(recs["e_traj"][i]))
        lo, hi = float(recs["t_lo"][i]), float(recs["t_hi"][i])
        if cur is not None and cur[0] == key and lo <= cur[2]:
            cur[2] = max(cur[2], hi)
            continue
        if cur is not None:
            out.append((cur[0][0], cur[0][1], cur[1], cur[2]))
        cur = [key, lo, hi]
    if cur is not None:
        out.append((cur[0][0], cur[0][1], cur[1], cur[2]))
    return np.array(out, dtype=TRAJ_DTYPE)
