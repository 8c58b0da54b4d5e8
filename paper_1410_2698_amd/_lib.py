"""ctypes declarations of the C ABI in include/tds.h (argument marshalling only).

The library is built in-tree (``paper_1410_2698_amd/libtds.so``); loading
fails loudly when it is missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtds.so")

TDS_OK, TDS_E_INVALID, TDS_E_OVERFLOW, TDS_E_NOMEM, TDS_E_DEVICE, TDS_E_BUSY = range(6)
TDS_PREC_DEFAULT, TDS_PREC_FP64, TDS_PREC_FP32_RECHECK = 0, 1, 2
TDS_LAYOUT_DEFAULT, TDS_LAYOUT_TEMPORAL, TDS_LAYOUT_SPATIAL = 0, 1, 2

c_dbl_p = ctypes.POINTER(ctypes.c_double)
c_u32_p = ctypes.POINTER(ctypes.c_uint32)
c_u64_p = ctypes.POINTER(ctypes.c_uint64)


class tds_segments(ctypes.Structure):
    _fields_ = [("xs", ctypes.c_void_p), ("ys", ctypes.c_void_p), ("zs", ctypes.c_void_p),
                ("ts", ctypes.c_void_p), ("xe", ctypes.c_void_p), ("ye", ctypes.c_void_p),
                ("ze", ctypes.c_void_p), ("te", ctypes.c_void_p), ("traj_id", ctypes.c_void_p),
                ("n", ctypes.c_uint64), ("on_device", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class tds_build_params(ctypes.Structure):
    _fields_ = [("num_bins", ctypes.c_uint32), ("layout", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 6)]


class tds_search_params(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("out_on_device", ctypes.c_int32),
                ("chunk", ctypes.c_uint32), ("grid_waves", ctypes.c_uint32),
                ("device_capacity", ctypes.c_uint64), ("tile", ctypes.c_uint32),
                ("refine", ctypes.c_uint32), ("deal", ctypes.c_uint32),
                ("output", ctypes.c_uint32), ("reserved", ctypes.c_uint64 * 2)]


class tds_stats(ctypes.Structure):
    _fields_ = [("query_segments", ctypes.c_uint64), ("active_segments", ctypes.c_uint64),
                ("work_items", ctypes.c_uint64), ("candidate_tests", ctypes.c_uint64),
                ("fp64_evals", ctypes.c_uint64), ("results", ctypes.c_uint64),
                ("passes", ctypes.c_uint32), ("stage_flushes", ctypes.c_uint32),
                ("kernel_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("filter_tests", ctypes.c_uint64), ("block_tests", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class tds_index_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("num_bins", ctypes.c_uint32), ("device", ctypes.c_uint32),
                ("t_min", ctypes.c_double), ("t_max", ctypes.c_double),
                ("bin_width", ctypes.c_double), ("device_bytes", ctypes.c_uint64),
                ("layout", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class tds_request(ctypes.Structure):
    _fields_ = [("q_begin", ctypes.c_uint64), ("q_count", ctypes.c_uint64), ("d", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_end", ctypes.c_double),
                ("out_offset", ctypes.c_uint64), ("out_capacity", ctypes.c_uint64)]


class tds_server_params(ctypes.Structure):
    _fields_ = [("max_batch_segments", ctypes.c_uint64), ("max_batch_requests", ctypes.c_uint32),
                ("slots", ctypes.c_uint32), ("result_capacity", ctypes.c_uint64),
                ("default_reserve", ctypes.c_uint64), ("max_pending", ctypes.c_uint32),
                ("cpu_route_tests", ctypes.c_uint32), ("search", tds_search_params)]


class tds_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("requeued", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("max_batch_requests_seen", ctypes.c_uint64),
                ("cpu_routed", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class tds_traj_interval(ctypes.Structure):
    _fields_ = [("q_traj", ctypes.c_uint32), ("e_traj", ctypes.c_uint32),
                ("t_lo", ctypes.c_double), ("t_hi", ctypes.c_double)]


# exported name -> (restype, argtypes)
SIGNATURES = {
    "tds_abi_version": (ctypes.c_uint32, []),
    "tds_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "tds_build_index": (ctypes.c_int, [ctypes.POINTER(tds_segments), ctypes.POINTER(tds_build_params),
                                       ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "tds_index_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "tds_index_info_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(tds_index_info)]),
    "tds_index_export": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "tds_schedule": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(tds_segments), ctypes.c_double,
                                    ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "tds_search": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(tds_segments), ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_void_p, ctypes.c_uint64,
                                  c_u64_p, ctypes.POINTER(tds_search_params), ctypes.c_void_p,
                                  ctypes.POINTER(tds_stats)]),
    "tds_search_begin": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(tds_segments),
                                        ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_void_p, ctypes.c_uint64,
                                        ctypes.POINTER(tds_search_params), ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "tds_search_end": (ctypes.c_int, [ctypes.c_void_p, c_u64_p, ctypes.POINTER(tds_stats)]),
    "tds_search_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(tds_segments),
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_void_p, ctypes.c_uint64, c_u64_p,
                                          ctypes.POINTER(tds_search_params), ctypes.c_void_p,
                                          ctypes.POINTER(tds_stats)]),
    "tds_search_params_default": (None, [ctypes.POINTER(tds_search_params)]),
    "tds_self_join": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_void_p, ctypes.c_uint64, c_u64_p,
                                     ctypes.POINTER(tds_search_params), ctypes.c_void_p,
                                     ctypes.POINTER(tds_stats)]),
    "tds_fsg_build": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_uint32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "tds_fsg_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "tds_fsg_search": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(tds_segments), ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                      ctypes.c_uint64, c_u64_p, ctypes.POINTER(tds_search_params),
                                      ctypes.c_void_p, ctypes.POINTER(tds_stats)]),
    "tds_merge_trajectories": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                              ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, c_u64_p,
                                              ctypes.c_void_p]),
    "tds_last_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(tds_stats)]),
    "tds_search_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(tds_segments),
                                        ctypes.POINTER(tds_request), ctypes.c_uint32, ctypes.c_void_p,
                                        ctypes.c_uint64, c_u64_p, ctypes.POINTER(tds_search_params),
                                        ctypes.c_void_p, ctypes.POINTER(tds_stats)]),
    "tds_batcher_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                          ctypes.c_uint64, ctypes.POINTER(tds_search_params),
                                          ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "tds_batcher_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(tds_segments),
                                       ctypes.POINTER(tds_request), ctypes.c_uint32, ctypes.c_void_p,
                                       c_u64_p, ctypes.POINTER(tds_stats)]),
    "tds_batcher_replays": (ctypes.c_uint64, [ctypes.c_void_p]),
    "tds_batcher_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "tds_server_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(tds_server_params),
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "tds_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(tds_segments), ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                         ctypes.c_int, c_u64_p]),
    "tds_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]),
    "tds_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                       ctypes.c_uint64, c_u64_p, ctypes.POINTER(ctypes.c_double)]),
    "tds_server_stats_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(tds_server_stats)]),
    "tds_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
}

_lib = None


class TdsError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = load().tds_status_str(status).decode() if _lib is not None else f"status {status}"
        super().__init__(f"{what}: {msg}" if what else msg)


def load():
    """Load libtds.so and declare every entry point; raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() or "
                               "python paper_1410_2698_amd/build.py")
        # torch (the source of device memory and streams) is loaded first, so
        # that libtds.so binds to the HIP runtime torch brings; loaded the
        # other way round, the process holds two HIP runtimes and torch's
        # streams and memory are not valid in the library's
        import torch  # noqa: F401
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int, what: str = ""):
    if status != TDS_OK:
        raise TdsError(status, what)
