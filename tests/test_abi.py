"""The C ABI library loads, exports every declared entry point, and its struct
layouts agree with include/*.h.  No GPU needed: nothing here launches work."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

from paper_1410_2698_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(tds_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_headers_exist():
    assert HEADERS


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_functions()
    assert "tds_search" in names and "tds_build_index" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(declared_functions()) <= set(_lib.SIGNATURES), \
        set(declared_functions()) - set(_lib.SIGNATURES)


def test_version_and_status_strings():
    lib = _lib.load()
    assert lib.tds_abi_version() == 4
    assert lib.tds_status_str(0) == b"TDS_OK"
    assert b"OVERFLOW" in lib.tds_status_str(2)
    assert lib.tds_status_str(12345) == b"unknown tds status"


def test_search_params_default():
    lib = _lib.load()
    p = _lib.tds_search_params()
    p.chunk = 77
    lib.tds_search_params_default(ctypes.byref(p))
    assert p.precision == _lib.TDS_PREC_FP32_RECHECK and p.chunk == 0 and p.out_on_device == 0


def test_argument_validation_without_device_work():
    lib = _lib.load()
    out = ctypes.c_void_p()
    assert lib.tds_build_index(None, None, None, ctypes.byref(out)) == _lib.TDS_E_INVALID
    seg = _lib.tds_segments()  # n = 0, NULL arrays
    assert lib.tds_build_index(ctypes.byref(seg), None, None, ctypes.byref(out)) == _lib.TDS_E_INVALID
    n = ctypes.c_uint64(7)
    assert lib.tds_search(None, ctypes.byref(seg), 1.0, 0.0, 1.0, None, 0, ctypes.byref(n), None,
                          None, None) == _lib.TDS_E_INVALID
    assert lib.tds_index_destroy(None) == _lib.TDS_OK
    assert lib.tds_last_stats(None, None) == _lib.TDS_E_INVALID
    assert lib.tds_index_info_get(None, None) == _lib.TDS_E_INVALID
    n_out = ctypes.c_uint64(5)
    assert lib.tds_merge_trajectories(None, 0, 0, None, 0, 0, ctypes.byref(n_out), None) == _lib.TDS_OK
    assert n_out.value == 0
    assert lib.tds_merge_trajectories(None, 3, 0, None, 0, 0, ctypes.byref(n_out), None) == \
        _lib.TDS_E_INVALID
    assert lib.tds_self_join(None, 1.0, 0.0, 1.0, None, 0, ctypes.byref(n_out), None, None,
                             None) == _lib.TDS_E_INVALID


def test_struct_layouts_match_header(tmp_path):
    """Compile a C program against include/tds.h and compare sizes/offsets."""
    structs = {
        "tds_segments": _lib.tds_segments, "tds_build_params": _lib.tds_build_params,
        "tds_search_params": _lib.tds_search_params, "tds_stats": _lib.tds_stats,
        "tds_index_info": _lib.tds_index_info, "tds_request": _lib.tds_request,
        "tds_server_params": _lib.tds_server_params, "tds_server_stats": _lib.tds_server_stats,
        "tds_traj_interval": _lib.tds_traj_interval,
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tds.h"', "int main(void){"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append('printf("tds_result %zu\\n", sizeof(tds_result));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                       check=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)
    import paper_1410_2698_amd as tds
    assert int(got["tds_result"]) == tds.RESULT_DTYPE.itemsize == 32
    assert int(got["tds_traj_interval"]) == tds.TRAJ_DTYPE.itemsize == 24


def test_binding_loads_one_hip_runtime():
    """Loaded through the binding first thing in a process, libtds.so must
    share torch's HIP runtime (one libamdhip64 mapped): with two, torch's
    streams and device memory are invalid in the library's runtime."""
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1410_2698_amd import _lib\n"
            "_lib.load()\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n") % ROOT
    r = subprocess.run(["python3", "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.split()[-1] == "1"
