"""Host-only checks of the C-ABI library: it loads, exports every entry point the
header declares, and rejects bad arguments before touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1310_6736_amd import ks

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ks.h")


def _lib():
    if not os.path.exists(ks.LIB_PATH):
        from paper_1310_6736_amd import build
        build.build_library()
    return ks.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\*?\s+\*?(ks_[a-z_0-9]+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["ks_detect", "ks_detect_device", "ks_detect_batch", "ks_histograms", "ks_seed_traces",
                 "ks_server_create", "ks_server_submit", "ks_server_poll", "ks_server_stats", "ks_server_destroy",
                 "ks_context_create", "ks_context_destroy", "ks_status_str"]:
        assert must in names


def test_library_exports_every_declared_function():
    L = _lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    for name in ks.EXPORTS:
        assert hasattr(L, name), name


def test_status_strings():
    L = _lib()
    assert L.ks_status_str(0) == b"ok"
    assert L.ks_status_str(-1) == b"invalid argument"
    assert L.ks_status_str(-4) == b"request larger than the budget"
    assert L.ks_status_str(-99) == b"unknown status"


def _detect(vol=np.zeros((4, 4, 4), np.uint8), dtype=0, dims=(4, 4, 4), bins=32, sp=2, scales=(1, 2), method=0,
            max_iter=5, cap=8, out=True, nfound=True):
    L = _lib()
    buf = (ks.Region * max(cap, 1))()
    nf = C.c_int32()
    return L.ks_detect(C.c_void_p(vol.ctypes.data) if vol is not None else None, dtype,
                       (C.c_int32 * 3)(*dims) if dims is not None else None, bins, sp,
                       (C.c_int32 * 2)(*scales) if scales is not None else None, method, max_iter,
                       buf if out else None, cap, C.byref(nf) if nfound else None)


@pytest.mark.parametrize("kw", [
    dict(vol=None), dict(dims=None), dict(scales=None), dict(dtype=3), dict(dtype=-1),
    dict(dims=(0, 4, 4)), dict(dims=(4, 70000, 1)), dict(dims=(65535, 65535, 1)),
    dict(bins=1), dict(bins=257), dict(sp=0), dict(scales=(0, 2)), dict(scales=(3, 2)), dict(scales=(1, 33)),
    dict(method=2), dict(max_iter=-1), dict(cap=-1), dict(out=False), dict(nfound=False),
])
def test_detect_rejects_bad_arguments_before_any_gpu_call(kw):
    assert _detect(**kw) == ks.KS_E_INVALID


def test_null_context_is_rejected():
    L = _lib()
    nf = C.c_int32()
    dims = (C.c_int32 * 3)(4, 4, 4)
    sc = (C.c_int32 * 2)(1, 2)
    assert L.ks_detect_device(None, C.c_void_p(1), 0, dims, 32, 2, sc, 0, 5, None, 0, C.byref(nf), None) == -1
    assert L.ks_seed_traces(None, C.c_void_p(1), 0, dims, 32, 2, sc, 0, 5, None, 0, C.byref(nf), None) == -1
    assert L.ks_histograms(None, C.c_void_p(1), 0, dims, 32, 0, sc, 0, None, None, None, None) == -1
    assert L.ks_detect_batch(None, 0, None, None, None) == -1
    assert L.ks_last_stats(None, None) == -1
    assert L.ks_context_destroy(None) == -1
    assert L.ks_server_poll(None, 1, None, 0, C.byref(nf)) == -1
    assert L.ks_server_destroy(None) == -1


def test_server_create_rejects_bad_arguments():
    L = _lib()
    h = C.c_void_p()
    assert L.ks_server_create(0, 0, 4, C.byref(h)) == -1
    assert L.ks_server_create(0, 1 << 30, 0, C.byref(h)) == -1
    assert L.ks_server_create(0, 1 << 30, 17, C.byref(h)) == -1
    assert L.ks_server_create(-1, 1 << 30, 2, C.byref(h)) == -1
    assert L.ks_server_create(0, 1 << 30, 2, None) == -1


def test_context_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = _lib()
    h = C.c_void_p()
    assert L.ks_context_create(0, C.byref(h)) == ks.KS_E_DEVICE


def build_consumer(out_dir):
    """Compiles tests/abi_consumer.c as strict C99 against include/ks.h and links
    it to libks.so (host compiler only)."""
    import subprocess
    _lib()
    exe = os.path.join(out_dir, "abi_consumer")
    libdir = os.path.dirname(ks.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
                    "-o", exe, os.path.join(ROOT, "tests", "abi_consumer.c"), "-L", libdir, "-lks",
                    "-Wl,-rpath," + libdir], check=True)
    return exe


def test_header_is_c99_and_links(tmp_path):
    exe = build_consumer(str(tmp_path))
    assert os.path.exists(exe)
