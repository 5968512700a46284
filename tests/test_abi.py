"""Host-side checks of the C ABI: the library loads and exports every function
include/lnf.h declares; calls that need no GPU behave as documented."""
import ctypes
import os
import re

import pytest

from paper_1807_03119_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if hdr.endswith(".h"):
            text = open(os.path.join(ROOT, "include", hdr)).read()
            names += re.findall(r"LNF_API\s+[\w\s\*]+?\b(lnf_\w+)\s*\(", text)
    return names


def test_header_declares_core_entry_points():
    names = set(_declared_functions())
    for core in ("lnf_create", "lnf_filter", "lnf_destroy", "lnf_strerror"):
        assert core in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_and_version():
    assert _lib.lnf_strerror(0) == "success"
    assert "invalid" in _lib.lnf_strerror(_lib.LNF_EINVAL)
    assert _lib.lnf_strerror(12345) == "unknown status code"
    assert _lib.lnf_version() >= 10000


def test_tile_variants_argument_checks():
    assert _lib.lnf_tile_variants(_lib.LNF_MEAN9, _lib.LNF_U16, 3) >= 1
    assert _lib.lnf_tile_variants(_lib.LNF_MINVAR9, _lib.LNF_U8, 1) >= 1
    for bad in ((_lib.LNF_MEAN9, 3, 1), (_lib.LNF_MEAN9, _lib.LNF_U8, 0),
                (_lib.LNF_MEAN9, _lib.LNF_U8, _lib.LNF_RADIUS_MAX + 1), (7, _lib.LNF_U8, 1)):
        assert _lib.lib().lnf_tile_variants(*bad) == _lib.LNF_EINVAL


def test_null_arguments_rejected_without_touching_the_gpu():
    lib = _lib.lib()
    assert lib.lnf_create(None, None) == _lib.LNF_EINVAL
    assert lib.lnf_destroy(None) == _lib.LNF_OK
    dims = (ctypes.c_int64 * 3)(4, 4, 4)
    assert lib.lnf_filter(None, None, dims, 1, 1, None, None) == _lib.LNF_EINVAL


def test_create_bad_options():
    lib = _lib.lib()
    h = ctypes.c_void_p()
    opt = _lib.lnf_options(ctypes.sizeof(_lib.lnf_options), 5, 0, -1, 0)
    assert lib.lnf_create(ctypes.byref(h), ctypes.byref(opt)) == _lib.LNF_EINVAL
    opt = _lib.lnf_options(4, 0, 0, -1, 0)
    assert lib.lnf_create(ctypes.byref(h), ctypes.byref(opt)) == _lib.LNF_EINVAL
    # unknown geometry bits, and the two offset bits together
    for flags in (8, 0x80000000, _lib.LNF_GEOM_OFFSET_1 | _lib.LNF_GEOM_OFFSET_2R1,
                  _lib.LNF_GEOM_CROSS | _lib.LNF_GEOM_OFFSET_1 | _lib.LNF_GEOM_OFFSET_2R1):
        opt = _lib.lnf_options(ctypes.sizeof(_lib.lnf_options), 0, 0, -1, flags)
        assert lib.lnf_create(ctypes.byref(h), ctypes.byref(opt)) == _lib.LNF_EINVAL


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert _lib.lib().lnf_create(ctypes.byref(h), None) == _lib.LNF_EDEVICE


def test_host_otsu_matches_oracle():
    """The library's exact host-side Otsu (no GPU needed) against the oracle."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(4)
    cases = [np.zeros(256, np.uint64), np.bincount([7] * 9, minlength=256)]
    for _ in range(30):
        levels = int(rng.choice([2, 3, 17, 256, 4096]))
        h = rng.integers(0, 1000, levels).astype(np.uint64)
        h[rng.integers(0, levels, levels // 3)] = 0
        cases.append(h)
    big = np.zeros(65536, np.uint64)
    big[[100, 4000, 65535]] = [2 ** 40, 3 * 2 ** 39, 12345]  # huge counts: wide arithmetic
    cases.append(big)
    for h in cases:
        assert _lib.lnf_otsu_threshold(h) == oracle.otsu_threshold(h)
