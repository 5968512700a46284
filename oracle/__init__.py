"""CPU oracle of the nine-cluster local noise filter.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU
library (``paper_1807_03119_amd``) and never imports it.

The arithmetic lives in ``lnf_oracle.c`` (brute force over the nine clusters,
straight from the definition) and ``otsu.py`` (exact Otsu threshold); this
module only compiles the C file with gcc and marshals numpy arrays into it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .otsu import histogram, otsu_threshold  # noqa: F401

MEAN9 = 0
MINVAR9 = 1
BOX = 0      # cubic clusters of side 2r+1
CROSS = 1    # eq. 2's three lines of 2r+1 voxels through the cluster centre
# diagonal offset of the eight outer clusters
OFFSET_R = 0       # d = r
OFFSET_ONE = 1     # d = 1
OFFSET_TILE = 2    # d = 2r+1

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lnf_oracle.c")
LIB_PATH = os.path.join(_HERE, "liblnf_oracle.so")
_lib = None


def build(src: str = _SRC, out: str = LIB_PATH) -> str:
    """Compile the oracle with gcc (always recompiles).  The tests also compile
    deliberately broken copies of the source this way, to show that the pins
    catch them."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", "-Wall", "-Wextra",
           "-o", tmp, src]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    _lib = open_library(LIB_PATH)
    return _lib


def open_library(path: str):
    """ctypes handle of a compiled oracle, with its argument types set."""
    lib = ctypes.CDLL(path)
    i64, vp = ctypes.c_int64, ctypes.c_void_p
    lib.lnfo_filter.argtypes = [vp, i64, i64, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.c_uint32, vp]
    lib.lnfo_filter_geom.argtypes = [vp, i64, i64, i64, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_uint32, ctypes.c_int, ctypes.c_int,
                                     vp]
    lib.lnfo_cluster_stats_geom.argtypes = [vp, i64, i64, i64, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_int, i64, i64, i64, vp, vp]
    lib.lnfo_filter_points.argtypes = [vp, i64, i64, i64, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_uint32, vp, i64, vp]
    lib.lnfo_cluster_stats.argtypes = [vp, i64, i64, i64, ctypes.c_int, ctypes.c_int,
                                       i64, i64, i64, vp, vp]
    lib.lnfo_threads.argtypes = []
    lib.lnfo_set_threads.argtypes = [ctypes.c_int]
    lib.lnfo_set_threads.restype = None
    for f in (lib.lnfo_filter, lib.lnfo_filter_geom, lib.lnfo_filter_points,
              lib.lnfo_cluster_stats, lib.lnfo_cluster_stats_geom, lib.lnfo_threads):
        f.restype = ctypes.c_int
    return lib


def _dtype_code(vol: np.ndarray) -> int:
    if vol.dtype == np.uint8:
        return 1
    if vol.dtype == np.uint16:
        return 2
    raise TypeError(f"oracle takes uint8 or uint16 volumes, got {vol.dtype}")


def filter_volume(vol: np.ndarray, r: int, rule: int = MEAN9, gate: int = 0,
                  shape: int = BOX, offset: int = OFFSET_R) -> np.ndarray:
    """Filter a whole [z, y, x] volume (cluster shape and diagonal offset as above)."""
    vol = np.ascontiguousarray(vol)
    nz, ny, nx = vol.shape
    out = np.empty_like(vol)
    rc = _load().lnfo_filter_geom(vol.ctypes.data, nx, ny, nz, _dtype_code(vol), r, rule, gate,
                                  shape, offset, out.ctypes.data)
    if rc:
        raise ValueError("oracle rejected the arguments")
    return out


def filter_points(vol: np.ndarray, r: int, xyz, rule: int = MEAN9, gate: int = 0) -> np.ndarray:
    """Filtered values at the voxels xyz[m, 3] = (x, y, z); returns uint32[m]."""
    vol = np.ascontiguousarray(vol)
    nz, ny, nx = vol.shape
    pts = np.ascontiguousarray(np.asarray(xyz, dtype=np.int64).reshape(-1, 3))
    out = np.empty(pts.shape[0], dtype=np.uint32)
    rc = _load().lnfo_filter_points(vol.ctypes.data, nx, ny, nz, _dtype_code(vol), r, rule,
                                    gate, pts.ctypes.data, pts.shape[0], out.ctypes.data)
    if rc:
        raise ValueError("oracle rejected the arguments")
    return out


def cluster_stats(vol: np.ndarray, r: int, x: int, y: int, z: int, shape: int = BOX,
                  offset: int = OFFSET_R):
    """(sums[9], sums of squares[9]) of the nine clusters about voxel (x, y, z)."""
    vol = np.ascontiguousarray(vol)
    nz, ny, nx = vol.shape
    s = np.zeros(9, dtype=np.uint64)
    q = np.zeros(9, dtype=np.uint64)
    rc = _load().lnfo_cluster_stats_geom(vol.ctypes.data, nx, ny, nz, _dtype_code(vol), r, shape,
                                         offset, x, y, z, s.ctypes.data, q.ctypes.data)
    if rc:
        raise ValueError("oracle rejected the arguments")
    return s, q


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().lnfo_threads())


def set_threads(n: int) -> None:
    """Run the oracle's parallel loops on n threads from now on."""
    _load().lnfo_set_threads(int(n))
