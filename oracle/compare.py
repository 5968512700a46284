"""Oracle of the paper's comparison filters (Section "Other Filters"): mean,
sigma, Okada, entropy.  TEST INFRASTRUCTURE ONLY (see the package docstring).

The per-voxel arithmetic is in ``lnf_oracle.c`` (``lnfo_compare``); this module
computes the two global inputs from the whole volume in exact or plainly
defined arithmetic:
  - the sigma filter's half width w = floor(2 sigma), sigma the standard
    deviation of all voxel values (population), from exact integer sums;
  - the entropy filter's per-level weights -p log2 p, p = count / N, in fixed
    point: floor(value * 2^32 + 1/2), evaluated in fp64 with the C library's
    log2 (Python's math.log2), and the threshold likewise.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import _dtype_code, _load

MEAN, SIGMA, OKADA, ENTROPY = 0, 1, 2, 3
FIXED_ONE = 1 << 32


def _isqrt(n: int) -> int:
    return math.isqrt(n)


def sigma_half_width(vol: np.ndarray) -> int:
    """floor(2 sigma) of the volume's values, exact."""
    v = vol.astype(np.int64).ravel()
    n = int(v.size)
    s = int(v.sum())
    q = int(np.sum(v * v, dtype=np.uint64))
    # (2 sigma)^2 = 4 (n q - s^2) / n^2; floor(sqrt(x / y)) = isqrt(floor(x / y))
    return _isqrt((4 * (n * q - s * s)) // (n * n))


def entropy_weights(vol: np.ndarray) -> np.ndarray:
    """Fixed-point -p log2 p for every grey level of the volume's dtype."""
    levels = 256 if vol.dtype == np.uint8 else 65536
    hist = np.bincount(vol.ravel(), minlength=levels)
    n = int(vol.size)
    w = np.zeros(levels, dtype=np.int64)
    for level in np.nonzero(hist)[0]:
        p = int(hist[level]) / n
        w[level] = math.floor(-p * math.log2(p) * FIXED_ONE + 0.5)
    return w


def fixed(value: float) -> int:
    """A threshold in the weights' 2^-32 fixed point."""
    return math.floor(value * FIXED_ONE + 0.5)


def filter_compare(vol: np.ndarray, kind: int, r: int = 1, param: int = 0,
                   weights: np.ndarray | None = None, gate: int = 0) -> np.ndarray:
    vol = np.ascontiguousarray(vol)
    nz, ny, nx = vol.shape
    out = np.empty_like(vol)
    lib = _load()
    lib.lnfo_compare.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                 ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p]
    lib.lnfo_compare.restype = ctypes.c_int
    wp = None
    if weights is not None:
        weights = np.ascontiguousarray(weights, dtype=np.int64)
        wp = weights.ctypes.data
    rc = lib.lnfo_compare(vol.ctypes.data, nx, ny, nz, _dtype_code(vol), kind, r, int(param), wp,
                          gate, out.ctypes.data)
    if rc:
        raise ValueError("oracle rejected the arguments")
    return out


def mean_filter(vol, r, gate=0):
    return filter_compare(vol, MEAN, r, 0, None, gate)


def sigma_filter(vol, r, half_width=None, gate=0):
    w = sigma_half_width(vol) if half_width is None else int(half_width)
    return filter_compare(vol, SIGMA, r, w, None, gate)


def okada_filter(vol, t_d, gate=0):
    return filter_compare(vol, OKADA, 1, int(t_d), None, gate)


def entropy_filter(vol, r, t_e, gate=0):
    return filter_compare(vol, ENTROPY, r, fixed(t_e), entropy_weights(vol), gate)
