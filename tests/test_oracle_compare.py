"""Pins of the comparison-filter oracle (paper, Section "Other Filters": the
mean filter eq. 4, sigma eq. 5, Okada eq. 6, entropy eq. 7) against library
routines, numpy formulations written independently, closed forms and special
cases.  The readings of the garbled formulas are stated in oracle/compare.py."""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import compare
from paper_1807_03119_amd import phantom as ph


def _vols():
    return [ph.small_u8(1000, dims=(12, 10, 9)),
            ph.ct_u12((11, 9, 13), seed=2001),
            ph.random_volume((8, 7, 6), np.uint16, seed=3, kind="uniform"),
            ph.random_volume((9, 5, 7), np.uint8, seed=4, kind="low")]


def _windows(vol, r):
    """All (2r+1)^3 clamped neighbours of every voxel: array [k, z, y, x]."""
    p = np.pad(vol.astype(np.int64), r, mode="edge")
    nz, ny, nx = vol.shape
    out = []
    for dz in range(2 * r + 1):
        for dy in range(2 * r + 1):
            for dx in range(2 * r + 1):
                out.append(p[dz:dz + nz, dy:dy + ny, dx:dx + nx])
    return np.stack(out)


def _round_half_up(num, den):
    return (2 * num + den) // (2 * den)


@pytest.mark.parametrize("r", [1, 2, 3])
def test_mean_filter_equals_convolution(r):
    for vol in _vols():
        m = 2 * r + 1
        s = ndimage.convolve(vol.astype(np.int64), np.ones((m, m, m), np.int64), mode="nearest")
        np.testing.assert_array_equal(compare.mean_filter(vol, r),
                                      _round_half_up(s, m ** 3).astype(vol.dtype))


@pytest.mark.parametrize("r", [1, 2])
def test_sigma_filter_numpy_bruteforce(r):
    for vol in _vols():
        w = _windows(vol, r)
        p0 = vol.astype(np.int64)[None]
        for hw in (0, 3, 40, 1000):
            sel = np.abs(w - p0) <= hw
            num = np.where(sel, w, 0).sum(0)
            den = sel.sum(0)
            want = _round_half_up(num, den).astype(vol.dtype)
            np.testing.assert_array_equal(compare.sigma_filter(vol, r, hw), want)


def test_sigma_special_cases_and_half_width():
    for vol in _vols():
        # a zero range keeps only values equal to the centre: the identity
        np.testing.assert_array_equal(compare.sigma_filter(vol, 2, 0), vol)
        # a range wider than the data is the plain mean filter
        np.testing.assert_array_equal(compare.sigma_filter(vol, 2, 1 << 20),
                                      compare.mean_filter(vol, 2))
        sd = float(np.std(vol.astype(np.float64)))
        w = compare.sigma_half_width(vol)
        assert w == math.floor(2 * sd) or abs(2 * sd - round(2 * sd)) < 1e-9


def test_okada_filter_numpy_bruteforce():
    for vol in _vols():
        p = np.pad(vol.astype(np.int64), 1, mode="edge")
        nz, ny, nx = vol.shape
        c = p[1:-1, 1:-1, 1:-1]
        nbs = [c, p[1:-1, 1:-1, :-2], p[1:-1, 1:-1, 2:], p[1:-1, :-2, 1:-1], p[1:-1, 2:, 1:-1],
               p[:-2, 1:-1, 1:-1], p[2:, 1:-1, 1:-1]]
        for td in (0, 1, 25, 1 << 20):
            sel = [np.abs(v - c) < td for v in nbs]
            num = sum(np.where(s, v, 0) for s, v in zip(sel, nbs))
            den = sum(s.astype(np.int64) for s in sel)
            want = np.where(den > 0, _round_half_up(num, np.maximum(den, 1)), 0).astype(vol.dtype)
            np.testing.assert_array_equal(compare.okada_filter(vol, td), want)
        # t_d = 1 keeps only equal neighbours: the identity; t_d = 0 keeps none
        np.testing.assert_array_equal(compare.okada_filter(vol, 1), vol)
        assert not compare.okada_filter(vol, 0).any()


def test_entropy_filter_against_float_sums():
    for vol in _vols():
        n = vol.size
        hist = np.bincount(vol.ravel())
        wf = np.zeros(hist.size)
        nzl = hist > 0
        p = hist[nzl] / n
        wf[nzl] = -p * np.log2(p)
        h = _windows(vol, 1)
        hsum = wf[h].sum(0)
        vals = np.unique(np.round(hsum, 9))
        # thresholds midway between distinct window entropies: float and fixed point agree
        for t in ([vals[len(vals) // 2] - 1e-3] if len(vals) == 1 else
                  [(vals[i] + vals[i + 1]) / 2 for i in (0, len(vals) // 2, len(vals) - 2)]):
            want = np.where(hsum > t, vol, 0).astype(vol.dtype)
            np.testing.assert_array_equal(compare.entropy_filter(vol, 1, t), want)
        np.testing.assert_array_equal(compare.entropy_filter(vol, 1, -1.0), vol)
        assert not compare.entropy_filter(vol, 1, 1e9).any()


def test_entropy_two_level_closed_form():
    # two equally frequent levels: every voxel weighs -0.5 log2 0.5 = 1/2, so a
    # 3^3 window sums to 13.5 wherever it lies
    z, y, x = np.meshgrid(np.arange(6), np.arange(6), np.arange(6), indexing="ij")
    vol = (((x + y + z) % 2) * 200 + 10).astype(np.uint8)
    np.testing.assert_array_equal(compare.entropy_filter(vol, 1, 13.4), vol)
    assert not compare.entropy_filter(vol, 1, 13.6).any()
    assert compare.entropy_weights(vol)[10] == 1 << 31


def test_comparison_gate():
    vol = ph.ct_u12((10, 9, 8), seed=2002)
    for fn in (lambda g: compare.mean_filter(vol, 1, g), lambda g: compare.sigma_filter(vol, 1, 50, g),
               lambda g: compare.okada_filter(vol, 30, g), lambda g: compare.entropy_filter(vol, 1, 0.5, g)):
        base, gated = fn(0), fn(1500)
        np.testing.assert_array_equal(gated, np.where(base < 1500, 0, base))
