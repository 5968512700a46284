"""Otsu's data threshold, exactly, in Python integers.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; never called by the product
path).

Paper, Section "Our Method", eq. 1: the threshold T minimises the within-class
variance w0(T)*s0^2(T) + w1(T)*s1^2(T) of the two classes it separates.  Because
the total variance is the sum of the within-class and between-class variances,
the same T maximises the between-class variance w0*w1*(mu0 - mu1)^2, which in
counts is  (N*s0 - n0*S)^2 / (N^2 * n0 * n1).  The comparison below is done by
cross-multiplication in exact integers.

Readings where the paper is silent: class 0 holds the levels v < T and class 1
the levels v >= T (T is the lower limit of the kept intensity range); among
equal optima the lowest T wins; only T with both classes non-empty are valid;
if no T is valid (at most one level present) T is that level (0 for an empty
histogram), so that a gate at T keeps everything.
"""
from __future__ import annotations

import numpy as np


def histogram(vol: np.ndarray, levels: int | None = None) -> np.ndarray:
    """Counts of each grey level of an unsigned integer volume."""
    if levels is None:
        levels = int(np.iinfo(vol.dtype).max) + 1
    return np.bincount(np.asarray(vol).ravel(), minlength=levels).astype(np.uint64)


def otsu_threshold(hist) -> int:
    h = [int(v) for v in hist]
    total_n = sum(h)
    total_s = sum(v * c for v, c in enumerate(h))
    best_t, best_num, best_den = None, 0, 1
    n0 = s0 = 0
    for t in range(1, len(h)):
        n0 += h[t - 1]
        s0 += (t - 1) * h[t - 1]
        n1 = total_n - n0
        if n0 == 0 or n1 == 0:
            continue
        num = (total_n * s0 - n0 * total_s) ** 2
        den = n0 * n1
        if best_t is None or num * best_den > best_num * den:
            best_t, best_num, best_den = t, num, den
    if best_t is None:
        present = [v for v, c in enumerate(h) if c]
        return present[0] if present else 0
    return best_t
