"""Oracle of the first-hit pass and the surface pipeline.  TEST INFRASTRUCTURE
ONLY (see the package docstring).

The paper filters at the first point where each ray meets the surface, the
surface being where the data reach Otsu's threshold T (Section "Our Method";
eq. 1 for T).  For rays parallel to the z axis through pixel (x, y) that point
is the first voxel of the column, in the ray's direction, whose value is
>= T.  The filtered value there is the dense filter's value at that voxel.
"""
from __future__ import annotations

import numpy as np

from . import MEAN9, filter_points

MISS = 0xFFFFFFFF  # value reported for a ray that meets no voxel >= T


def first_hit(vol: np.ndarray, threshold: int, direction: int = 1) -> np.ndarray:
    """int64 [ny*nx, 3]: row y*nx + x holds (x, y, z) of the first voxel with
    value >= threshold met by the ray through (x, y) travelling towards +z
    (direction 1, from z = 0) or -z (direction -1, from z = nz - 1); z = -1
    where the column holds no such voxel.  Walks the slices in the ray's
    order, one plane at a time."""
    if direction not in (1, -1):
        raise ValueError("direction is 1 or -1")
    nz, ny, nx = vol.shape
    hit = np.full((ny, nx), -1, dtype=np.int64)
    order = range(nz) if direction == 1 else range(nz - 1, -1, -1)
    for z in order:
        newly = (hit < 0) & (vol[z].astype(np.int64) >= int(threshold))
        hit[newly] = z
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), hit.ravel()], 1)


def surface(vol: np.ndarray, r: int, threshold: int, direction: int = 1, rule: int = MEAN9,
            gate: int = 0):
    """(values uint32 [ny*nx], hits): the filter at each ray's first hit, MISS
    where the ray meets nothing."""
    hits = first_hit(vol, threshold, direction)
    vals = np.full(hits.shape[0], MISS, dtype=np.uint32)
    ok = hits[:, 2] >= 0
    if ok.any():
        vals[ok] = filter_points(vol, r, hits[ok], rule, gate)
    return vals, hits
