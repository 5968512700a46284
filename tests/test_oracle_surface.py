"""Pins of the first-hit oracle (the paper's surface intersection point,
Section "Our Method") to facts other than itself: a ray-by-ray scan on tiny
volumes, thresholds that every voxel or no voxel reaches, a ramp with a closed
form hit, planted voxels, and the dense filter at the hit."""
import numpy as np
import pytest

import oracle
from oracle import surface


def _scan(vol, t, direction):
    """Each ray on its own: step along the column, stop at the first value >= t."""
    nz, ny, nx = vol.shape
    rows = []
    for y in range(ny):
        for x in range(nx):
            z = 0 if direction == 1 else nz - 1
            hit = -1
            while 0 <= z < nz:
                if int(vol[z, y, x]) >= t:
                    hit = z
                    break
                z += direction
            rows.append((x, y, hit))
    return np.array(rows, dtype=np.int64)


@pytest.mark.parametrize("direction", [1, -1])
@pytest.mark.parametrize("dtype,t", [(np.uint8, 200), (np.uint16, 40000), (np.uint16, 65535)])
def test_first_hit_equals_ray_scan(direction, dtype, t):
    rng = np.random.default_rng(int(t) + direction)
    hi = 256 if dtype == np.uint8 else 65536
    vol = rng.integers(0, hi, (9, 6, 7)).astype(dtype)
    np.testing.assert_array_equal(surface.first_hit(vol, t, direction), _scan(vol, t, direction))


def test_threshold_zero_and_above_max():
    vol = np.random.default_rng(3).integers(0, 4096, (5, 4, 6)).astype(np.uint16)
    h = surface.first_hit(vol, 0, 1)
    assert np.all(h[:, 2] == 0)
    assert np.all(surface.first_hit(vol, 0, -1)[:, 2] == 4)
    assert np.all(surface.first_hit(vol, 4096, 1)[:, 2] == -1)
    # rows enumerate the pixels x-fastest
    assert list(map(tuple, h[:7, :2])) == [(0, 0), (1, 0), (2, 0), (3, 0), (4, 0), (5, 0), (0, 1)]


@pytest.mark.parametrize("k,t", [(3, 7), (1, 0), (5, 40), (2, 200)])
def test_ramp_closed_form(k, t):
    """v = k z along every column: the forward ray first reaches t at z =
    ceil(t / k), the backward ray at the last slice whenever that one does."""
    nz = 30
    vol = np.broadcast_to((np.arange(nz) * k)[:, None, None], (nz, 3, 4)).astype(np.uint16)
    want = -(-t // k) if -(-t // k) < nz else -1
    assert np.all(surface.first_hit(vol, t, 1)[:, 2] == want)
    back = surface.first_hit(vol, t, -1)[:, 2]
    assert np.all(back == (nz - 1 if (nz - 1) * k >= t else -1))


def test_planted_voxels():
    vol = np.zeros((12, 3, 4), dtype=np.uint8)
    vol[7, 1, 2] = 90
    vol[3, 1, 2] = 50   # below the threshold: the ray passes through it
    vol[10, 2, 0] = 255
    vol[2, 2, 0] = 80
    h = surface.first_hit(vol, 60, 1).reshape(3, 4, 3)
    assert h[1, 2, 2] == 7 and h[2, 0, 2] == 2 and h[0, 0, 2] == -1
    hb = surface.first_hit(vol, 60, -1).reshape(3, 4, 3)
    assert hb[1, 2, 2] == 7 and hb[2, 0, 2] == 10


@pytest.mark.parametrize("rule", [oracle.MEAN9, oracle.MINVAR9])
def test_surface_values_are_the_dense_filter_at_the_hit(rule):
    from paper_1807_03119_amd import phantom as ph
    vol = ph.ct_u12((24, 20, 18), seed=61)
    t = int(np.percentile(vol, 80))
    dense = oracle.filter_volume(vol, 2, rule)
    vals, hits = surface.surface(vol, 2, t, 1, rule)
    for (x, y, z), v in zip(hits, vals):
        assert v == (surface.MISS if z < 0 else dense[z, y, x])
    assert (hits[:, 2] >= 0).any() and (hits[:, 2] < 0).any()
