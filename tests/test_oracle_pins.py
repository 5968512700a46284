"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself or retypes its arithmetic: each
check is a hand-derived fixture, a closed form, an invariant, a library
routine, or a brute force written in a different formulation (centre list
spelled out, exact rational means and centred variances) on tiny inputs.

Filter definition: paper Section "Our Method", eqs. 2-3 and the figure of the
nine average clusters; threshold: eq. 1.
"""
from fractions import Fraction
import itertools
import os

import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_1807_03119_amd import phantom as ph

DTYPES = [np.uint8, np.uint16]


def _read_golden(path):
    rows = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


# ---------------------------------------------------------------------------
# independent brute force: explicit centres, exact rational statistics
# ---------------------------------------------------------------------------

def _centres(r):
    # S_0, then the eight diagonal neighbours: x varies fastest, then y, then z
    base = [(0, 0, 0), (-1, -1, -1), (1, -1, -1), (-1, 1, -1), (1, 1, -1),
            (-1, -1, 1), (1, -1, 1), (-1, 1, 1), (1, 1, 1)]
    return [(r * a, r * b, r * c) for a, b, c in base]


def _fraction_filter(vol, r, rule):
    nz, ny, nx = vol.shape
    out = np.zeros_like(vol)
    cube = range(-r, r + 1)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        means, variances = [], []
        for cx, cy, cz in _centres(r):
            vals = [int(vol[min(max(z + cz + c, 0), nz - 1),
                            min(max(y + cy + b, 0), ny - 1),
                            min(max(x + cx + a, 0), nx - 1)])
                    for c in cube for b in cube for a in cube]
            m = Fraction(sum(vals), len(vals))
            means.append(m)
            variances.append(sum((v - m) ** 2 for v in vals) / len(vals))
        if rule == oracle.MEAN9:
            val = round(sum(means) / 9)
        else:
            best = min(range(9), key=lambda k: (variances[k], k))
            val = round(means[best])
        out[z, y, x] = val
    return out


@pytest.mark.parametrize("rule", [oracle.MEAN9, oracle.MINVAR9])
@pytest.mark.parametrize("r", [1, 2])
@pytest.mark.parametrize("dims,kind,dtype", [
    ((5, 4, 3), "uniform", np.uint8),
    ((1, 2, 3), "uniform", np.uint16),
    ((6, 3, 4), "low", np.uint8),
    ((4, 4, 4), "extreme", np.uint16),
    ((7, 1, 1), "uniform", np.uint16),
])
def test_bruteforce_fractions(rule, r, dims, kind, dtype):
    vol = ph.random_volume(dims, dtype, seed=11 + r, kind=kind)
    got = oracle.filter_volume(vol, r, rule)
    want = _fraction_filter(vol, r, rule)
    np.testing.assert_array_equal(got, want)


def test_bruteforce_fractions_r3_odd():
    vol = ph.random_volume((3, 5, 2), np.uint8, seed=5, kind="low")
    for rule in (oracle.MEAN9, oracle.MINVAR9):
        np.testing.assert_array_equal(oracle.filter_volume(vol, 3, rule),
                                      _fraction_filter(vol, 3, rule))


# ---------------------------------------------------------------------------
# closed forms (hand-derived fixtures)
# ---------------------------------------------------------------------------

def test_step_edge_golden(golden_dir):
    rows = _read_golden(os.path.join(golden_dir, "step_edge_mean9_r1.txt"))
    nx, x0 = 12, 6
    vol = np.full((5, 4, nx), 20, dtype=np.uint8)
    vol[:, :, x0:] = 220
    out = oracle.filter_volume(vol, 1)
    for x, want in rows:
        col = out[:, :, x0 + int(x)]
        assert np.all(col == int(want)), (x, col)


def test_impulse_golden(golden_dir):
    rows = _read_golden(os.path.join(golden_dir, "impulse_mean9_r1.txt"))
    vol = np.zeros((15, 15, 15), dtype=np.uint16)
    c = 7
    vol[c, c, c] = 2700
    out = oracle.filter_volume(vol, 1)
    for dx, dy, dz, want in rows:
        dx, dy, dz = int(dx), int(dy), int(dz)
        # every sign and axis permutation of the offset gives the same value
        for perm in itertools.permutations((dx, dy, dz)):
            for sg in itertools.product((-1, 1), repeat=3):
                px, py, pz = (c + s * d for s, d in zip(sg, perm))
                assert out[pz, py, px] == int(want), (perm, sg)


def test_otsu_golden(golden_dir):
    rows = _read_golden(os.path.join(golden_dir, "otsu_small.txt"))
    counts = [int(v) for v in rows[0][1:]]
    assert oracle.otsu_threshold(counts) == int(rows[1][1])


def _kernel_k(r):
    """The nine-cluster sum as one convolution kernel: the centre box plus, along
    every axis, the two boxes shifted by -r and +r (a box of radius 2r with the
    centre counted twice)."""
    m = 2 * r + 1
    w = 4 * r + 1
    k = np.zeros((w, w, w), dtype=np.int64)
    k[r:r + m, r:r + m, r:r + m] += 1
    c1 = np.ones(w, dtype=np.int64)
    c1[2 * r] += 1
    k += c1[:, None, None] * c1[None, :, None] * c1[None, None, :]
    return k


@pytest.mark.parametrize("r", [1, 2, 3])
@pytest.mark.parametrize("dtype", DTYPES)
def test_mean9_equals_convolution_with_k(r, dtype):
    k = _kernel_k(r)
    n = (2 * r + 1) ** 3
    assert k.sum() == 9 * n
    for dims, kind in (((9, 7, 5), "uniform"), ((16, 12, 10), "extreme"), ((3, 11, 4), "uniform")):
        vol = ph.random_volume(dims, dtype, seed=100 * r + len(dims), kind=kind)
        s = ndimage.convolve(vol.astype(np.int64), k, mode="nearest")
        want = np.vectorize(lambda t: round(Fraction(int(t), 9 * n)))(s)
        np.testing.assert_array_equal(oracle.filter_volume(vol, r), want.astype(dtype))


@pytest.mark.parametrize("r", [1, 2, 3])
def test_step_edge_closed_form_all_r(r):
    """MEAN9 across a step a->b: 1D weights w(t) = M^2*[|t|<=r] + (2M)^2*([|t|<=2r] + [t==0]).
    MINVAR9 reproduces the step exactly: some cluster always lies on one side."""
    m = 2 * r + 1
    t = np.arange(-2 * r, 2 * r + 1)
    w = m * m * (np.abs(t) <= r) + (2 * m) ** 2 * ((np.abs(t) <= 2 * r).astype(int) + (t == 0))
    assert w.sum() == 9 * m ** 3
    a, b = 300, 3700
    nx, x0 = 8 * r + 4, 4 * r + 2
    vol = np.full((3, 4, nx), a, dtype=np.uint16)
    vol[:, :, x0:] = b
    out = oracle.filter_volume(vol, r)
    outv = oracle.filter_volume(vol, r, oracle.MINVAR9)
    for x in range(2 * r, nx - 2 * r):
        num = sum(int(wt) * (a if x + int(tt) < x0 else b) for tt, wt in zip(t, w))
        assert np.all(out[:, :, x] == round(Fraction(num, 9 * m ** 3)))
        assert np.all(outv[:, :, x] == (a if x < x0 else b))


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("rule", [oracle.MEAN9, oracle.MINVAR9])
@pytest.mark.parametrize("dtype", DTYPES)
def test_constant_volume_unchanged(rule, dtype):
    top = int(np.iinfo(dtype).max)
    for dims in ((1, 1, 1), (1, 5, 3), (6, 2, 1), (7, 7, 7)):
        for c in (0, 1, 77, top):
            vol = np.full(dims[::-1], c, dtype=dtype)
            for r in (1, 2, 4):
                assert np.all(oracle.filter_volume(vol, r, rule) == c)


@pytest.mark.parametrize("r", [1, 2])
def test_affine_ramp_reproduced(r):
    nx, ny, nz = 20, 18, 16
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    vol = (100 + 3 * x + 5 * y + 7 * z).astype(np.uint16)
    out = oracle.filter_volume(vol, r)
    e = 2 * r
    np.testing.assert_array_equal(out[e:-e, e:-e, e:-e], vol[e:-e, e:-e, e:-e])


@pytest.mark.parametrize("rule", [oracle.MEAN9, oracle.MINVAR9])
@pytest.mark.parametrize("r", [1, 2, 3])
def test_output_within_window_range(rule, r):
    vol = ph.small_u8(seed=1001, dims=(24, 20, 18))
    out = oracle.filter_volume(vol, r, rule)
    w = 4 * r + 1
    lo = ndimage.minimum_filter(vol, size=w, mode="nearest")
    hi = ndimage.maximum_filter(vol, size=w, mode="nearest")
    assert np.all(out >= lo) and np.all(out <= hi)


def _minvar_tie_mask(vol, r):
    """Voxels where several clusters share the least variance but differ in mean
    (there the lowest-index rule makes the result orientation dependent)."""
    nz, ny, nx = vol.shape
    n = (2 * r + 1) ** 3
    mask = np.zeros(vol.shape, dtype=bool)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        s, q = oracle.cluster_stats(vol, r, x, y, z)
        v = [n * int(qq) - int(ss) ** 2 for ss, qq in zip(s, q)]
        mv = min(v)
        sums = {int(s[k]) for k in range(9) if v[k] == mv}
        mask[z, y, x] = len(sums) > 1
    return mask


@pytest.mark.parametrize("rule", [oracle.MEAN9, oracle.MINVAR9])
@pytest.mark.parametrize("r", [1, 2])
def test_flip_and_transpose_equivariance(rule, r):
    vol = ph.small_u8(seed=1002, dims=(14, 14, 14))
    out = oracle.filter_volume(vol, r, rule)
    ties = _minvar_tie_mask(vol, r) if rule == oracle.MINVAR9 else np.zeros(vol.shape, bool)
    ops = [lambda a: a[::-1], lambda a: a[:, ::-1], lambda a: a[:, :, ::-1],
           lambda a: a.transpose(0, 2, 1), lambda a: a.transpose(2, 1, 0),
           lambda a: a.transpose(1, 0, 2)[::-1, :, ::-1]]
    for op in ops:
        got = oracle.filter_volume(np.ascontiguousarray(op(vol)), r, rule)
        want = op(out)
        keep = ~op(ties)
        np.testing.assert_array_equal(got[keep], want[keep])
    assert ties.mean() < 0.01


@pytest.mark.parametrize("rule", [oracle.MEAN9, oracle.MINVAR9])
@pytest.mark.parametrize("r", [1, 3])
def test_shift_and_complement(rule, r):
    vol = ph.small_u8(seed=1003, dims=(16, 13, 11))
    out = oracle.filter_volume(vol, r, rule).astype(np.int64)
    shifted = (vol.astype(np.uint16) + 1000)
    np.testing.assert_array_equal(oracle.filter_volume(shifted, r, rule).astype(np.int64),
                                  out + 1000)
    comp = (255 - vol).astype(np.uint8)
    np.testing.assert_array_equal(oracle.filter_volume(comp, r, rule).astype(np.int64),
                                  255 - out)


def test_gate_writes_zero_below_threshold():
    """Outputs below T become 0; an output equal to T is kept (thresholds
    include values the output takes)."""
    vol = ph.small_u8(seed=1004, dims=(16, 16, 16))
    for rule in (oracle.MEAN9, oracle.MINVAR9):
        plain = oracle.filter_volume(vol, 1, rule)
        taken = (int(plain.min()), int(np.median(plain)), int(plain.max()))
        assert all(np.count_nonzero(plain == t) for t in taken)
        for t in (0, 1, 50, 101, 255, 256) + taken:
            gated = oracle.filter_volume(vol, 1, rule, gate=t)
            want = np.where(plain >= t, plain, 0)
            np.testing.assert_array_equal(gated, want)


def test_points_match_volume():
    vol = ph.ct_u12((33, 17, 9), seed=7)
    rng = np.random.default_rng(3)
    pts = np.stack([rng.integers(0, 33, 200), rng.integers(0, 17, 200), rng.integers(0, 9, 200)], 1)
    for rule in (oracle.MEAN9, oracle.MINVAR9):
        full = oracle.filter_volume(vol, 2, rule, gate=1100)
        got = oracle.filter_points(vol, 2, pts, rule, gate=1100)
        np.testing.assert_array_equal(got, full[pts[:, 2], pts[:, 1], pts[:, 0]])


def test_cluster_stats_sum_matches_box_filter():
    """Each cluster sum equals a (2r+1)^3 box sum (scipy uniform filter in exact
    integers via convolution) taken at the cluster's centre."""
    vol = ph.random_volume((10, 9, 8), np.uint16, seed=21)
    for r in (1, 2):
        box = ndimage.convolve(vol.astype(np.int64), np.ones((2 * r + 1,) * 3, np.int64),
                               mode="nearest")
        sq = ndimage.convolve(vol.astype(np.int64) ** 2, np.ones((2 * r + 1,) * 3, np.int64),
                              mode="nearest")
        for (x, y, z) in ((r, r, r), (5, 4, 3), (9 - r, 8 - r, 7 - r)):
            s, q = oracle.cluster_stats(vol, r, x, y, z)
            for k, (cx, cy, cz) in enumerate(_centres(r)):
                assert int(s[k]) == box[z + cz, y + cy, x + cx]
                assert int(q[k]) == sq[z + cz, y + cy, x + cx]


def test_rejects_bad_arguments():
    vol = np.zeros((4, 4, 4), np.uint8)
    with pytest.raises(ValueError):
        oracle.filter_volume(vol, 0)
    with pytest.raises(ValueError):
        oracle.filter_volume(vol, 9)
    with pytest.raises(TypeError):
        oracle.filter_volume(vol.astype(np.int32), 1)
    with pytest.raises(ValueError):
        oracle.filter_points(vol, 1, [[4, 0, 0]])


# ---------------------------------------------------------------------------
# Otsu (eq. 1)
# ---------------------------------------------------------------------------

def _otsu_eq1_bruteforce(hist):
    """Argmin over T of w0*var0 + w1*var1 (eq. 1) in exact fractions, lowest T on ties."""
    levels = [v for v, c in enumerate(hist) for _ in range(int(c))]
    n = len(levels)
    best = None
    for t in range(1, len(hist)):
        c0 = [v for v in levels if v < t]
        c1 = [v for v in levels if v >= t]
        if not c0 or not c1:
            continue

        def var(c):
            m = Fraction(sum(c), len(c))
            return sum((v - m) ** 2 for v in c) / len(c)
        sw = Fraction(len(c0), n) * var(c0) + Fraction(len(c1), n) * var(c1)
        if best is None or sw < best[0]:
            best = (sw, t)
    return None if best is None else best[1]


def test_otsu_matches_eq1_bruteforce():
    rng = np.random.default_rng(9)
    for trial in range(40):
        levels = int(rng.integers(2, 24))
        hist = rng.integers(0, 6, levels)
        if trial % 3 == 0:
            hist[rng.integers(0, levels, levels // 2)] = 0
        want = _otsu_eq1_bruteforce(hist)
        got = oracle.otsu_threshold(hist)
        if want is None:
            present = np.nonzero(hist)[0]
            assert got == (int(present[0]) if len(present) else 0)
        else:
            assert got == want


def test_otsu_two_levels_and_degenerate():
    for a, b in ((0, 1), (20, 220), (3, 4095)):
        h = np.zeros(b + 1, np.int64)
        h[a] = 5
        h[b] = 9
        assert oracle.otsu_threshold(h) == a + 1
    h = np.zeros(256, np.int64)
    h[42] = 10
    assert oracle.otsu_threshold(h) == 42
    assert oracle.otsu_threshold(np.zeros(16, np.int64)) == 0


def test_otsu_separates_bimodal_phantom():
    vol = ph.small_u8()
    t = oracle.otsu_threshold(oracle.histogram(vol))
    # background ~20 (sigma 20) and objects 40..220: the cut lies between the modes
    assert 25 < t < 140


# ---------------------------------------------------------------------------
# geometry variants: eq. 2's cross clusters and the diagonal offset d
# ---------------------------------------------------------------------------

GEOMETRIES = [(shape, off) for shape in (oracle.BOX, oracle.CROSS)
              for off in (oracle.OFFSET_R, oracle.OFFSET_ONE, oracle.OFFSET_TILE)]


def _offset_distance(r, off):
    return {oracle.OFFSET_R: r, oracle.OFFSET_ONE: 1, oracle.OFFSET_TILE: 2 * r + 1}[off]


def _members(r, shape):
    """Member offsets of one cluster, with multiplicity: the cube, or the three
    axis lines of eq. 2 (so the centre appears three times)."""
    span = range(-r, r + 1)
    if shape == oracle.BOX:
        return [(a, b, c) for c in span for b in span for a in span]
    return ([(t, 0, 0) for t in span] + [(0, t, 0) for t in span] + [(0, 0, t) for t in span])


def _fraction_filter_geom(vol, r, rule, shape, off):
    nz, ny, nx = vol.shape
    d = _offset_distance(r, off)
    members = _members(r, shape)
    out = np.zeros_like(vol)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        means, variances = [], []
        for cx, cy, cz in _centres(d):
            vals = [int(vol[min(max(z + cz + c, 0), nz - 1),
                            min(max(y + cy + b, 0), ny - 1),
                            min(max(x + cx + a, 0), nx - 1)]) for a, b, c in members]
            m = Fraction(sum(vals), len(vals))
            means.append(m)
            variances.append(sum((v - m) ** 2 for v in vals) / len(vals))
        if rule == oracle.MEAN9:
            val = round(sum(means) / 9)
        else:
            best = min(range(9), key=lambda k: (variances[k], k))
            val = round(means[best])
        out[z, y, x] = val
    return out


@pytest.mark.parametrize("shape,off", GEOMETRIES)
@pytest.mark.parametrize("rule", [oracle.MEAN9, oracle.MINVAR9])
@pytest.mark.parametrize("r", [1, 2])
def test_geometry_bruteforce_fractions(shape, off, rule, r):
    for i, (dims, kind, dtype) in enumerate([((5, 4, 3), "uniform", np.uint8),
                                             ((4, 3, 4), "low", np.uint16),
                                             ((3, 3, 3), "extreme", np.uint16)]):
        vol = ph.random_volume(dims, dtype, seed=100 + 7 * i + r, kind=kind)
        got = oracle.filter_volume(vol, r, rule, shape=shape, offset=off)
        want = _fraction_filter_geom(vol, r, rule, shape, off)
        np.testing.assert_array_equal(got, want, err_msg=f"{dims} {kind} shape {shape} off {off}")


def _stamped_kernel(r, shape, off):
    """Convolution kernel of the nine-cluster sum, built by stamping the cluster
    shape at the nine centres (library convolution, not the oracle's loops)."""
    d = _offset_distance(r, off)
    h = d + r
    k = np.zeros((2 * h + 1,) * 3, dtype=np.int64)
    stamp = np.zeros((2 * r + 1,) * 3, dtype=np.int64)
    if shape == oracle.BOX:
        stamp[...] = 1
    else:
        stamp[r, r, :] += 1  # x line (arrays are [z, y, x])
        stamp[r, :, r] += 1  # y line
        stamp[:, r, r] += 1  # z line
    for sz, sy, sx in [(0, 0, 0)] + list(itertools.product((-1, 1), repeat=3)):
        cz, cy, cx = h + sz * d, h + sy * d, h + sx * d
        k[cz - r:cz + r + 1, cy - r:cy + r + 1, cx - r:cx + r + 1] += stamp
    return k


@pytest.mark.parametrize("shape,off", GEOMETRIES)
@pytest.mark.parametrize("r", [1, 2, 3])
def test_geometry_mean9_equals_stamped_convolution(shape, off, r):
    vol = ph.small_u8(1000 + r, dims=(19, 17, 13)).astype(np.uint16) * 16
    k = _stamped_kernel(r, shape, off)
    n = (2 * r + 1) ** 3 if shape == oracle.BOX else 3 * (2 * r + 1)
    assert k.sum() == 9 * n
    s = ndimage.convolve(vol.astype(np.int64), k, mode="nearest")  # nearest = clamp to edge
    want = ((2 * s + 9 * n) // (18 * n)).astype(np.uint16)
    got = oracle.filter_volume(vol, r, oracle.MEAN9, shape=shape, offset=off)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("name,shape,off,h", [
    ("impulse_mean9_cross_r1.txt", oracle.CROSS, oracle.OFFSET_R, 8100),
    ("impulse_mean9_box_d3_r1.txt", oracle.BOX, oracle.OFFSET_TILE, 24300),
])
def test_geometry_impulse_golden(golden_dir, name, shape, off, h):
    rows = _read_golden(os.path.join(golden_dir, name))
    vol = np.zeros((21, 21, 21), dtype=np.uint16)
    c = 10
    vol[c, c, c] = h
    out = oracle.filter_volume(vol, 1, oracle.MEAN9, shape=shape, offset=off)
    for dx, dy, dz, want in rows:
        dx, dy, dz = int(dx), int(dy), int(dz)
        for perm in itertools.permutations((dx, dy, dz)):
            for sg in itertools.product((-1, 1), repeat=3):
                px, py, pz = (c + s * d for s, d in zip(sg, perm))
                assert out[pz, py, px] == int(want), (name, perm, sg)


@pytest.mark.parametrize("shape,off", GEOMETRIES)
@pytest.mark.parametrize("rule", [oracle.MEAN9, oracle.MINVAR9])
def test_geometry_constant_and_ramp(shape, off, rule):
    for dims, c in (((1, 1, 1), 9), ((7, 5, 6), 4095)):
        vol = np.full(dims[::-1], c, dtype=np.uint16)
        np.testing.assert_array_equal(oracle.filter_volume(vol, 2, rule, shape=shape, offset=off),
                                      vol)
    if rule == oracle.MEAN9:
        # point-symmetric kernel: an affine ramp is reproduced away from the faces
        r = 2
        d = _offset_distance(r, off)
        z, y, x = np.meshgrid(np.arange(20), np.arange(18), np.arange(22), indexing="ij")
        vol = (100 + 3 * x + 5 * y + 7 * z).astype(np.uint16)
        out = oracle.filter_volume(vol, r, rule, shape=shape, offset=off)
        m = d + r
        np.testing.assert_array_equal(out[m:-m, m:-m, m:-m], vol[m:-m, m:-m, m:-m])


def test_geometry_offset_one_is_default_at_r1():
    vol = ph.small_u8(1001, dims=(12, 11, 10))
    for shape in (oracle.BOX, oracle.CROSS):
        for rule in (oracle.MEAN9, oracle.MINVAR9):
            np.testing.assert_array_equal(
                oracle.filter_volume(vol, 1, rule, shape=shape, offset=oracle.OFFSET_ONE),
                oracle.filter_volume(vol, 1, rule, shape=shape, offset=oracle.OFFSET_R))
