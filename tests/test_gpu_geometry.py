"""Geometry variants on the GPU (eq. 2's cross clusters; diagonal offset 1 or
2r+1) against the oracle, element by element.  Bit-exact: integer sums, and
fp64 roundings that are exact by construction."""
import numpy as np
import pytest

import oracle
from paper_1807_03119_amd import _lib
from paper_1807_03119_amd import phantom as ph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (LNF_GEOM_* flags, oracle shape, oracle offset); the default geometry is the
# MEAN9 / MINVAR9 kernels' and is covered by the other tests
GEOMS = [
    (_lib.LNF_GEOM_OFFSET_1, oracle.BOX, oracle.OFFSET_ONE),
    (_lib.LNF_GEOM_OFFSET_2R1, oracle.BOX, oracle.OFFSET_TILE),
    (_lib.LNF_GEOM_CROSS, oracle.CROSS, oracle.OFFSET_R),
    (_lib.LNF_GEOM_CROSS | _lib.LNF_GEOM_OFFSET_1, oracle.CROSS, oracle.OFFSET_ONE),
    (_lib.LNF_GEOM_CROSS | _lib.LNF_GEOM_OFFSET_2R1, oracle.CROSS, oracle.OFFSET_TILE),
]
RULES = [(_lib.LNF_MEAN9, oracle.MEAN9), (_lib.LNF_MINVAR9, oracle.MINVAR9)]


def _filter(rule, geom, gate=0):
    from paper_1807_03119_amd.api import Filter
    return Filter(rule, gate, geometry=geom)


def _check(f, vol, r, shape, off, orule, gate=0, what=""):
    got = f(torch.from_numpy(np.ascontiguousarray(vol)).cuda(), r).cpu().numpy()
    want = oracle.filter_volume(vol, r, orule, gate, shape=shape, offset=off)
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        z, y, x = bad[0]
        raise AssertionError(f"{what}: {len(bad)} mismatches, first at x={x} y={y} z={z}: "
                             f"got {got[z, y, x]} want {want[z, y, x]}")


@pytest.mark.parametrize("geom,shape,off", GEOMS)
@pytest.mark.parametrize("rule,orule", RULES)
def test_geometry_small_shapes_all_radii(geom, shape, off, rule, orule):
    shapes = [(21, 17, 13), (1, 1, 1), (2, 9, 3), (40, 10, 6)]
    with _filter(rule, geom) as f:
        for i, dims in enumerate(shapes):
            for dtype in (np.uint8, np.uint16):
                vol = ph.random_volume(dims, dtype, seed=500 + 13 * i, kind="uniform")
                for r in (1, 2, 3, 4):
                    _check(f, vol, r, shape, off, orule,
                           what=f"geom {geom} rule {rule} {dims} {dtype.__name__} r={r}")


@pytest.mark.parametrize("geom,shape,off", GEOMS)
def test_geometry_phantom_and_extremes(geom, shape, off):
    vol = ph.ct_u12((70, 45, 33), seed=2600)
    ext = ph.random_volume((35, 27, 19), np.uint16, seed=9, kind="extreme")
    low = ph.random_volume((35, 27, 19), np.uint8, seed=10, kind="low")  # many variance ties
    for rule, orule in RULES:
        with _filter(rule, geom) as f:
            for r in (1, 2, 3):
                _check(f, vol, r, shape, off, orule, what=f"phantom geom {geom} r={r}")
            for v in (ext, low):
                _check(f, v, 2, shape, off, orule, what=f"extremes geom {geom}")


def test_geometry_gate_batch_and_otsu():
    geom, shape, off = GEOMS[2]  # crosses at offset r
    vol = ph.ct_u12((50, 30, 20), seed=2700)
    with _filter(_lib.LNF_MEAN9, geom, gate=1000) as f:
        _check(f, vol, 2, shape, off, oracle.MEAN9, gate=1000, what="gated cross")
    jobs = [(ph.small_u8(80 + r, dims=(23, 19, 11)), r) for r in (1, 2)]
    jobs += [(ph.ct_u12((31, 17, 29), seed=90 + r), r) for r in (1, 3)]
    with _filter(_lib.LNF_MINVAR9, geom) as f:
        outs = f.batch([(torch.from_numpy(v).cuda(), r) for v, r in jobs])
        for (v, r), o in zip(jobs, outs):
            np.testing.assert_array_equal(
                o.cpu().numpy(), oracle.filter_volume(v, r, oracle.MINVAR9, shape=shape, offset=off))
    with _filter(_lib.LNF_MEAN9, geom) as f:
        out, t = f.filter_otsu(torch.from_numpy(vol).cuda(), 1)
        assert t == oracle.otsu_threshold(oracle.histogram(vol))
        np.testing.assert_array_equal(
            out.cpu().numpy(), oracle.filter_volume(vol, 1, oracle.MEAN9, t, shape=shape, offset=off))


def test_geometry_points_rejected():
    with _filter(_lib.LNF_MEAN9, _lib.LNF_GEOM_CROSS) as f:
        vol = torch.zeros((8, 8, 8), dtype=torch.uint16, device="cuda")
        xyz = torch.zeros((1, 3), dtype=torch.int32, device="cuda")
        out = torch.zeros(1, dtype=torch.int32, device="cuda")
        rc = _lib.lnf_filter_points(f.handle, vol, _lib.dims_of(vol), _lib.LNF_U16, 1, xyz, 1, out)
        assert rc == _lib.LNF_EINVAL


@pytest.mark.parametrize("geom,shape,off", GEOMS)
def test_geometry_z_strips(geom, shape, off):
    """Explicit z-strip depths, ragged and down to one slice: every strip
    restarts the z-sums and the pending-output rings of the per-plane tile."""
    vol = ph.ct_u12((37, 21, 45), seed=2800)
    for rule, orule in RULES:
        with _filter(rule, geom) as f:
            for r in (1, 2):
                want = oracle.filter_volume(vol, r, orule, shape=shape, offset=off)
                for zs in (1, 3, 7, 16, 44):
                    got = f(torch.from_numpy(vol).cuda(), r, zs=zs).cpu().numpy()
                    if not np.array_equal(got, want):
                        bad = np.argwhere(got != want)
                        raise AssertionError(f"geom {geom} rule {rule} r={r} zs={zs}: "
                                             f"{len(bad)} mismatches, first {bad[0]}")
