"""Surface-point mode: values at listed voxels equal the oracle (and the dense
filter); points outside the volume are flagged, never read out of bounds."""
import numpy as np
import pytest

import oracle
from paper_1807_03119_amd import _lib
from paper_1807_03119_amd import phantom as ph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("rule,orule", [(_lib.LNF_MEAN9, oracle.MEAN9),
                                        (_lib.LNF_MINVAR9, oracle.MINVAR9)])
@pytest.mark.parametrize("gate", [0, 900])
def test_points_match_oracle(rule, orule, gate):
    from paper_1807_03119_amd.api import Filter
    vol = ph.ct_u12((70, 45, 33), seed=81)
    rng = np.random.default_rng(2)
    pts = np.concatenate([
        np.stack([rng.integers(0, 70, 500), rng.integers(0, 45, 500), rng.integers(0, 33, 500)], 1),
        np.array([[0, 0, 0], [69, 44, 32], [0, 44, 0], [69, 0, 32]])]).astype(np.int32)
    with Filter(rule, gate) as f:
        dev = torch.from_numpy(vol).cuda()
        for r in (1, 2, 3, 4):
            got = f.points(dev, r, torch.from_numpy(pts)).cpu().numpy().astype(np.uint32)
            want = oracle.filter_points(vol, r, pts.astype(np.int64), orule, gate=gate)
            np.testing.assert_array_equal(got, want)


def test_points_u8_and_outside_points():
    from paper_1807_03119_amd.api import Filter
    vol = ph.small_u8(1002, dims=(20, 10, 5))
    pts = np.array([[0, 0, 0], [19, 9, 4], [20, 0, 0], [-1, 3, 3], [5, 10, 1], [3, 3, 5]],
                   np.int32)
    with Filter() as f:
        got = f.points(torch.from_numpy(vol).cuda(), 2, torch.from_numpy(pts)).cpu().numpy()
    got = got.astype(np.uint32)
    want = oracle.filter_points(vol, 2, pts[:2].astype(np.int64))
    np.testing.assert_array_equal(got[:2], want)
    assert np.all(got[2:] == 0xFFFFFFFF)


@pytest.mark.parametrize("rule,orule", [(_lib.LNF_MEAN9, oracle.MEAN9),
                                        (_lib.LNF_MINVAR9, oracle.MINVAR9)])
def test_points_extremes_and_tiny_volumes(rule, orule):
    """Full-range values (sum and variance limits) and volumes smaller than a
    cluster, where every sample is clamped; every voxel of each volume."""
    from paper_1807_03119_amd.api import Filter
    vols = [ph.random_volume((19, 13, 11), np.uint16, seed=91, kind="extreme"),
            ph.random_volume((1, 1, 1), np.uint16, seed=92, kind="uniform"),
            ph.random_volume((2, 1, 3), np.uint8, seed=93, kind="uniform"),
            ph.random_volume((5, 7, 2), np.uint8, seed=94, kind="extreme")]
    with Filter(rule, 0) as f:
        for vol in vols:
            nz, ny, nx = vol.shape
            zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
            pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1).astype(np.int32)
            dev = torch.from_numpy(vol).cuda()
            for r in (1, 2, 3, 4):
                got = f.points(dev, r, torch.from_numpy(pts)).cpu().numpy().astype(np.uint32)
                want = oracle.filter_points(vol, r, pts.astype(np.int64), orule)
                np.testing.assert_array_equal(got, want, err_msg=f"{vol.shape} r={r}")
