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
