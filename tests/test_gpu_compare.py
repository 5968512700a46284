"""The paper's comparison filters on the GPU (Section "Other Filters": mean,
sigma, Okada, entropy) against the oracle, element by element (bit-exact:
integer arithmetic; the entropy weights are the same fixed-point definition
evaluated independently on both sides)."""
import numpy as np
import pytest

from oracle import compare
from paper_1807_03119_amd import _lib
from paper_1807_03119_amd import phantom as ph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _filter(gate=0):
    from paper_1807_03119_amd.api import Filter
    return Filter(_lib.LNF_MEAN9, gate)


def _vols():
    return [ph.small_u8(1100, dims=(45, 37, 21)),
            ph.ct_u12((70, 41, 19), seed=2800),
            ph.random_volume((33, 9, 14), np.uint16, seed=21, kind="uniform"),
            ph.random_volume((17, 23, 6), np.uint8, seed=22, kind="low"),
            ph.random_volume((1, 1, 1), np.uint16, seed=23),
            ph.random_volume((2, 5, 3), np.uint8, seed=24)]


def _dev(v):
    return torch.from_numpy(np.ascontiguousarray(v)).cuda()


def _same(got, want, what):
    got = got.cpu().numpy()
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        z, y, x = bad[0]
        raise AssertionError(f"{what}: {len(bad)} mismatches, first at x={x} y={y} z={z}: "
                             f"got {got[z, y, x]} want {want[z, y, x]}")


def test_mean_filter_all_radii():
    with _filter() as f:
        for i, v in enumerate(_vols()):
            for r in (1, 2, 3, 4):
                _same(f.mean(_dev(v), r), compare.mean_filter(v, r), f"mean vol {i} r={r}")


def test_sigma_filter_explicit_and_automatic_width():
    with _filter() as f:
        for i, v in enumerate(_vols()):
            for r in (1, 2):
                for hw in (0, 7, 200):
                    out, used = f.sigma(_dev(v), r, hw)
                    assert used == hw
                    _same(out, compare.sigma_filter(v, r, hw), f"sigma vol {i} r={r} w={hw}")
            out, used = f.sigma(_dev(v), 1)
            assert used == compare.sigma_half_width(v), i
            _same(out, compare.sigma_filter(v, 1), f"sigma auto vol {i}")
        v = _vols()[1]
        for r in (3, 4):
            _same(f.sigma(_dev(v), r, 300)[0], compare.sigma_filter(v, r, 300), f"sigma r={r}")


def test_okada_filter():
    with _filter() as f:
        for i, v in enumerate(_vols()):
            for td in (0, 1, 15, 400, 1 << 20):
                _same(f.okada(_dev(v), td), compare.okada_filter(v, td), f"okada vol {i} t_d={td}")


def test_entropy_filter():
    with _filter() as f:
        for i, v in enumerate(_vols()):
            for r in (1, 2):
                for te in (-1.0, 0.05, 0.5, 2.0, 7.25, 1e6):
                    _same(f.entropy(_dev(v), r, te), compare.entropy_filter(v, r, te),
                          f"entropy vol {i} r={r} t_e={te}")
        v = _vols()[0]
        for r in (3, 4):
            _same(f.entropy(_dev(v), r, 3.0), compare.entropy_filter(v, r, 3.0), f"entropy r={r}")


def test_comparison_filters_gated():
    v = ph.ct_u12((40, 30, 12), seed=2900)
    with _filter(gate=1200) as f:
        d = _dev(v)
        _same(f.mean(d, 1), compare.mean_filter(v, 1, 1200), "gated mean")
        _same(f.sigma(d, 1, 60)[0], compare.sigma_filter(v, 1, 60, 1200), "gated sigma")
        _same(f.okada(d, 80), compare.okada_filter(v, 80, 1200), "gated okada")
        _same(f.entropy(d, 1, 0.5), compare.entropy_filter(v, 1, 0.5, 1200), "gated entropy")


def test_comparison_bad_arguments():
    with _filter() as f:
        v = torch.zeros((4, 4, 4), dtype=torch.uint16, device="cuda")
        o = torch.empty_like(v)
        dims = _lib.dims_of(v)
        assert _lib.lnf_filter_mean(f.handle, v, dims, _lib.LNF_U16, 0, o) == _lib.LNF_EINVAL
        assert _lib.lnf_filter_mean(f.handle, v, dims, _lib.LNF_U16, 1, v) == _lib.LNF_EINVAL
        assert _lib.lnf_filter_entropy(f.handle, v, dims, _lib.LNF_U16, 1, float("nan"), o) == \
            _lib.LNF_EINVAL
        assert _lib.lnf_filter_sigma(f.handle, v, dims, _lib.LNF_U16, 5, 1, o)[0] == _lib.LNF_EINVAL


def test_entropy_filter_z_strips():
    """A volume deep enough for several z-strips: each strip restarts the
    running z-sums of the separable entropy kernel."""
    v = ph.ct_u12((37, 21, 70), seed=2950)
    with _filter() as f:
        for r in (2, 3):
            _same(f.entropy(_dev(v), r, 2.5), compare.entropy_filter(v, r, 2.5), f"entropy r={r}")
