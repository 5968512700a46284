"""Batch path (one graph launch over many volumes) and the autotuner: every
output byte-identical to the oracle and to single-volume calls."""
import os
import tempfile

import numpy as np
import pytest

import oracle
from paper_1807_03119_amd import _lib
from paper_1807_03119_amd import phantom as ph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RULES = {"mean9": (_lib.LNF_MEAN9, oracle.MEAN9), "minvar9": (_lib.LNF_MINVAR9, oracle.MINVAR9)}


def _filter(rule, gate=0):
    from paper_1807_03119_amd.api import Filter
    return Filter(RULES[rule][0], gate)


def _small_jobs(seed, n=10):
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(n):
        dims = tuple(int(v) for v in rng.integers(1, 70, 3))
        if i == 0:
            dims = (1, 1, 1)
        if i == 1:
            dims = (3, 2, 1)
        dt = np.uint8 if i % 2 == 0 else np.uint16
        kind = ["uniform", "low", "extreme"][i % 3]
        jobs.append((ph.random_volume(dims, dt, seed=seed * 100 + i, kind=kind),
                     int(rng.integers(1, _lib.LNF_RADIUS_MAX + 1))))
    return jobs


@pytest.mark.parametrize("rule", ["mean9", "minvar9"])
@pytest.mark.parametrize("gate", [0, 60])
def test_batch_small_mixed_vs_oracle(rule, gate):
    jobs = _small_jobs(5 + gate)
    with _filter(rule, gate) as f:
        outs = f.batch([(torch.from_numpy(v).cuda(), r) for v, r in jobs])
        torch.cuda.synchronize()
    for (vol, r), out in zip(jobs, outs):
        want = oracle.filter_volume(vol, r, RULES[rule][1], gate=gate)
        np.testing.assert_array_equal(out.cpu().numpy(), want, err_msg=f"{vol.shape} r={r}")


@pytest.mark.parametrize("rule", ["mean9", "minvar9"])
def test_batch_full_mixed_workload_equals_single_calls(rule):
    """The 64-volume mixed batch (axes 64..384, uint8/uint16, r in 1..3)."""
    jobs = ph.batch_jobs()
    vols = [ph.batch_volume(j, device="cuda") for j in jobs]
    with _filter(rule) as f:
        outs = f.batch([(v, j.radius) for v, j in zip(vols, jobs)])
        singles = [f(v, j.radius) for v, j in zip(vols, jobs)]
        torch.cuda.synchronize()
        rng = np.random.default_rng(11)
        for i, (j, v, o, s) in enumerate(zip(jobs, vols, outs, singles)):
            assert torch.equal(o.view(torch.uint8), s.view(torch.uint8)), f"job {i} {j}"
            if i % 8 == 0:  # sampled oracle check on every eighth job
                nx, ny, nz = j.dims
                pts = np.stack([rng.integers(0, nx, 300), rng.integers(0, ny, 300),
                                rng.integers(0, nz, 300)], 1)
                vol = v.cpu().numpy()
                want = oracle.filter_points(vol, j.radius, pts, RULES[rule][1])
                got = o.cpu().numpy()[pts[:, 2], pts[:, 1], pts[:, 0]]
                np.testing.assert_array_equal(got.astype(np.uint32), want)


def test_batch_repeated_calls_reuse_slots():
    with _filter("mean9") as f:
        for rep in range(7):
            jobs = _small_jobs(100 + rep, n=5)
            outs = f.batch([(torch.from_numpy(v).cuda(), r) for v, r in jobs])
            for (vol, r), out in zip(jobs, outs):
                np.testing.assert_array_equal(out.cpu().numpy(), oracle.filter_volume(vol, r))


def test_batch_shared_input_different_radii():
    vol = torch.from_numpy(ph.small_u8(1001, dims=(40, 30, 20))).cuda()
    with _filter("mean9") as f:
        outs = f.batch([(vol, r) for r in (1, 2, 3, 4)])
        for r, o in zip((1, 2, 3, 4), outs):
            np.testing.assert_array_equal(o.cpu().numpy(),
                                          oracle.filter_volume(vol.cpu().numpy(), r))


def test_batch_errors_launch_nothing():
    with _filter("mean9") as f:
        h = f.handle
        a = torch.zeros((8, 8, 8), dtype=torch.uint16, device="cuda")
        b = torch.full((8, 8, 8), 7, dtype=torch.uint16, device="cuda")
        c = torch.full((8, 8, 8), 7, dtype=torch.uint16, device="cuda")
        assert _lib.lnf_filter_batch(h, [], n=0) == _lib.LNF_OK
        assert _lib.lnf_filter_batch(h, [(a, b, 1)], n=-1) == _lib.LNF_EINVAL
        assert _lib.lnf_filter_batch(h, [(a, b, 1)], n=_lib.LNF_BATCH_MAX + 1) == _lib.LNF_EINVAL
        # a good job next to a bad one: nothing may run
        assert _lib.lnf_filter_batch(h, [(a, b, 1), (a, c, 9)]) == _lib.LNF_EINVAL
        # two jobs writing the same output
        assert _lib.lnf_filter_batch(h, [(a, b, 1), (c, b, 2)]) == _lib.LNF_EINVAL
        # an output that is another job's input
        assert _lib.lnf_filter_batch(h, [(a, b, 1), (b, c, 2)]) == _lib.LNF_EINVAL
        torch.cuda.synchronize()
        assert int(b.to(torch.int32).sum()) == 7 * 512 and int(c.to(torch.int32).sum()) == 7 * 512


@pytest.mark.parametrize("rule", ["mean9", "minvar9"])
def test_tune_keeps_results_and_cache_roundtrip(rule):
    vol = torch.from_numpy(ph.ct_u12((96, 80, 72), seed=2400)).cuda()
    want = {r: oracle.filter_volume(vol.cpu().numpy(), r, RULES[rule][1]) for r in (1, 3)}
    with _filter(rule) as f:
        scratch = [torch.empty_like(vol) for _ in range(2)]
        f.tune([(vol, scratch[0], 1), (vol, scratch[1], 3)])
        for r in (1, 3):
            np.testing.assert_array_equal(f(vol, r).cpu().numpy(), want[r])
            np.testing.assert_array_equal(f.batch([(vol, r)])[0].cpu().numpy(), want[r])
        with tempfile.TemporaryDirectory() as d:
            path = os.path.join(d, "tune.txt")
            assert _lib.lnf_tune_save(f.handle, path) == 0
            lines = [ln for ln in open(path) if not ln.startswith("#")]
            assert len(lines) >= 2
            with _filter(rule) as g:
                assert _lib.lnf_tune_load(g.handle, path) == 0
                np.testing.assert_array_equal(g(vol, 3).cpu().numpy(), want[3])
            bad = os.path.join(d, "bad.txt")
            open(bad, "w").write("12 not numbers\n")
            assert _lib.lnf_tune_load(f.handle, bad) == _lib.LNF_EINVAL
            assert _lib.lnf_tune_load(f.handle, os.path.join(d, "missing")) == _lib.LNF_EINVAL


def test_batch_extreme_values_both_types():
    """Extreme-valued uint16 and uint8 volumes of every radius in one batch."""
    from paper_1807_03119_amd.api import Filter
    jobs = [(ph.random_volume((50, 40, 30), np.uint16, seed=60 + r, kind="extreme"), r)
            for r in (1, 2, 3, 4)]
    jobs += [(ph.random_volume((33, 20, 17), np.uint8, seed=70 + r, kind="extreme"), r)
             for r in (1, 4)]
    with Filter(_lib.LNF_MEAN9, 0) as f:
        outs = f.batch([(torch.from_numpy(v).cuda(), r) for v, r in jobs])
        for (v, r), o in zip(jobs, outs):
            np.testing.assert_array_equal(o.cpu().numpy(), oracle.filter_volume(v, r))
