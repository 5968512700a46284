"""Batch path (one launch per (radius, dtype) group over many volumes, as a
per-tile grid or a persistent tile queue) and the autotuner: every output
byte-identical to the oracle and to single-volume calls."""
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
@pytest.mark.parametrize("mode", [_lib.LNF_BATCH_GRID, _lib.LNF_BATCH_PERSISTENT])
def test_batch_full_mixed_workload_equals_single_calls(rule, mode):
    """The 64-volume mixed batch (axes 64..384, uint8/uint16, r in 1..3)."""
    jobs = ph.batch_jobs()
    vols = [ph.batch_volume(j, device="cuda") for j in jobs]
    with _filter(rule) as f:
        outs = f.batch([(v, j.radius) for v, j in zip(vols, jobs)], mode=mode)
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


@pytest.mark.parametrize("rule", ["mean9", "minvar9"])
@pytest.mark.parametrize("gate", [0, 900])
def test_batch_persistent_queue_small_and_repeated(rule, gate):
    """The tile queue hands out every tile exactly once, also when there are
    fewer tiles than resident workgroups, and the counters start at zero on
    every call (the table upload clears them)."""
    with _filter(rule, gate) as f:
        for rep in range(3):
            jobs = _small_jobs(300 + rep + gate, n=9)
            outs = f.batch([(torch.from_numpy(v).cuda(), r) for v, r in jobs],
                           mode=_lib.LNF_BATCH_PERSISTENT)
            for (vol, r), out in zip(jobs, outs):
                want = oracle.filter_volume(vol, r, RULES[rule][1], gate=gate)
                np.testing.assert_array_equal(out.cpu().numpy(), want, err_msg=f"{vol.shape} r={r}")


@pytest.mark.parametrize("geom", [_lib.LNF_GEOM_CROSS, _lib.LNF_GEOM_OFFSET_1,
                                  _lib.LNF_GEOM_OFFSET_2R1,
                                  _lib.LNF_GEOM_CROSS | _lib.LNF_GEOM_OFFSET_1])
@pytest.mark.parametrize("rule", ["mean9", "minvar9"])
def test_batch_geometry_variants_one_grid_per_group(geom, rule):
    """Geometry-variant contexts batch their jobs by group like the default
    geometry: the same bytes as single calls and as the oracle."""
    from paper_1807_03119_amd.api import Filter
    shape = oracle.CROSS if geom & _lib.LNF_GEOM_CROSS else oracle.BOX
    offset = (oracle.OFFSET_ONE if geom & _lib.LNF_GEOM_OFFSET_1 else
              oracle.OFFSET_TILE if geom & _lib.LNF_GEOM_OFFSET_2R1 else oracle.OFFSET_R)
    jobs = _small_jobs(400 + geom, n=8)
    with Filter(RULES[rule][0], 0, geometry=geom) as f:
        devs = [torch.from_numpy(v).cuda() for v, _ in jobs]
        outs = f.batch([(d, r) for d, (_, r) in zip(devs, jobs)])
        for d, (vol, r), out in zip(devs, jobs, outs):
            got = out.cpu().numpy()
            np.testing.assert_array_equal(got, f(d, r).cpu().numpy())
            want = oracle.filter_volume(vol, r, RULES[rule][1], shape=shape, offset=offset)
            np.testing.assert_array_equal(got, want, err_msg=f"{vol.shape} r={r}")
        assert _lib.lnf_filter_batch(f.handle, [(devs[0], torch.empty_like(devs[0]), 1)],
                                     mode=_lib.LNF_BATCH_PERSISTENT) == _lib.LNF_EINVAL


def test_batch_minvar9_wide_tile_groups():
    """MINVAR9 groups of large planes take the wide tile (the single-volume
    default there); same bytes as single calls."""
    vols = [ph.ct_u12((300, 280, 24), seed=2500 + i) for i in range(2)]
    vols.append(ph.random_volume((260, 256, 20), np.uint8, seed=2600))
    with _filter("minvar9") as f:
        devs = [torch.from_numpy(v).cuda() for v in vols]
        for r in (1, 3):
            outs = f.batch([(d, r) for d in devs])
            for d, v, o in zip(devs, vols, outs):
                np.testing.assert_array_equal(o.cpu().numpy(), f(d, r).cpu().numpy())
            np.testing.assert_array_equal(outs[0].cpu().numpy(),
                                          oracle.filter_volume(vols[0], r, oracle.MINVAR9))


@pytest.mark.parametrize("r", [2, 3])
def test_batch_minvar9_narrow_fallback_many_tiles_per_workgroup(r):
    """uint16 MINVAR9 tiles keep uint32 sums of squares and run again with
    fp64 sums when they load a value too large for them.  12-bit data with
    scattered bright voxels make some tiles of each kind; in the queue mode
    each workgroup takes several tiles in turn (the volume has about two
    tiles per resident workgroup).  Both launch modes, against the oracle."""
    rng = np.random.default_rng(90 + r)
    vol = rng.integers(0, 4096, (64, 512, 512), dtype=np.uint16)
    pts = rng.integers(0, [64, 512, 512], size=(40, 3))
    vol[pts[:, 0], pts[:, 1], pts[:, 2]] = 60000
    want = oracle.filter_volume(vol, r, oracle.MINVAR9)
    dev = torch.from_numpy(vol).cuda()
    with _filter("minvar9") as f:
        for mode in (_lib.LNF_BATCH_GRID, _lib.LNF_BATCH_PERSISTENT):
            out = f.batch([(dev, r)], mode=mode)[0]
            np.testing.assert_array_equal(out.cpu().numpy(), want, err_msg=f"mode {mode}")


def test_batch_call_captured_in_a_graph_replays_exactly():
    """A batch call (grid and queue mode) captured in a HIP graph: every replay,
    with eager batch calls and synchronisations between the replays, gives the
    eager bytes; the queue counters start at zero on every replay.  Captures
    beyond the reserved table slots are refused with LNF_EBUSY."""
    jobs = _small_jobs(700, n=9)
    other = _small_jobs(701, n=4)
    with _filter("mean9") as f:
        devs = [torch.from_numpy(v).cuda() for v, _ in jobs]
        want = [f(d, r).cpu().numpy() for d, (_, r) in zip(devs, jobs)]
        outs = [torch.empty_like(d) for d in devs]
        triples = [(d, o, r) for d, o, (_, r) in zip(devs, outs, jobs)]
        graphs = []
        for mode in (_lib.LNF_BATCH_GRID, _lib.LNF_BATCH_PERSISTENT):
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                rc = _lib.lnf_filter_batch(f.handle, triples, mode=mode)
            assert rc == _lib.LNF_OK
            graphs.append(g)
            for rep in range(3):
                for o in outs:
                    o.zero_()
                torch.cuda.synchronize()
                g.replay()
                torch.cuda.synchronize()
                for o, w, (v, r) in zip(outs, want, jobs):
                    np.testing.assert_array_equal(o.cpu().numpy(), w, err_msg=f"mode {mode} rep {rep} r={r}")
                # eager work between replays, on the same context
                eo = f.batch([(torch.from_numpy(v).cuda(), r) for v, r in other])
                torch.cuda.synchronize()
                np.testing.assert_array_equal(eo[0].cpu().numpy(), oracle.filter_volume(*other[0]))
        # two more captures fit the four reserved slots; the fifth is refused
        codes = []
        for _ in range(3):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                codes.append(_lib.lnf_filter_batch(f.handle, triples))
            graphs.append(g)
        assert codes == [_lib.LNF_OK, _lib.LNF_OK, _lib.LNF_EBUSY]
        del graphs
