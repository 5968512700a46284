"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

Integer work, so the bar is equality of every output byte.  Small volumes are
compared in full; the full-size workloads on sampled voxels (random points
plus faces, edges and corners) that the oracle evaluates one by one.
"""
import numpy as np
import pytest

import oracle
from paper_1807_03119_amd import _lib
from paper_1807_03119_amd import phantom as ph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RULES = {"mean9": (_lib.LNF_MEAN9, oracle.MEAN9), "minvar9": (_lib.LNF_MINVAR9, oracle.MINVAR9)}


@pytest.fixture(scope="module")
def filters():
    from paper_1807_03119_amd.api import Filter
    fs = {}

    def get(rule, gate=0):
        key = (rule, gate)
        if key not in fs:
            fs[key] = Filter(RULES[rule][0], gate)
        return fs[key]
    yield get
    for f in fs.values():
        f.close()


def _gpu(filt, vol, r, **kw):
    dev = torch.from_numpy(np.ascontiguousarray(vol)).cuda()
    out = filt(dev, r, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _assert_same(got, want, vol, r, what):
    if np.array_equal(got, want):
        return
    bad = np.argwhere(got != want)
    z, y, x = (int(v) for v in bad[0])
    s, q = oracle.cluster_stats(vol, r, x, y, z)
    raise AssertionError(f"{what}: {len(bad)} mismatches; first at (x,y,z)=({x},{y},{z}) "
                         f"gpu={got[z, y, x]} oracle={want[z, y, x]} sums={s.tolist()} "
                         f"sq={q.tolist()}")


def _sample_points(dims, m, seed):
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    pts = [np.stack([rng.integers(0, nx, m), rng.integers(0, ny, m), rng.integers(0, nz, m)], 1)]
    edge = []
    def around(n):
        return sorted({min(max(v, 0), n - 1) for v in (0, 1, n // 2, n - 2, n - 1)})
    for x in around(nx):
        for y in around(ny):
            for z in around(nz):
                edge.append((x, y, z))
    pts.append(np.array(edge, dtype=np.int64))
    # whole face rows through the volume
    k = min(nx, 512)
    pts.append(np.stack([np.arange(k), np.zeros(k, np.int64), np.full(k, nz - 1)], 1))
    k = min(ny, 512)
    pts.append(np.stack([np.full(k, nx - 1), np.arange(k), np.zeros(k, np.int64)], 1))
    return np.concatenate(pts).astype(np.int64)


# ---------------------------------------------------------------------------
# small volumes, compared in full
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("rule", ["mean9", "minvar9"])
@pytest.mark.parametrize("r", [1, 2, 3])
@pytest.mark.parametrize("seed", [1000, 1001, 1002])
def test_small_phantom_64cube_u8(filters, rule, r, seed):
    vol = ph.small_u8(seed)
    got = _gpu(filters(rule), vol, r)
    want = oracle.filter_volume(vol, r, RULES[rule][1])
    _assert_same(got, want, vol, r, f"64^3 u8 seed {seed} r={r} {rule}")


# odd and even row lengths: even ones take the paired staging, whose tiles at
# the x faces substitute the edge element (tiles covering one face or both)
ODD_DIMS = [(1, 1, 1), (1, 1, 7), (7, 1, 1), (1, 9, 1), (2, 3, 5), (13, 11, 7), (17, 1, 3),
            (65, 17, 9), (64, 16, 8), (63, 15, 31), (97, 35, 21), (4, 7, 3), (6, 5, 9),
            (34, 9, 11), (66, 20, 10), (128, 3, 5), (96, 35, 21)]


@pytest.mark.parametrize("rule", ["mean9", "minvar9"])
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
@pytest.mark.parametrize("kind", ["uniform", "extreme", "low"])
def test_odd_shapes_all_radii(filters, rule, dtype, kind):
    for i, dims in enumerate(ODD_DIMS):
        vol = ph.random_volume(dims, dtype, seed=31 * i + 7, kind=kind)
        for r in range(1, _lib.LNF_RADIUS_MAX + 1):
            got = _gpu(filters(rule), vol, r)
            want = oracle.filter_volume(vol, r, RULES[rule][1])
            _assert_same(got, want, vol, r, f"{dims} {dtype.__name__} {kind} r={r} {rule}")


@pytest.mark.parametrize("rule", ["mean9", "minvar9"])
def test_ct_phantom_u12_medium(filters, rule):
    vol = ph.ct_u12((130, 67, 45), seed=2100)
    for r in (1, 2, 3, 4):
        got = _gpu(filters(rule), vol, r)
        want = oracle.filter_volume(vol, r, RULES[rule][1])
        _assert_same(got, want, vol, r, f"130x67x45 u12 r={r} {rule}")


@pytest.mark.parametrize("rule", ["mean9", "minvar9"])
def test_tile_and_strip_independence(filters, rule):
    """Every z-strip depth and tile variant gives the same bytes (and the oracle's)."""
    vol = ph.ct_u12((96, 80, 72), seed=2200)
    rc, oc = RULES[rule]
    for r in (1, 2, 3, 4):
        want = oracle.filter_volume(vol, r, oc)
        nvar = _lib.lnf_tile_variants(rc, _lib.LNF_U16, r)
        for variant in range(nvar):
            for zs in (1, 2, 5, 16, 71, 72, 0):
                got = _gpu(filters(rule), vol, r, variant=variant, zs=zs)
                _assert_same(got, want, vol, r, f"variant {variant} zs {zs} r={r} {rule}")


@pytest.mark.parametrize("rule", ["mean9", "minvar9"])
def test_gate(filters, rule):
    vol = ph.small_u8(1000)
    t_otsu = oracle.otsu_threshold(oracle.histogram(vol))
    for t in (1, 101, t_otsu, 255):
        got = _gpu(filters(rule, gate=t), vol, 1)
        want = oracle.filter_volume(vol, 1, RULES[rule][1], gate=t)
        _assert_same(got, want, vol, 1, f"gate {t} {rule}")


def test_constant_and_extreme_full_range_u16(filters):
    for c in (0, 1, 4095, 65535):
        vol = np.full((9, 70, 33), c, np.uint16)
        for rule in RULES:
            for r in (1, 4):
                assert np.all(_gpu(filters(rule), vol, r) == c)


def test_repeat_calls_deterministic(filters):
    vol = ph.ct_u12((160, 100, 40), seed=2300)
    dev = torch.from_numpy(vol).cuda()
    for rule in RULES:
        f = filters(rule)
        first = f(dev, 3).cpu().numpy()
        for _ in range(4):
            assert np.array_equal(f(dev, 3).cpu().numpy(), first)


# ---------------------------------------------------------------------------
# full-size workloads, sampled
# ---------------------------------------------------------------------------

def _full_size(filters, dims, r, rule, seed, m=20000):
    vol_dev = ph.ct_u12(dims, seed=seed, device="cuda")
    out = filters(rule)(vol_dev, r)
    torch.cuda.synchronize()
    vol = vol_dev.cpu().numpy()
    got = out.cpu().numpy()
    pts = _sample_points(dims, m, seed + r)
    want = oracle.filter_points(vol, r, pts, RULES[rule][1])
    g = got[pts[:, 2], pts[:, 1], pts[:, 0]].astype(np.uint32)
    if not np.array_equal(g, want):
        i = int(np.nonzero(g != want)[0][0])
        raise AssertionError(f"{dims} r={r} {rule}: {int((g != want).sum())} of {len(pts)} "
                             f"samples differ; first at {pts[i].tolist()}: gpu {g[i]} oracle "
                             f"{want[i]}")
    return vol, got


@pytest.mark.parametrize("rule", ["mean9", "minvar9"])
@pytest.mark.parametrize("r", [2, 3])
def test_full_512cube_u12_sampled(filters, r, rule):
    _full_size(filters, (512, 512, 512), r, rule, seed=2000)


def test_full_1024x1024x1536_u12_sampled(filters):
    """The at-scale volume (3 GiB), both rules, r=3; outputs sampled on the device."""
    dims = (1024, 1024, 1536)
    vol_dev = ph.ct_u12(dims, seed=3000, device="cuda")
    vol = vol_dev.cpu().numpy()
    pts = _sample_points(dims, 8000, 3003)
    idx = torch.from_numpy(pts.astype(np.int64)).cuda()
    for rule in ("mean9", "minvar9"):
        out = filters(rule)(vol_dev, 3)
        # torch has no uint16 gather on the device: gather the same bits as int16
        g = out.view(torch.int16)[idx[:, 2], idx[:, 1], idx[:, 0]].cpu().numpy()
        g = g.view(np.uint16).astype(np.uint32)
        del out
        want = oracle.filter_points(vol, 3, pts, RULES[rule][1])
        if not np.array_equal(g, want):
            i = int(np.nonzero(g != want)[0][0])
            raise AssertionError(f"{dims} r=3 {rule}: {int((g != want).sum())} of {len(pts)} "
                                 f"samples differ; first at {pts[i].tolist()}: gpu {g[i]} "
                                 f"oracle {want[i]}")


def test_largest_plane_u8(filters):
    """nx*ny just below 2^31 (the largest slice the ABI accepts), one slice deep."""
    nx, ny, nz = 65536, 32767, 1
    g = torch.Generator(device="cuda")
    g.manual_seed(77)
    dev = torch.randint(0, 256, (nz, ny, nx), generator=g, device="cuda", dtype=torch.int32)
    dev = dev.to(torch.uint8)
    out = filters("mean9")(dev, 1)
    torch.cuda.synchronize()
    vol = dev.cpu().numpy()
    got = out.cpu().numpy()
    pts = _sample_points((nx, ny, nz), 4000, 5)
    want = oracle.filter_points(vol, 1, pts, oracle.MEAN9)
    assert np.array_equal(got[pts[:, 2], pts[:, 1], pts[:, 0]].astype(np.uint32), want)


# ---------------------------------------------------------------------------
# error paths (host-side checks; nothing invalid reaches the GPU)
# ---------------------------------------------------------------------------

def test_error_codes(filters):
    f = filters("mean9")
    h = f.handle
    vol = torch.zeros((8, 8, 8), dtype=torch.uint16, device="cuda")
    out = torch.empty_like(vol)
    dims = (8, 8, 8)
    assert _lib.lnf_filter(h, vol, dims, _lib.LNF_U16, 1, out) == 0
    assert _lib.lnf_filter(h, vol, dims, 3, 1, out) == _lib.LNF_EINVAL
    assert _lib.lnf_filter(h, vol, dims, _lib.LNF_U16, 0, out) == _lib.LNF_EINVAL
    assert _lib.lnf_filter(h, vol, dims, _lib.LNF_U16, 5, out) == _lib.LNF_EINVAL
    assert _lib.lnf_filter(h, vol, (0, 8, 8), _lib.LNF_U16, 1, out) == _lib.LNF_EINVAL
    assert _lib.lnf_filter(h, vol, dims, _lib.LNF_U16, 1, vol) == _lib.LNF_EINVAL  # in place
    assert _lib.lnf_filter(h, 0, dims, _lib.LNF_U16, 1, out) == _lib.LNF_EINVAL
    # dims larger than the allocation behind the pointer
    assert _lib.lnf_filter(h, vol, (8, 8, 9), _lib.LNF_U16, 1, out) == _lib.LNF_EINVAL
    # host memory is not device memory
    host = torch.zeros((8, 8, 8), dtype=torch.uint16)
    assert _lib.lnf_filter(h, host, dims, _lib.LNF_U16, 1, out) == _lib.LNF_EDEVICE
    torch.cuda.synchronize()


@pytest.mark.parametrize("variant", [0, 1])
def test_minvar9_extreme_values_every_variant(variant):
    """MINVAR9 at the type's extremes: variance numerators near their bound
    (the packed 64-bit keys hold v below 2^48), both tile variants."""
    from paper_1807_03119_amd.api import Filter
    u16 = ph.random_volume((70, 33, 20), np.uint16, seed=5, kind="extreme")
    u8 = ph.random_volume((45, 38, 21), np.uint8, seed=6, kind="extreme")
    with Filter(_lib.LNF_MINVAR9, 0) as f:
        for v in (u16, u8):
            for r in (1, 2, 3, 4):
                got = _gpu(f, v, r, variant=variant)
                _assert_same(got, oracle.filter_volume(v, r, oracle.MINVAR9), v, r,
                             f"minvar9 extremes v{variant} r={r}")


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_extreme_values_every_variant(variant):
    """Voxels at the type's extremes (0 and the maximum) give the largest
    cluster sums the kernels can see; bit-exact for both voxel types."""
    from paper_1807_03119_amd.api import Filter
    u16 = ph.random_volume((70, 33, 20), np.uint16, seed=3, kind="extreme")
    u8 = ph.random_volume((45, 38, 21), np.uint8, seed=4, kind="extreme")
    with Filter(_lib.LNF_MEAN9, 0) as f:
        for v in (u16, u8):
            for r in (1, 2, 3, 4):
                got = _gpu(f, v, r, variant=variant)
                _assert_same(got, oracle.filter_volume(v, r), v, r, f"extremes v{variant} r={r}")


def test_unknown_flags_rejected():
    import ctypes
    h = ctypes.c_void_p()
    for flags in (8, 6, 0x80000000):
        opt = _lib.lnf_options(ctypes.sizeof(_lib.lnf_options), 0, 0, -1, flags)
        assert _lib.lib().lnf_create(ctypes.byref(h), ctypes.byref(opt)) == _lib.LNF_EINVAL


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_misaligned_base_takes_elementwise_staging(dtype):
    """A volume whose base is not aligned to a pair of elements (a view one
    element into a buffer) is staged element by element; results identical."""
    from paper_1807_03119_amd.api import Filter
    vol = ph.random_volume((70, 21, 13), dtype, seed=77)
    n = vol.size
    tdt = torch.uint8 if dtype == np.uint8 else torch.uint16
    buf = torch.zeros(n + 1, dtype=tdt, device="cuda")
    buf[1:].copy_(torch.from_numpy(vol.reshape(-1)).cuda())
    view = buf[1:].view(vol.shape)  # base one element past an aligned address
    with Filter(_lib.LNF_MEAN9, 0) as f:
        for r in (1, 2, 3, 4):
            want = oracle.filter_volume(vol, r)
            got = f(view, r).cpu().numpy()
            _assert_same(got, want, vol, r, f"misaligned {dtype.__name__} r={r}")
