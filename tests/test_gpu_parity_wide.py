"""Whole-volume parity on the paths the kernels take at full size.

The 64-wide MEAN9 tiles stage element pairs only where the tile's x halo lies
inside the volume, and run packed (px | qx << 16 per LDS word) with an
unpacked rerun for tiles whose x-pass sums do not fit 16 bits.  Volumes here
are wide enough for interior tiles of every tile variant, and their data
drive both modes: 12-bit data stay packed, full-range and extreme data make
tiles fall back, and isolated bright voxels make only some tiles fall back.
The benchmark volumes (512^3, and the z-strip seams of 1024 x 1024 x 1536)
are compared with the oracle in full.  Bit-exact throughout (paper, Section
"Our Method", eqs. 2-3; the mean filter is eq. 4).
"""
import numpy as np
import pytest

import oracle
from oracle import compare
from paper_1807_03119_amd import _lib
from paper_1807_03119_amd import phantom as ph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

WIDE = (200, 40, 24)  # nx, ny, nz: interior 64-wide tiles at every radius


def _dev(v):
    return torch.from_numpy(np.ascontiguousarray(v)).cuda()


def _same(got, want, what):
    if np.array_equal(got, want):
        return
    bad = np.argwhere(got != want)
    z, y, x = (int(v) for v in bad[0])
    raise AssertionError(f"{what}: {len(bad)} of {got.size} differ; first at (x,y,z)=({x},{y},{z}) "
                         f"gpu={got[z, y, x]} oracle={want[z, y, x]}")


def _volume(kind, dims=WIDE, seed=11):
    """[z, y, x] test volume of the given kind."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    if kind == "u8":
        return rng.integers(0, 256, (nz, ny, nx), dtype=np.uint8)
    if kind == "u12":
        return rng.integers(0, 4096, (nz, ny, nx), dtype=np.uint16)
    if kind == "u16":
        return rng.integers(0, 65536, (nz, ny, nx), dtype=np.uint16)
    if kind == "u16_extreme":
        return ph.random_volume(dims, np.uint16, seed=seed, kind="extreme")
    if kind == "u12_hot":
        v = rng.integers(0, 4096, (nz, ny, nx), dtype=np.uint16)
        # a few bright voxels: only the tiles whose halo holds one fall back
        for x, y, z in ((5, 3, 2), (nx // 2, ny // 2, nz // 2), (nx - 1, ny - 1, nz - 1)):
            v[z, y, x] = 65000
        return v
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["u8", "u12", "u16", "u16_extreme", "u12_hot"])
def test_wide_mean9_every_variant(kind):
    from paper_1807_03119_amd.api import Filter
    vol = _volume(kind)
    dt = _lib.LNF_U8 if vol.dtype == np.uint8 else _lib.LNF_U16
    dev = _dev(vol)
    with Filter(_lib.LNF_MEAN9, 0) as f:
        for r in range(1, _lib.LNF_RADIUS_MAX + 1):
            want = oracle.filter_volume(vol, r)
            for variant in [-1] + list(range(_lib.lnf_tile_variants(_lib.LNF_MEAN9, dt, r))):
                for zs in (0, 7):
                    got = f(dev, r, variant=variant, zs=zs).cpu().numpy()
                    _same(got, want, f"{kind} r={r} variant {variant} zs {zs}")


@pytest.mark.parametrize("slab", [(50, 3), (9, 1), (93, 3)])
def test_wide_mean9_falls_back_mid_strip(slab):
    """A dim volume with a bright slab deep in z: packed tiles stop at the
    slab and rerun unpacked from there, keeping the slices before it.  Every
    variant, z-strips of the default, 7 and 40 slices, r = 1..4."""
    from paper_1807_03119_amd.api import Filter
    z, depth = slab
    rng = np.random.default_rng(17 + z)
    vol = rng.integers(0, 1024, (96, 40, 200), dtype=np.uint16)
    vol[z:z + depth, 5:30, 20:180] = rng.integers(60000, 65536, (depth, 25, 160), dtype=np.uint16)
    dev = _dev(vol)
    with Filter(_lib.LNF_MEAN9, 0) as f:
        for r in range(1, _lib.LNF_RADIUS_MAX + 1):
            want = oracle.filter_volume(vol, r)
            for variant in [-1] + list(range(_lib.lnf_tile_variants(_lib.LNF_MEAN9, _lib.LNF_U16, r))):
                for zs in (0, 7, 40):
                    got = f(dev, r, variant=variant, zs=zs).cpu().numpy()
                    _same(got, want, f"slab {slab} r={r} variant {variant} zs {zs}")


@pytest.mark.parametrize("kind", ["u12_hot", "u16"])
def test_wide_mean9_gated(kind):
    """The gate applies after the packed and the unpacked runs alike."""
    from paper_1807_03119_amd.api import Filter
    vol = _volume(kind, seed=12)
    dev = _dev(vol)
    for gate in (1500, 30000):
        with Filter(_lib.LNF_MEAN9, gate) as f:
            for r in (1, 3):
                got = f(dev, r).cpu().numpy()
                _same(got, oracle.filter_volume(vol, r, oracle.MEAN9, gate), f"{kind} T={gate} r={r}")


@pytest.mark.parametrize("kind", ["u8", "u12", "u16"])
def test_wide_mean_filter(kind):
    from paper_1807_03119_amd.api import Filter
    vol = _volume(kind, seed=13)
    dev = _dev(vol)
    with Filter(_lib.LNF_MEAN9, 0) as f:
        for r in range(1, _lib.LNF_RADIUS_MAX + 1):
            got = f.mean(dev, r).cpu().numpy()
            _same(got, compare.mean_filter(vol, r), f"mean filter {kind} r={r}")


@pytest.mark.parametrize("kind", ["u8", "u12", "u16", "u16_extreme", "u12_hot"])
def test_wide_minvar9_both_tiles(kind):
    from paper_1807_03119_amd.api import Filter
    vol = _volume(kind, dims=(260, 40, 20), seed=14)
    dev = _dev(vol)
    with Filter(_lib.LNF_MINVAR9, 0) as f:
        for r in range(1, _lib.LNF_RADIUS_MAX + 1):
            want = oracle.filter_volume(vol, r, oracle.MINVAR9)
            for variant in (-1, 0, 1):
                got = f(dev, r, variant=variant).cpu().numpy()
                _same(got, want, f"minvar9 {kind} r={r} variant {variant}")


# (r, b, v): values below 2^b keep the uint32 sums of squares of the z- and
# x-passes exact; v is the least value whose (2r+1)^2 squares pass 2^32
NARROW_LIMITS = [(1, 14, 21846), (2, 13, 13108), (3, 13, 9363)]


@pytest.mark.parametrize("r,b,v", NARROW_LIMITS)
@pytest.mark.parametrize("where", ["mid", "end"])
def test_minvar9_narrow_squares_limit(r, b, v, where):
    """uint16 MINVAR9 tiles keep their sums of squares in uint32 through the
    z- and x-passes while every value they load is below 2^b, and run again
    with fp64 sums once one reaches it.  Whole planes at 2^b - 1 give the
    largest narrow sums; 2^b, and v (which would wrap the uint32 sums), make
    the tiles that load them run again, from blocks in mid-strip ("mid") or
    from the last planes of the volume ("end").  Both tile variants, z-strips
    of the default, 7 and 40 slices."""
    from paper_1807_03119_amd.api import Filter
    m = (2 * r + 1) ** 2
    assert m * ((1 << b) - 1) ** 2 < 1 << 32 <= m * ((2 << b) - 1) ** 2  # b: the most bits
    assert m * (v - 1) ** 2 < 1 << 32 <= m * v ** 2
    rng = np.random.default_rng(40 + r)
    base = rng.integers(0, 4096, (48, 40, 200), dtype=np.uint16)
    with Filter(_lib.LNF_MINVAR9, 0) as f:
        for value in ((1 << b) - 1, 1 << b, v):
            vol = base.copy()
            if where == "mid":
                vol[30:30 + 2 * r + 1] = value
            else:
                vol[-1] = value
            want = oracle.filter_volume(vol, r, oracle.MINVAR9)
            dev = _dev(vol)
            for variant in (0, 1):
                for zs in (0, 7, 40):
                    got = f(dev, r, variant=variant, zs=zs).cpu().numpy()
                    _same(got, want, f"r={r} value {value} {where} variant {variant} zs {zs}")


def test_tile_config_matches_its_launch():
    """lnf_tile_config reports the configuration lnf_filter launches: the
    same bytes come out when that configuration is passed explicitly."""
    from paper_1807_03119_amd.api import Filter
    vol = _volume("u12", dims=(130, 70, 90), seed=15)
    dev = _dev(vol)
    for rule in (_lib.LNF_MEAN9, _lib.LNF_MINVAR9):
        with Filter(rule, 0) as f:
            for r in (1, 3):
                variant, zs = f.tile_config((130, 70, 90), _lib.LNF_U16, r)
                assert 0 <= variant < _lib.lnf_tile_variants(rule, _lib.LNF_U16, r)
                assert 1 <= zs <= 90
                a = f(dev, r).cpu().numpy()
                b = f(dev, r, variant=variant, zs=zs).cpu().numpy()
                assert np.array_equal(a, b)


@pytest.fixture(scope="module")
def c2_volume():
    """The 512^3 uint16 12-bit CT phantom of the benchmark (device and host)."""
    dev = ph.ct_u12((512, 512, 512), seed=2000, device="cuda")
    torch.cuda.synchronize()
    return dev, dev.cpu().numpy()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("rule", ["mean9", "minvar9"])
@pytest.mark.parametrize("r", [2, 3])
def test_full_512_cube(c2_volume, rule, r):
    """Every voxel of the benchmark volume against the brute-force oracle."""
    from paper_1807_03119_amd.api import Filter
    dev, host = c2_volume
    rc, oc = (_lib.LNF_MEAN9, oracle.MEAN9) if rule == "mean9" else (_lib.LNF_MINVAR9, oracle.MINVAR9)
    with Filter(rc, 0) as f:
        got = f(dev, r).cpu().numpy()
    print(f"512^3 {rule} r={r}: oracle on {oracle.threads()} threads", flush=True)
    _same(got, oracle.filter_volume(host, r, oc), f"512^3 {rule} r={r}")


@pytest.mark.timeout(900)
def test_scale_volume_strip_seams():
    """1024 x 1024 x 1536 at r = 3, both rules: the default launch (whose x-y
    tiles alone fill the GPU, so it runs one z-strip per column) and the same
    tile forced into 384-slice z-strips.  Whole z-slices on both sides of every
    seam, plus the first, middle and last slices, against the oracle."""
    from paper_1807_03119_amd.api import Filter
    dims = (1024, 1024, 1536)
    dev = ph.ct_u12(dims, seed=3000, device="cuda")
    out = torch.empty_like(dev)
    host = None
    nx, ny, nz = dims
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    for rc, oc in ((_lib.LNF_MEAN9, oracle.MEAN9), (_lib.LNF_MINVAR9, oracle.MINVAR9)):
        with Filter(rc, 0) as f:
            variant, zs_default = f.tile_config(dims, _lib.LNF_U16, 3)
            for zs in sorted({zs_default, 384}):
                f(dev, 3, out=out, variant=variant, zs=zs)
                torch.cuda.synchronize()
                if host is None:
                    host = dev.cpu().numpy()
                seams = list(range(zs, nz, zs))
                assert zs == zs_default or len(seams) == 3
                zsl = sorted({0, nz // 2, nz - 1} | {z for s in seams for z in (s - 1, s)})
                print(f"rule {rc} variant {variant} zs {zs}: slices {zsl}", flush=True)
                for z in zsl:
                    pts = np.stack([xx.ravel(), yy.ravel(), np.full(xx.size, z)], 1)
                    want = oracle.filter_points(host, 3, pts, oc).reshape(ny, nx)
                    got = out[z].cpu().numpy().astype(np.uint32)
                    if not np.array_equal(got, want):
                        bad = np.argwhere(got != want)
                        raise AssertionError(f"rule {rc} zs {zs} slice {z}: {len(bad)} differ, "
                                             f"first (y,x)={tuple(bad[0])}")
    del dev, out
    torch.cuda.empty_cache()
