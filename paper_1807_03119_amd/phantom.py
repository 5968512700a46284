"""Seeded synthetic CT phantoms: the inputs every test and benchmark feeds to
both the HIP path and the CPU oracle.

The paper evaluates its filter on an SRuCT scan of a tachinid fly (Section
"CT Data and 3D Visualisation"), which is not available.  These generators
stand in for it: random ellipsoids and tubes of constant grey value on a
constant background, plus additive noise, rounded and clipped to the bit depth
of the volume.  This module holds no part of the filter's arithmetic; it only
draws numbers from numpy's PCG64 generator (and, for the large volumes built on
the GPU, torch's device generator) in a fixed order, so that a seed fixes every
byte.

Volumes are numpy arrays indexed ``[z, y, x]`` (x fastest), matching the
device layout.  Dimensions are always quoted as ``(nx, ny, nz)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# --------------------------------------------------------------------------
# primitive painters (all draws happen in the callers, in a fixed order)
# --------------------------------------------------------------------------


def _rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly random rotation: QR of a 3x3 Gaussian, signs fixed by R's diagonal."""
    g = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))


def _bbox(centre, ext, dims):
    lo = [max(int(math.floor(centre[i] - ext[i])), 0) for i in range(3)]
    hi = [min(int(math.ceil(centre[i] + ext[i])), dims[i] - 1) for i in range(3)]
    return lo, hi


def _paint_ellipsoid(clean, centre, semi, rot, value):
    """Set every voxel centre p with |diag(1/semi) rot^T (p - centre)| <= 1."""
    nz, ny, nx = clean.shape
    a = rot @ np.diag(1.0 / np.asarray(semi) ** 2) @ rot.T
    ext = [max(semi)] * 3
    lo, hi = _bbox(centre, ext, (nx, ny, nz))
    if any(hi[i] < lo[i] for i in range(3)):
        return
    dx = np.arange(lo[0], hi[0] + 1, dtype=np.float64) - centre[0]
    dy = np.arange(lo[1], hi[1] + 1, dtype=np.float64) - centre[1]
    dz = np.arange(lo[2], hi[2] + 1, dtype=np.float64) - centre[2]
    yy = dy[None, :, None]
    zz = dz[:, None, None]
    # q = p^T A p split as dx*(A00 dx + lin(y,z)) + quad(y,z)
    lin = 2.0 * (a[0, 1] * yy + a[0, 2] * zz)
    quad = a[1, 1] * yy * yy + 2.0 * a[1, 2] * yy * zz + a[2, 2] * zz * zz
    xx = dx[None, None, :]
    q = xx * (a[0, 0] * xx + lin) + quad
    sub = clean[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1]
    np.copyto(sub, value, where=q <= 1.0)


def _paint_cylinder(clean, centre, axis, radius, half_len, value):
    """Set every voxel centre within `radius` of the axis segment of half length `half_len`."""
    nz, ny, nx = clean.shape
    ext = [abs(axis[i]) * half_len + radius * math.sqrt(max(0.0, 1.0 - axis[i] ** 2)) + 1.0
           for i in range(3)]
    lo, hi = _bbox(centre, ext, (nx, ny, nz))
    if any(hi[i] < lo[i] for i in range(3)):
        return
    dx = (np.arange(lo[0], hi[0] + 1, dtype=np.float64) - centre[0])[None, None, :]
    dy = (np.arange(lo[1], hi[1] + 1, dtype=np.float64) - centre[1])[None, :, None]
    dz = (np.arange(lo[2], hi[2] + 1, dtype=np.float64) - centre[2])[:, None, None]
    t = dx * axis[0] + dy * axis[1] + dz * axis[2]
    d2 = dx * dx + dy * dy + dz * dz - t * t
    mask = (np.abs(t) <= half_len) & (d2 <= radius * radius)
    sub = clean[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1]
    np.copyto(sub, value, where=mask)


# --------------------------------------------------------------------------
# the phantom recipe
# --------------------------------------------------------------------------


@dataclass(frozen=True)
class PhantomSpec:
    """Recipe of one phantom family.

    Lengths are fractions of ``min(dims)``; centres are fractions of each axis.
    ``noise`` is ``"gauss"`` (constant sigma) or ``"sqrt"`` (sigma = k*sqrt(value),
    a Gaussian stand-in for photon-counting noise).
    """
    n_ellipsoids: int
    n_cylinders: int
    background: int
    lo: int
    hi: int
    scale: int  # grey values are multiplied by this (1 for 8-bit, 16 for 12-bit)
    noise: str
    sigma: float
    vmax: int
    dtype: type


SPEC_U8 = PhantomSpec(6, 0, 20, 40, 220, 1, "gauss", 20.0, 255, np.uint8)
SPEC_U12 = PhantomSpec(40, 20, 20, 40, 220, 16, "sqrt", 4.0, 4095, np.uint16)
# 8-bit recipe lifted to 12 bits (used for the mixed-dtype batch)
SPEC_U8X16 = PhantomSpec(6, 0, 20, 40, 220, 16, "gauss", 320.0, 4095, np.uint16)


def phantom(dims, spec: PhantomSpec, seed: int, noise_slab: int = 32) -> np.ndarray:
    """Generate one phantom of dims ``(nx, ny, nz)``; returns ``[z, y, x]`` array.

    Draw order: for each ellipsoid (centre[3], semi-axes[3], rotation[9],
    grey value), then for each tube (centre[3], axis[3], radius, half length,
    grey value), then the noise field in z-slabs of ``noise_slab`` slices, C order.
    """
    nx, ny, nz = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    clean = np.full((nz, ny, nx), spec.background * spec.scale, dtype=np.int32)
    for sh in _shape_params((nx, ny, nz), spec, rng):
        if sh[0] == "ellipsoid":
            _paint_ellipsoid(clean, *sh[1:])
        else:
            _paint_cylinder(clean, *sh[1:])
    out = np.empty((nz, ny, nx), dtype=spec.dtype)
    for z0 in range(0, nz, noise_slab):
        z1 = min(nz, z0 + noise_slab)
        g = rng.standard_normal((z1 - z0, ny, nx))
        cl = clean[z0:z1].astype(np.float64)
        if spec.noise == "gauss":
            noisy = cl + spec.sigma * g
        else:
            noisy = cl + spec.sigma * np.sqrt(cl) * g
        np.rint(noisy, out=noisy)
        np.clip(noisy, 0, spec.vmax, out=noisy)
        out[z0:z1] = noisy.astype(spec.dtype)
    return out


def _shape_params(dims, spec: PhantomSpec, rng: np.random.Generator):
    """Draw every shape of the phantom, in the order `phantom` documents."""
    nx, ny, nz = dims
    ref = float(min(nx, ny, nz))
    shapes = []
    for _ in range(spec.n_ellipsoids):
        c = rng.uniform(0.2, 0.8, 3) * np.array([nx, ny, nz], dtype=np.float64)
        semi = rng.uniform(0.05, 0.3, 3) * ref
        rot = _rotation(rng)
        val = int(rng.integers(spec.lo, spec.hi + 1)) * spec.scale
        shapes.append(("ellipsoid", c, semi, rot, val))
    for _ in range(spec.n_cylinders):
        c = rng.uniform(0.2, 0.8, 3) * np.array([nx, ny, nz], dtype=np.float64)
        ax = rng.standard_normal(3)
        ax = ax / np.linalg.norm(ax)
        rad = float(rng.uniform(0.01, 0.04)) * ref
        half = float(rng.uniform(0.1, 0.4)) * ref
        val = int(rng.integers(spec.lo, spec.hi + 1)) * spec.scale
        shapes.append(("cylinder", c, ax, rad, half, val))
    return shapes


def _z_extent(sh):
    """Conservative z-range of a shape (voxel-centre coordinates)."""
    if sh[0] == "ellipsoid":
        c, semi = sh[1], sh[2]
        e = max(semi)
    else:
        c, ax, rad, half = sh[1], sh[2], sh[3], sh[4]
        e = abs(ax[2]) * half + rad + 1.0
    return c[2] - e - 1.0, c[2] + e + 1.0


def phantom_device(dims, spec: PhantomSpec, seed: int, device, slab: int = 64):
    """The same recipe as `phantom`, rasterised and noised on a torch device.

    Shape parameters come from numpy's PCG64 (same draws as `phantom`); the
    noise field comes from torch's generator on `device` seeded with `seed`,
    drawn in z-slabs of `slab` slices, in float32.  Used for the large volumes,
    whose numpy generation would take minutes.  Returns a [z, y, x] tensor.
    """
    import torch
    nx, ny, nz = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    shapes = _shape_params((nx, ny, nz), spec, rng)
    tdt = torch.uint8 if spec.dtype == np.uint8 else torch.uint16
    out = torch.empty((nz, ny, nx), dtype=tdt, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    f64 = torch.float64
    xs = torch.arange(nx, device=device, dtype=f64)
    ys = torch.arange(ny, device=device, dtype=f64)
    for z0 in range(0, nz, slab):
        z1 = min(nz, z0 + slab)
        zs = torch.arange(z0, z1, device=device, dtype=f64)
        clean = torch.full((z1 - z0, ny, nx), float(spec.background * spec.scale),
                           dtype=torch.float32, device=device)
        for sh in shapes:
            zlo, zhi = _z_extent(sh)
            if zhi < z0 or zlo > z1 - 1:
                continue
            if sh[0] == "ellipsoid":
                _, c, semi, rot, val = sh
                a = rot @ np.diag(1.0 / np.asarray(semi) ** 2) @ rot.T
                dx = (xs - c[0])[None, None, :]
                dy = (ys - c[1])[None, :, None]
                dz = (zs - c[2])[:, None, None]
                lin = 2.0 * (float(a[0, 1]) * dy + float(a[0, 2]) * dz)
                quad = float(a[1, 1]) * dy * dy + 2.0 * float(a[1, 2]) * dy * dz + \
                    float(a[2, 2]) * dz * dz
                q = dx * (float(a[0, 0]) * dx + lin) + quad
                clean.masked_fill_(q <= 1.0, float(val))
            else:
                _, c, ax, rad, half, val = sh
                dx = (xs - c[0])[None, None, :]
                dy = (ys - c[1])[None, :, None]
                dz = (zs - c[2])[:, None, None]
                t = dx * float(ax[0]) + dy * float(ax[1]) + dz * float(ax[2])
                d2 = dx * dx + dy * dy + dz * dz - t * t
                clean.masked_fill_((t.abs() <= half) & (d2 <= rad * rad), float(val))
        g = torch.randn(clean.shape, generator=gen, device=device, dtype=torch.float32)
        if spec.noise == "gauss":
            noisy = clean + spec.sigma * g
        else:
            noisy = clean + spec.sigma * torch.sqrt(clean) * g
        noisy = torch.clamp(torch.round(noisy), 0, spec.vmax)
        out[z0:z1] = noisy.to(torch.int32).to(tdt)
    return out


# --------------------------------------------------------------------------
# workload presets
# --------------------------------------------------------------------------

def small_u8(seed: int = 1000, dims=(64, 64, 64)) -> np.ndarray:
    """64^3 uint8: 6 ellipsoids (grey 40..220) on 20, Gaussian noise sigma 20."""
    return phantom(dims, SPEC_U8, seed)


def ct_u12(dims=(512, 512, 512), seed: int = 2000, device=None):
    """uint16 holding 12-bit data: 40 ellipsoids + 20 tubes, sigma = 4*sqrt(value).

    With `device` given, generated there by `phantom_device` (a torch tensor)."""
    if device is not None:
        return phantom_device(dims, SPEC_U12, seed, device)
    return phantom(dims, SPEC_U12, seed)


def random_volume(dims, dtype, seed: int, kind: str = "uniform") -> np.ndarray:
    """Unstructured test volumes.

    ``uniform``: every value of the dtype equally likely.
    ``extreme``: only 0 and the dtype's maximum (worst case for sums and squares).
    ``low``: values in 0..3 (many exact ties between sub-region statistics).
    """
    nx, ny, nz = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    top = np.iinfo(dtype).max
    if kind == "uniform":
        v = rng.integers(0, top + 1, size=(nz, ny, nx), dtype=np.int64)
    elif kind == "extreme":
        v = rng.integers(0, 2, size=(nz, ny, nx), dtype=np.int64) * top
    elif kind == "low":
        v = rng.integers(0, 4, size=(nz, ny, nx), dtype=np.int64)
    else:
        raise ValueError(kind)
    return v.astype(dtype)


@dataclass(frozen=True)
class BatchJob:
    dims: tuple  # (nx, ny, nz)
    dtype: type
    radius: int
    seed: int


def batch_jobs(n: int = 64, seed: int = 4000, lo: int = 64, hi: int = 384):
    """The mixed batch: per volume each axis uniform in [lo, hi], dtype uniform in
    {uint8, uint16}, radius uniform in {1, 2, 3}.  Volume i uses seed ``seed+1+i``."""
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(n):
        dims = tuple(int(v) for v in rng.integers(lo, hi + 1, 3))
        dt = np.uint8 if int(rng.integers(0, 2)) == 0 else np.uint16
        r = int(rng.integers(1, 4))
        jobs.append(BatchJob(dims, dt, r, seed + 1 + i))
    return jobs


def batch_volume(job: BatchJob, device=None):
    """Volume of one batch job (numpy, or a tensor generated on `device`)."""
    spec = SPEC_U8 if job.dtype == np.uint8 else SPEC_U8X16
    if device is not None:
        return phantom_device(job.dims, spec, job.seed, device)
    return phantom(job.dims, spec, job.seed)


@dataclass(frozen=True)
class Request:
    t_arrival: float   # seconds from trace start
    side: int          # cube side (voxels)
    radius: int
    refilter: bool     # True: re-filter a resident volume at a new radius
    pick: float        # uniform [0,1): which resident volume / which crop origin
    pool_index: int    # which pre-generated source volume a new upload is cropped from


def serve_trace(rate: float = 300.0, duration: float = 60.0, seed: int = 5000,
                side_lo: int = 128, side_hi: int = 512, p_refilter: float = 0.3,
                pool: int = 64):
    """Open-loop Poisson request trace: exponential gaps at `rate`/s for
    `duration` s; cube side log-uniform in [side_lo, side_hi]; radius in {1,2,3};
    with probability `p_refilter` a request re-filters a resident volume."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        side = int(round(math.exp(rng.uniform(math.log(side_lo), math.log(side_hi)))))
        r = int(rng.integers(1, 4))
        refilter = bool(rng.uniform() < p_refilter)
        pick = float(rng.uniform())
        pidx = int(rng.integers(0, pool))
        out.append(Request(t, side, r, refilter, pick, pidx))
    return out
