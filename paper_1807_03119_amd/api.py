"""Tensor-level convenience layer over the C ABI (argument marshalling only).

    from paper_1807_03119_amd.api import Filter
    f = Filter(rule=LNF_MEAN9, gate=0)
    out = f(vol_gpu_uint16, radius=3)          # torch tensor [z, y, x] on cuda

Volumes are contiguous ``[z, y, x]`` torch tensors of dtype uint8 or uint16 on
the context's device.  The work is enqueued on the current torch stream.
"""
from __future__ import annotations

from . import _lib
from ._lib import LNF_MEAN9, LNF_MINVAR9, LnfError  # noqa: F401


def _require_cuda(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor (the filter runs only on the GPU)")


class Filter:
    """One lnf context: a rule and a gate threshold on one device."""

    def __init__(self, rule: int = LNF_MEAN9, gate: int = 0, device: int | None = None,
                 geometry: int = 0):
        """geometry: 0 (cubes, diagonal offset r) or LNF_GEOM_* bits of the C API."""
        import torch
        dev = torch.cuda.current_device() if device is None else int(device)
        self.rule, self.gate, self.device, self.geometry = rule, int(gate), dev, int(geometry)
        self._h = _lib.lnf_create(rule, int(gate), dev, int(geometry))

    @property
    def handle(self):
        return self._h

    def __call__(self, vol, radius: int, out=None, stream=None, variant: int = -1, zs: int = 0):
        import torch
        _require_cuda(vol, "vol")
        dt = _lib.dtype_code(vol)
        dims = _lib.dims_of(vol)
        if out is None:
            out = torch.empty_like(vol)
        _require_cuda(out, "out")
        rc = _lib.lnf_filter_tiled(self._h, vol, dims, dt, int(radius), out, stream,
                                   variant=variant, zs=zs)
        if rc != _lib.LNF_OK:
            raise LnfError(rc, "lnf_filter")
        return out

    def tile_config(self, dims, dtype: int, radius: int):
        """(variant, zs) that a call on a volume of dims {nx, ny, nz} would use."""
        return _lib.lnf_tile_config(self._h, dims, dtype, int(radius))

    def filter_otsu(self, vol, radius: int, out=None, stream=None):
        """The paper's automatic pipeline: Otsu threshold of `vol`, then the filter
        gated at it.  Returns (out, T)."""
        import torch
        _require_cuda(vol, "vol")
        if out is None:
            out = torch.empty_like(vol)
        rc, t = _lib.lnf_filter_otsu(self._h, vol, _lib.dims_of(vol), _lib.dtype_code(vol),
                                     int(radius), out, stream)
        if rc != _lib.LNF_OK:
            raise LnfError(rc, "lnf_filter_otsu")
        return out, t

    # ---- the paper's comparison filters (context gate applies; rule unused) ----
    def _compare(self, name, fn, vol, out, *args):
        import torch
        _require_cuda(vol, "vol")
        if out is None:
            out = torch.empty_like(vol)
        res = fn(self._h, vol, _lib.dims_of(vol), _lib.dtype_code(vol), *args[:-1], out, args[-1])
        rc = res[0] if isinstance(res, tuple) else res
        if rc != _lib.LNF_OK:
            raise LnfError(rc, name)
        return (out, res[1]) if isinstance(res, tuple) else out

    def mean(self, vol, radius: int, out=None, stream=None):
        """The paper's mean filter (eq. 4)."""
        return self._compare("lnf_filter_mean", _lib.lnf_filter_mean, vol, out, int(radius), stream)

    def sigma(self, vol, radius: int, half_width: int = -1, out=None, stream=None):
        """Sigma filter (eq. 5); half_width < 0: floor(2 sigma) of the volume.
        Returns (out, half width used)."""
        return self._compare("lnf_filter_sigma", _lib.lnf_filter_sigma, vol, out, int(radius),
                             int(half_width), stream)

    def okada(self, vol, t_d: int, out=None, stream=None):
        """Okada filter (eq. 6) over the six face neighbours."""
        return self._compare("lnf_filter_okada", _lib.lnf_filter_okada, vol, out, int(t_d), stream)

    def entropy(self, vol, radius: int, t_e: float, out=None, stream=None):
        """Entropy filter (eq. 7)."""
        return self._compare("lnf_filter_entropy", _lib.lnf_filter_entropy, vol, out, int(radius),
                             float(t_e), stream)

    def points(self, vol, radius: int, xyz, stream=None):
        """Filtered values at voxels xyz (int32 [n, 3] device tensor of (x, y, z))."""
        import torch
        _require_cuda(vol, "vol")
        xyz = xyz.to(device=vol.device, dtype=torch.int32).contiguous()
        out = torch.empty(xyz.shape[0], dtype=torch.int32, device=vol.device)  # uint32 bits
        rc = _lib.lnf_filter_points(self._h, vol, _lib.dims_of(vol), _lib.dtype_code(vol),
                                    int(radius), xyz, xyz.shape[0], out, stream)
        if rc != _lib.LNF_OK:
            raise LnfError(rc, "lnf_filter_points")
        return out

    def first_hit(self, vol, threshold: int, direction: int = 1, stream=None):
        """First voxel >= threshold along each z-ray (direction 1: from slice 0,
        -1: from the last slice): int32 [ny*nx, 3] of (x, y, z), z = -1 for a miss."""
        import torch
        _require_cuda(vol, "vol")
        nz, ny, nx = vol.shape
        xyz = torch.empty((ny * nx, 3), dtype=torch.int32, device=vol.device)
        rc = _lib.lnf_first_hit(self._h, vol, _lib.dims_of(vol), _lib.dtype_code(vol), threshold,
                                direction, xyz, stream)
        if rc != _lib.LNF_OK:
            raise LnfError(rc, "lnf_first_hit")
        return xyz

    def surface(self, vol, radius: int, threshold: int, direction: int = 1, stream=None):
        """The filter at each z-ray's first hit: (values [ny, nx] as int32 holding
        uint32 bits, 0xFFFFFFFF for a miss; hits [ny*nx, 3])."""
        import torch
        _require_cuda(vol, "vol")
        nz, ny, nx = vol.shape
        xyz = torch.empty((ny * nx, 3), dtype=torch.int32, device=vol.device)
        out = torch.empty((ny, nx), dtype=torch.int32, device=vol.device)
        rc = _lib.lnf_filter_surface(self._h, vol, _lib.dims_of(vol), _lib.dtype_code(vol),
                                     int(radius), threshold, direction, xyz, out, stream)
        if rc != _lib.LNF_OK:
            raise LnfError(rc, "lnf_filter_surface")
        return out, xyz

    def histogram(self, vol, stream=None):
        import torch
        _require_cuda(vol, "vol")
        levels = 256 if vol.dtype == torch.uint8 else 65536
        hist = torch.empty(levels, dtype=torch.int64, device=vol.device)
        rc = _lib.lnf_histogram(self._h, vol, _lib.dims_of(vol), _lib.dtype_code(vol), hist, stream)
        if rc != _lib.LNF_OK:
            raise LnfError(rc, "lnf_histogram")
        return hist

    def batch(self, items, stream=None, mode=None):
        """Filter [(vol, radius), ...] (or [(vol, out, radius), ...]) with one
        launch per (radius, dtype) group; returns the list of outputs.  mode:
        LNF_BATCH_GRID (None: the default) or LNF_BATCH_PERSISTENT."""
        import torch
        triples = []
        for it in items:
            if len(it) == 2:
                vol, r = it
                out = torch.empty_like(vol)
            else:
                vol, out, r = it
            _require_cuda(vol, "vol")
            triples.append((vol, out, r))
        rc = _lib.lnf_filter_batch(self._h, triples, stream=stream, mode=mode)
        if rc != _lib.LNF_OK:
            raise LnfError(rc, "lnf_filter_batch")
        return [t[1] for t in triples]

    def tune(self, items):
        """Autotune on [(vol, out, radius), ...]; outputs are overwritten."""
        rc = _lib.lnf_tune(self._h, list(items))
        if rc != _lib.LNF_OK:
            raise LnfError(rc, "lnf_tune")

    def close(self):
        if self._h is not None:
            _lib.lnf_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_cache: dict = {}


def filter_volume(vol, radius: int, rule: int = LNF_MEAN9, gate: int = 0, out=None, stream=None):
    """Filter one device volume with a cached context for (rule, gate, device)."""
    key = (rule, int(gate), vol.device.index)
    f = _cache.get(key)
    if f is None:
        f = _cache[key] = Filter(rule, gate, vol.device.index)
    return f(vol, radius, out=out, stream=stream)


class Server:
    """Request server over a Filter context (continuous batching).

    Host buffers handed to `put` / `submit` are referenced until the request
    using them completes; this wrapper keeps them alive until `sync`/`close`.
    """

    def __init__(self, filt: Filter, cap_bytes: int = 200 << 30, n_streams: int = 4,
                 max_batch: int = 256, mode: int = _lib.LNF_SERVE_BATCHED, fail_batch: int = 0,
                 batch_mvox: int = 0):
        """batch_mvox: voxel budget of a micro-batch in 2^20 voxels (0: 32)."""
        self.filt = filt
        self._s = _lib.lnf_server_create(filt.handle, mode, cap_bytes, n_streams, max_batch,
                                         fail_batch, batch_mvox)
        self._keep = []

    def put(self, host, dims=None, dtype=None, pitch=None, keep=None):
        """Upload a host volume (contiguous torch CPU tensor or numpy array, or a raw
        pointer with explicit dims/dtype); returns (rc, vol_id)."""
        if isinstance(host, int):
            ptr = host
        else:
            import numpy as np
            if isinstance(host, np.ndarray):
                ptr = host.ctypes.data
                dt = host.dtype
                dtype = dtype or (_lib.LNF_U8 if dt == np.uint8 else _lib.LNF_U16)
            else:
                ptr = host.data_ptr()
                dtype = dtype or _lib.dtype_code(host)
            if dims is None:
                nz, ny, nx = host.shape
                dims = (nx, ny, nz)
            self._keep.append(host)
        if keep is not None:
            self._keep.append(keep)
        return _lib.lnf_server_put_volume(self._s, ptr, dims, dtype, pitch)

    def submit(self, vol_id, radius, host_out=None, arrival_ns=0):
        ptr = 0
        if host_out is not None:
            ptr = host_out if isinstance(host_out, int) else (
                host_out.ctypes.data if hasattr(host_out, "ctypes") else host_out.data_ptr())
            self._keep.append(host_out)
        return _lib.lnf_server_submit(self._s, vol_id, radius, ptr, arrival_ns)

    def wait(self, ticket, timeout_ms=-1):
        return _lib.lnf_server_wait(self._s, ticket, timeout_ms)

    def poll(self, ticket):
        return _lib.lnf_server_poll(self._s, ticket)

    def cancel(self, ticket):
        return _lib.lnf_server_cancel(self._s, ticket)

    def release(self, vol_id):
        return _lib.lnf_server_release(self._s, vol_id)

    def sync(self):
        rc = _lib.lnf_server_sync(self._s)
        self._keep.clear()
        return rc

    def stats(self, reset=False):
        return _lib.lnf_server_stats(self._s, reset)

    def close(self):
        if self._s is not None:
            _lib.lnf_server_destroy(self._s)
            self._s = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
