"""ctypes binding of liblnf.so (include/lnf.h).

Argument marshalling only: every step of the filter runs in the HIP library.
Functions keep the C names; tensors are passed as device pointers and the
current torch stream is used unless a stream is given.  There is no CPU
fallback: if the library is missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblnf.so")

LNF_OK = 0
LNF_EINVAL = -1
LNF_EDEVICE = -2
LNF_ENOMEM = -3
LNF_EHIP = -4
LNF_EBUSY = -5
LNF_ENOTFOUND = -6
LNF_ECANCELED = -7
LNF_ETIMEDOUT = -8
LNF_ERANGE = -9
LNF_BATCH_NOALLOC_MAX = 256

LNF_U8 = 1
LNF_U16 = 2
LNF_MEAN9 = 0
LNF_MINVAR9 = 1
LNF_GEOM_CROSS = 1
LNF_GEOM_OFFSET_1 = 2
LNF_GEOM_OFFSET_2R1 = 4
LNF_RADIUS_MAX = 4


class LnfError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


class lnf_options(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("rule", ctypes.c_int32), ("gate_T", ctypes.c_uint32),
                ("device", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class lnf_tile(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("zs", ctypes.c_int32)]


class lnf_job(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("dims", ctypes.c_int64 * 3), ("dtype", ctypes.c_int32),
                ("radius", ctypes.c_int32)]


LNF_BATCH_MAX = 4096
LNF_BATCH_GRID = 0
LNF_BATCH_PERSISTENT = 1
LNF_SERVE_BATCHED = 0
LNF_SERVE_FIFO = 1


class lnf_server_options(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("mode", ctypes.c_int32), ("cap_bytes", ctypes.c_uint64),
                ("n_streams", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("fail_batch", ctypes.c_int32), ("batch_mvox", ctypes.c_int32)]


class lnf_server_stats_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("submitted", "completed", "failed", "cancelled", "batches", "evictions", "uploads",
                 "voxels", "bytes_in_use", "peak_bytes")] + \
               [(n, ctypes.c_double) for n in
                ("p50_ms", "p99_ms", "max_ms", "mean_ms", "busy_s", "gvox_per_s")]


_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int
_dims_t = ctypes.c_int64 * 3


def _declare(lib):
    sig = {
        "lnf_create": [ctypes.POINTER(_vp), ctypes.POINTER(lnf_options)],
        "lnf_destroy": [_vp],
        "lnf_filter": [_vp, _vp, ctypes.POINTER(ctypes.c_int64), _i32, _i32, _vp, _vp],
        "lnf_filter_tiled": [_vp, _vp, ctypes.POINTER(ctypes.c_int64), _i32, _i32, _vp, _vp,
                             ctypes.POINTER(lnf_tile)],
        "lnf_tile_variants": [_i32, _i32, _i32],
        "lnf_tile_config": [_vp, ctypes.POINTER(ctypes.c_int64), _i32, _i32, ctypes.POINTER(lnf_tile)],
        "lnf_filter_batch": [_vp, ctypes.POINTER(lnf_job), _i32, _vp],
        "lnf_filter_batch_mode": [_vp, ctypes.POINTER(lnf_job), _i32, _vp, _i32],
        "lnf_filter_batch_noalloc": [_vp, ctypes.POINTER(lnf_job), _i32, _vp],
        "lnf_tune": [_vp, ctypes.POINTER(lnf_job), _i32],
        "lnf_tune_save": [_vp, ctypes.c_char_p],
        "lnf_tune_load": [_vp, ctypes.c_char_p],
        "lnf_version": [],
        "lnf_histogram": [_vp, _vp, ctypes.POINTER(ctypes.c_int64), _i32, _vp, _vp],
        "lnf_filter_points": [_vp, _vp, ctypes.POINTER(ctypes.c_int64), _i32, _i32, _vp,
                              ctypes.c_int64, _vp, _vp],
        "lnf_otsu_threshold": [_vp, _i32, ctypes.POINTER(ctypes.c_uint32)],
        "lnf_first_hit": [_vp, _vp, ctypes.POINTER(ctypes.c_int64), _i32, ctypes.c_uint32, _i32,
                          _vp, _vp],
        "lnf_filter_surface": [_vp, _vp, ctypes.POINTER(ctypes.c_int64), _i32, _i32,
                               ctypes.c_uint32, _i32, _vp, _vp, _vp],
        "lnf_filter_otsu": [_vp, _vp, ctypes.POINTER(ctypes.c_int64), _i32, _i32, _vp, _vp,
                            ctypes.POINTER(ctypes.c_uint32)],
        "lnf_filter_mean": [_vp, _vp, ctypes.POINTER(ctypes.c_int64), _i32, _i32, _vp, _vp],
        "lnf_filter_sigma": [_vp, _vp, ctypes.POINTER(ctypes.c_int64), _i32, _i32,
                             ctypes.c_int64, _vp, _vp, ctypes.POINTER(ctypes.c_int64)],
        "lnf_filter_okada": [_vp, _vp, ctypes.POINTER(ctypes.c_int64), _i32, ctypes.c_uint32,
                             _vp, _vp],
        "lnf_filter_entropy": [_vp, _vp, ctypes.POINTER(ctypes.c_int64), _i32, _i32,
                               ctypes.c_double, _vp, _vp],
    }
    _u64, _i64 = ctypes.c_uint64, ctypes.c_int64
    sig.update({
        "lnf_server_create": [_vp, ctypes.POINTER(lnf_server_options), ctypes.POINTER(_vp)],
        "lnf_server_destroy": [_vp],
        "lnf_server_put_volume": [_vp, _vp, ctypes.POINTER(_i64), _i32, ctypes.POINTER(_i64),
                                  ctypes.POINTER(_u64)],
        "lnf_server_release": [_vp, _u64],
        "lnf_server_submit": [_vp, _u64, _i32, _vp, _i64, ctypes.POINTER(_u64)],
        "lnf_server_poll": [_vp, _u64, ctypes.POINTER(_i32)],
        "lnf_server_wait": [_vp, _u64, _i32],
        "lnf_server_cancel": [_vp, _u64],
        "lnf_server_sync": [_vp],
        "lnf_server_stats": [_vp, ctypes.POINTER(lnf_server_stats_t), _i32],
    })
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.lnf_server_now_ns.argtypes = []
    lib.lnf_server_now_ns.restype = ctypes.c_int64
    lib.lnf_strerror.argtypes = [_i32]
    lib.lnf_strerror.restype = ctypes.c_char_p


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1807_03119_amd.build` (needs hipcc)")
        handle = ctypes.CDLL(LIB_PATH)
        _declare(handle)
        _lib = handle
    return _lib


def strerror(code: int) -> str:
    if _lib is None and not os.path.exists(LIB_PATH):
        return f"status {code}"
    return lib().lnf_strerror(code).decode()


def _check(code: int, where: str) -> int:
    if code != LNF_OK:
        raise LnfError(code, where)
    return code


# ---------------------------------------------------------------------------
# tensor marshalling helpers
# ---------------------------------------------------------------------------

def dtype_code(t) -> int:
    import torch
    if t.dtype == torch.uint8:
        return LNF_U8
    if t.dtype == torch.uint16:
        return LNF_U16
    raise TypeError(f"volumes must be torch.uint8 or torch.uint16, got {t.dtype}")


def dims_of(t):
    """(nx, ny, nz) of a contiguous [z, y, x] tensor."""
    if t.dim() != 3:
        raise ValueError("volumes are 3D tensors indexed [z, y, x]")
    if not t.is_contiguous():
        raise ValueError("volumes must be contiguous (x fastest)")
    nz, ny, nx = t.shape
    return (int(nx), int(ny), int(nz))


def stream_ptr(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


# ---------------------------------------------------------------------------
# C functions under their C names
# ---------------------------------------------------------------------------

def lnf_version() -> int:
    return lib().lnf_version()


def lnf_strerror(code: int) -> str:
    return strerror(code)


def lnf_create(rule: int = LNF_MEAN9, gate_T: int = 0, device: int = -1, flags: int = 0):
    opt = lnf_options(ctypes.sizeof(lnf_options), rule, gate_T, device, flags)
    h = _vp()
    _check(lib().lnf_create(ctypes.byref(h), ctypes.byref(opt)), "lnf_create")
    return h


def lnf_destroy(h) -> None:
    _check(lib().lnf_destroy(h), "lnf_destroy")


def lnf_tile_variants(rule: int, dtype: int, radius: int) -> int:
    n = lib().lnf_tile_variants(rule, dtype, radius)
    if n < 0:
        raise LnfError(n, "lnf_tile_variants")
    return n


def lnf_tile_config(h, dims, dtype: int, radius: int):
    """(variant, zs) that lnf_filter would use for a volume of these dims."""
    t = lnf_tile(-1, 0)
    rc = lib().lnf_tile_config(h, _dims_t(*dims), dtype, radius, ctypes.byref(t))
    if rc:
        raise LnfError(rc, "lnf_tile_config")
    return t.variant, t.zs


def lnf_filter(h, vol, dims, dtype: int, radius: int, out, stream=None) -> int:
    """C signature; `vol`/`out` are tensors or raw device addresses (ints)."""
    vp = vol if isinstance(vol, int) else vol.data_ptr()
    op = out if isinstance(out, int) else out.data_ptr()
    d = _dims_t(*[int(v) for v in dims])
    return lib().lnf_filter(h, vp, d, dtype, radius, op, stream_ptr(stream))


def lnf_filter_tiled(h, vol, dims, dtype: int, radius: int, out, stream=None, variant: int = -1,
                     zs: int = 0) -> int:
    vp = vol if isinstance(vol, int) else vol.data_ptr()
    op = out if isinstance(out, int) else out.data_ptr()
    d = _dims_t(*[int(v) for v in dims])
    t = lnf_tile(variant, zs)
    return lib().lnf_filter_tiled(h, vp, d, dtype, radius, op, stream_ptr(stream),
                                  ctypes.byref(t))


def make_jobs(items):
    """ctypes array of lnf_job from (vol, out, radius) triples of tensors (or
    (in_ptr, out_ptr, dims, dtype, radius) tuples of raw values)."""
    arr = (lnf_job * max(len(items), 1))()
    for i, it in enumerate(items):
        if len(it) == 3:
            vol, out, r = it
            arr[i].in_ = vol.data_ptr()
            arr[i].out = out.data_ptr()
            arr[i].dims = (ctypes.c_int64 * 3)(*dims_of(vol))
            arr[i].dtype = dtype_code(vol)
            arr[i].radius = int(r)
        else:
            ip, op, dims, dt, r = it
            arr[i].in_, arr[i].out = int(ip), int(op)
            arr[i].dims = (ctypes.c_int64 * 3)(*[int(d) for d in dims])
            arr[i].dtype, arr[i].radius = int(dt), int(r)
    return arr


def lnf_filter_batch(h, jobs, n=None, stream=None, mode=None) -> int:
    """`jobs`: a make_jobs array (or a list accepted by make_jobs); mode None
    calls lnf_filter_batch, else lnf_filter_batch_mode."""
    if isinstance(jobs, (list, tuple)):
        n = len(jobs) if n is None else n
        jobs = make_jobs(jobs)
    n = len(jobs) if n is None else n
    if mode is None:
        return lib().lnf_filter_batch(h, jobs, n, stream_ptr(stream))
    return lib().lnf_filter_batch_mode(h, jobs, n, stream_ptr(stream), int(mode))


def lnf_filter_batch_noalloc(h, jobs, n=None, stream=None) -> int:
    """`jobs`: a make_jobs array (or a list accepted by make_jobs)."""
    if isinstance(jobs, (list, tuple)):
        n = len(jobs) if n is None else n
        jobs = make_jobs(jobs)
    n = len(jobs) if n is None else n
    return lib().lnf_filter_batch_noalloc(h, jobs, n, stream_ptr(stream))


def lnf_tune(h, jobs, n=None) -> int:
    if isinstance(jobs, (list, tuple)):
        n = len(jobs) if n is None else n
        jobs = make_jobs(jobs)
    n = len(jobs) if n is None else n
    return lib().lnf_tune(h, jobs, n)


def lnf_tune_save(h, path: str) -> int:
    return lib().lnf_tune_save(h, path.encode())


def lnf_tune_load(h, path: str) -> int:
    return lib().lnf_tune_load(h, path.encode())


# ---------------------------------------------------------------------------
# server
# ---------------------------------------------------------------------------

def lnf_server_now_ns() -> int:
    return lib().lnf_server_now_ns()


def lnf_server_create(h, mode=LNF_SERVE_BATCHED, cap_bytes=200 << 30, n_streams=4, max_batch=256,
                      fail_batch=0, batch_mvox=0):
    opt = lnf_server_options(ctypes.sizeof(lnf_server_options), mode, cap_bytes, n_streams,
                             max_batch, fail_batch, batch_mvox)
    srv = _vp()
    _check(lib().lnf_server_create(h, ctypes.byref(opt), ctypes.byref(srv)), "lnf_server_create")
    return srv


def lnf_server_destroy(srv) -> int:
    return lib().lnf_server_destroy(srv)


def lnf_server_put_volume(srv, host_ptr: int, dims, dtype: int, pitch=None):
    """Returns (rc, vol_id)."""
    d = _dims_t(*[int(v) for v in dims])
    p = (ctypes.c_int64 * 2)(*[int(v) for v in pitch]) if pitch is not None else None
    vid = ctypes.c_uint64()
    rc = lib().lnf_server_put_volume(srv, host_ptr, d, dtype, p, ctypes.byref(vid))
    return rc, vid.value


def lnf_server_release(srv, vol_id: int) -> int:
    return lib().lnf_server_release(srv, vol_id)


def lnf_server_submit(srv, vol_id: int, radius: int, host_out: int = 0, arrival_ns: int = 0):
    """Returns (rc, ticket)."""
    t = ctypes.c_uint64()
    rc = lib().lnf_server_submit(srv, vol_id, radius, host_out or None, arrival_ns, ctypes.byref(t))
    return rc, t.value


def lnf_server_poll(srv, ticket: int):
    """Returns (rc, done)."""
    d = ctypes.c_int()
    rc = lib().lnf_server_poll(srv, ticket, ctypes.byref(d))
    return rc, bool(d.value)


def lnf_server_wait(srv, ticket: int, timeout_ms: int = -1) -> int:
    return lib().lnf_server_wait(srv, ticket, timeout_ms)


def lnf_server_cancel(srv, ticket: int) -> int:
    return lib().lnf_server_cancel(srv, ticket)


def lnf_server_sync(srv) -> int:
    return lib().lnf_server_sync(srv)


def lnf_server_stats(srv, reset: bool = False) -> dict:
    st = lnf_server_stats_t()
    _check(lib().lnf_server_stats(srv, ctypes.byref(st), int(reset)), "lnf_server_stats")
    return {name: getattr(st, name) for name, _ in lnf_server_stats_t._fields_}


# ---------------------------------------------------------------------------
# Otsu threshold and gated pipeline
# ---------------------------------------------------------------------------

def lnf_histogram(h, vol, dims, dtype: int, hist, stream=None) -> int:
    vp = vol if isinstance(vol, int) else vol.data_ptr()
    hp = hist if isinstance(hist, int) else hist.data_ptr()
    return lib().lnf_histogram(h, vp, _dims_t(*[int(v) for v in dims]), dtype, hp,
                               stream_ptr(stream))


def lnf_otsu_threshold(hist) -> int:
    """Otsu threshold of a host histogram (numpy-compatible sequence of counts)."""
    import numpy as np
    arr = np.ascontiguousarray(np.asarray(hist, dtype=np.uint64))
    t = ctypes.c_uint32()
    _check(lib().lnf_otsu_threshold(arr.ctypes.data, int(arr.size), ctypes.byref(t)),
           "lnf_otsu_threshold")
    return t.value


def lnf_filter_otsu(h, vol, dims, dtype: int, radius: int, out, stream=None):
    """Returns (rc, T)."""
    vp = vol if isinstance(vol, int) else vol.data_ptr()
    op = out if isinstance(out, int) else out.data_ptr()
    t = ctypes.c_uint32()
    rc = lib().lnf_filter_otsu(h, vp, _dims_t(*[int(v) for v in dims]), dtype, radius, op,
                               stream_ptr(stream), ctypes.byref(t))
    return rc, t.value


def _p(t):
    return t if isinstance(t, int) else t.data_ptr()


def lnf_filter_mean(h, vol, dims, dtype: int, radius: int, out, stream=None) -> int:
    return lib().lnf_filter_mean(h, _p(vol), _dims_t(*[int(v) for v in dims]), dtype, radius,
                                 _p(out), stream_ptr(stream))


def lnf_filter_sigma(h, vol, dims, dtype: int, radius: int, half_width: int, out, stream=None):
    """Returns (rc, half width used)."""
    w = ctypes.c_int64()
    rc = lib().lnf_filter_sigma(h, _p(vol), _dims_t(*[int(v) for v in dims]), dtype, radius,
                                int(half_width), _p(out), stream_ptr(stream), ctypes.byref(w))
    return rc, w.value


def lnf_filter_okada(h, vol, dims, dtype: int, t_d: int, out, stream=None) -> int:
    return lib().lnf_filter_okada(h, _p(vol), _dims_t(*[int(v) for v in dims]), dtype, int(t_d),
                                  _p(out), stream_ptr(stream))


def lnf_filter_entropy(h, vol, dims, dtype: int, radius: int, t_e: float, out, stream=None) -> int:
    return lib().lnf_filter_entropy(h, _p(vol), _dims_t(*[int(v) for v in dims]), dtype, radius,
                                    float(t_e), _p(out), stream_ptr(stream))


def lnf_first_hit(h, vol, dims, dtype: int, threshold: int, direction: int, xyz,
                  stream=None) -> int:
    vp = vol if isinstance(vol, int) else vol.data_ptr()
    xp = xyz if isinstance(xyz, int) else xyz.data_ptr()
    return lib().lnf_first_hit(h, vp, _dims_t(*[int(v) for v in dims]), dtype, int(threshold),
                               int(direction), xp, stream_ptr(stream))


def lnf_filter_surface(h, vol, dims, dtype: int, radius: int, threshold: int, direction: int,
                       xyz, out, stream=None) -> int:
    vp = vol if isinstance(vol, int) else vol.data_ptr()
    xp = xyz if isinstance(xyz, int) else xyz.data_ptr()
    op = out if isinstance(out, int) else out.data_ptr()
    return lib().lnf_filter_surface(h, vp, _dims_t(*[int(v) for v in dims]), dtype, int(radius),
                                    int(threshold), int(direction), xp, op, stream_ptr(stream))


def lnf_filter_points(h, vol, dims, dtype: int, radius: int, xyz, n: int, out, stream=None) -> int:
    vp = vol if isinstance(vol, int) else vol.data_ptr()
    xp = xyz if isinstance(xyz, int) else xyz.data_ptr()
    op = out if isinstance(out, int) else out.data_ptr()
    return lib().lnf_filter_points(h, vp, _dims_t(*[int(v) for v in dims]), dtype, radius, xp,
                                   int(n), op, stream_ptr(stream))
