"""ctypes binding of libks.so (the gfx950 library), one function per C entry point.

Argument marshalling only: every step of the detection runs in the library's
kernels.  Device volumes are torch tensors on a ROCm device, shape (Z, Y, X),
dtype uint8, uint16 or int16, contiguous.  Importing this module does not load
the library; the first call does, and raises if it is not built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libks.so")

KS_OK, KS_E_INVALID, KS_E_NOMEM, KS_E_DEVICE, KS_E_TOO_LARGE, KS_E_NOT_READY, KS_E_SHUTDOWN = 0, -1, -2, -3, -4, -5, -6
KS_U8, KS_U16, KS_I16 = 0, 1, 2
KS_QUADRANT, KS_MEANSHIFT = 0, 1
KS_RANK_SALIENCY, KS_RANK_PDF_CHANGE = 0, 1
KS_HIST_CUBE, KS_HIST_OCTANTS, KS_HIST_MEANSHIFT, KS_HIST_SHELLS, KS_HIST_MS_MOVE, KS_HIST_MS_INNER = 0, 1, 2, 3, 4, 5

EXPORTS = [
    "ks_status_str", "ks_context_create", "ks_context_destroy", "ks_context_set_profiling", "ks_context_set_tuning",
    "ks_last_stats", "ks_detect", "ks_detect_device", "ks_seed_traces", "ks_bin_volume", "ks_histograms",
    "ks_detect_batch", "ks_server_create", "ks_server_submit", "ks_server_poll", "ks_server_drain",
    "ks_server_stats", "ks_server_reset_stats", "ks_server_destroy", "ks_roofline", "ks_context_set_tuning_small",
    "ks_context_set_ms_update", "ks_context_set_options", "ks_saliency_map", "ks_context_set_seeds",
    "ks_server_submit_tracked", "ks_abmsod", "ks_context_set_overlap", "ks_context_autotune",
    "ks_context_set_ms_group", "ks_count_roots", "ks_detect_device_noalloc", "ks_context_set_ms_chunks",
    "ks_context_autotune_batch",
]


class KsError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_str(status)} ({status})")
        self.status = status


class Region(C.Structure):
    _fields_ = [("x", C.c_int32), ("y", C.c_int32), ("z", C.c_int32), ("scale", C.c_int32),
                ("saliency", C.c_float), ("entropy", C.c_float), ("pdf_change", C.c_float), ("seed", C.c_int32)]


class SeedTrace(C.Structure):
    _fields_ = [("x0", C.c_int32), ("y0", C.c_int32), ("z0", C.c_int32), ("x", C.c_int32), ("y", C.c_int32),
                ("z", C.c_int32), ("scale", C.c_int32), ("iters", C.c_int32), ("stop", C.c_int32),
                ("keep", C.c_int32), ("objective", C.c_double), ("saliency64", C.c_double),
                ("saliency", C.c_float), ("entropy", C.c_float), ("pdf_change", C.c_float), ("pad", C.c_int32)]


class RunStats(C.Structure):
    _fields_ = [("trajectories", C.c_int64), ("evals", C.c_int64), ("window_evals", C.c_int64),
                ("voxel_visits", C.c_int64), ("final_visits", C.c_int64), ("regions", C.c_int64),
                ("ms_prep", C.c_double), ("ms_search", C.c_double), ("ms_rank", C.c_double),
                ("ms_total", C.c_double), ("swept_voxels", C.c_int64), ("lds_ops", C.c_int64),
                ("ms_search_quad", C.c_double), ("ms_search_ms", C.c_double)]


class Options(C.Structure):
    _fields_ = [("h_min", C.c_double), ("y_min", C.c_double), ("rank_by", C.c_int32), ("window", C.c_int32),
                ("win_lo", C.c_int32), ("win_hi", C.c_int32)]


def options(h_min=0.0, y_min=0.0, rank_by=0, window=None) -> Options:
    """Selection and binning options; window = (lo, hi) for a window level."""
    o = Options()
    o.h_min, o.y_min, o.rank_by = float(h_min), float(y_min), int(rank_by)
    o.window, o.win_lo, o.win_hi = (0, 0, 0) if window is None else (1, int(window[0]), int(window[1]))
    return o


class Ellipsoid(C.Structure):
    _fields_ = [("x0", C.c_int32), ("y0", C.c_int32), ("z0", C.c_int32), ("radius", C.c_int32),
                ("x", C.c_double * 3), ("h", C.c_double * 6), ("rho", C.c_double), ("entropy", C.c_double),
                ("iters", C.c_int32), ("stop", C.c_int32)]


KS_ABM_MAX_ITER, KS_ABM_CONVERGED, KS_ABM_DETERIORATED, KS_ABM_EMPTY, KS_ABM_DEGENERATE = 0, 1, 2, 3, 4


class Request(C.Structure):
    _fields_ = [("volume", C.c_void_p), ("dtype", C.c_int32), ("dims", C.c_int32 * 3), ("bins", C.c_int32),
                ("seed_spacing", C.c_int32), ("scales", C.c_int32 * 2), ("method", C.c_int32),
                ("max_iter", C.c_int32), ("options", Options), ("seeds", C.POINTER(C.c_int32)),
                ("n_seeds", C.c_int64), ("max_regions", C.c_int32), ("reserved", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("regions", C.POINTER(Region)), ("capacity", C.c_int32), ("n_found", C.c_int32),
                ("status", C.c_int32), ("pad", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64), ("refused", C.c_int64),
                ("queued_now", C.c_int64), ("in_flight", C.c_int64), ("bytes_in_use", C.c_int64),
                ("budget_bytes", C.c_int64), ("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("mean_ms", C.c_double), ("volumes_per_s", C.c_double), ("bytes_peak", C.c_int64)]


_lib = None


def lib():
    """Loads libks.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    L = C.CDLL(LIB_PATH)
    vp, i32, i32p = C.c_void_p, C.c_int32, C.POINTER(C.c_int32)
    L.ks_status_str.argtypes = [i32]
    L.ks_status_str.restype = C.c_char_p
    L.ks_context_create.argtypes = [i32, C.POINTER(vp)]
    L.ks_context_destroy.argtypes = [vp]
    L.ks_context_set_profiling.argtypes = [vp, i32]
    L.ks_context_set_tuning.argtypes = [vp, i32, i32]
    L.ks_context_set_tuning_small.argtypes = [vp, i32, i32]
    L.ks_context_set_ms_update.argtypes = [vp, i32]
    L.ks_context_set_options.argtypes = [vp, C.POINTER(Options)]
    L.ks_saliency_map.argtypes = [vp, vp, i32, C.POINTER(C.c_int32), i32, C.POINTER(C.c_int32), vp, vp, vp]
    L.ks_last_stats.argtypes = [vp, C.POINTER(RunStats)]
    L.ks_detect.argtypes = [vp, i32, i32p, i32, i32, i32p, i32, i32, vp, i32, i32p]
    L.ks_detect_device.argtypes = [vp, vp, i32, i32p, i32, i32, i32p, i32, i32, vp, i32, i32p, vp]
    L.ks_seed_traces.argtypes = [vp, vp, i32, i32p, i32, i32, i32p, i32, i32, vp, i32, i32p, vp]
    L.ks_bin_volume.argtypes = [vp, vp, i32, i32p, i32, vp, vp]
    L.ks_histograms.argtypes = [vp, vp, i32, i32p, i32, i32, i32p, i32, vp, vp, vp, vp]
    L.ks_detect_batch.argtypes = [vp, i32, C.POINTER(Request), C.POINTER(Result), vp]
    L.ks_server_create.argtypes = [i32, C.c_size_t, i32, C.POINTER(vp)]
    L.ks_server_submit.argtypes = [vp, C.POINTER(Request), C.POINTER(C.c_uint64)]
    L.ks_server_submit_tracked.argtypes = [vp, C.POINTER(Request), C.c_int64, i32, C.POINTER(C.c_uint64)]
    L.ks_context_set_seeds.argtypes = [vp, i32p, C.c_int64]
    L.ks_context_set_overlap.argtypes = [vp, i32]
    L.ks_context_set_ms_group.argtypes = [vp, i32]
    L.ks_context_set_ms_chunks.argtypes = [vp, i32]
    L.ks_context_autotune_batch.argtypes = [vp, i32, C.POINTER(Request), i32, i32p, vp]
    L.ks_context_autotune.argtypes = [vp, vp, i32, i32p, i32, i32, i32p, i32, i32, i32, i32p, vp]
    L.ks_abmsod.argtypes = [vp, vp, i32, i32p, i32, i32, i32p, i32, C.c_double, vp, i32, i32p, vp]
    L.ks_server_poll.argtypes = [vp, C.c_uint64, vp, i32, i32p]
    L.ks_server_drain.argtypes = [vp]
    L.ks_server_stats.argtypes = [vp, C.POINTER(ServerStats)]
    L.ks_server_reset_stats.argtypes = [vp]
    L.ks_server_destroy.argtypes = [vp]
    L.ks_roofline.argtypes = [i32, i32, C.POINTER(C.c_double)]
    L.ks_count_roots.argtypes = [vp, i32, vp, vp, vp]
    L.ks_detect_device_noalloc.argtypes = [vp, vp, i32, i32p, i32, i32, i32p, i32, i32, vp, i32, i32p, vp]
    for name in EXPORTS:
        if name != "ks_status_str":
            getattr(L, name).restype = i32
    _lib = L
    return L


def status_str(status: int) -> str:
    try:
        return lib().ks_status_str(status).decode()
    except Exception:  # library missing: still format the error
        return str(status)


def _check(status: int, what: str):
    if status != KS_OK:
        raise KsError(status, what)


def _i3(v):
    return (C.c_int32 * 3)(*[int(a) for a in v])


def _i2(v):
    return (C.c_int32 * 2)(*[int(a) for a in v])


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


_NP_DTYPE = {np.dtype(np.uint8): KS_U8, np.dtype(np.uint16): KS_U16, np.dtype(np.int16): KS_I16}


def _torch_dtype_code(t):
    import torch
    codes = {torch.uint8: KS_U8, torch.int16: KS_I16}
    if hasattr(torch, "uint16"):
        codes[torch.uint16] = KS_U16
    if t.dtype not in codes:
        raise TypeError(f"unsupported volume dtype {t.dtype}")
    return codes[t.dtype]


def _volume_args(t):
    """(device pointer, dtype code, dims) of a (Z, Y, X) device tensor."""
    if not t.is_cuda:
        raise ValueError("volume must be a device tensor")
    if not t.is_contiguous():
        raise ValueError("volume must be contiguous")
    if t.dim() != 3:
        raise ValueError("volume must have shape (Z, Y, X)")
    z, y, x = t.shape
    return C.c_void_p(t.data_ptr()), _torch_dtype_code(t), _i3((x, y, z))


# ks_region as a numpy record (the same fields, offsets and size as Region)
REGION_DTYPE = np.dtype([("x", "<i4"), ("y", "<i4"), ("z", "<i4"), ("scale", "<i4"), ("saliency", "<f4"),
                         ("entropy", "<f4"), ("pdf_change", "<f4"), ("seed", "<i4")])
assert REGION_DTYPE.itemsize == C.sizeof(Region)


def _region_buffer(capacity):
    """A numpy array of capacity ks_region records and its address for the library
    to fill (numpy-owned: converting a ctypes array costs far more per call)."""
    a = np.empty(max(int(capacity), 1), REGION_DTYPE)
    return a, C.c_void_p(a.ctypes.data)


def _regions(buf, n_found, capacity):
    # a view of the written records (a structured copy costs tens of microseconds)
    return buf[:max(0, min(int(n_found), int(capacity)))]


class Context:
    """A library context on one device (tables, work arena, graph cache)."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(lib().ks_context_create(int(device), C.byref(h)), "ks_context_create")
        self.handle = h

    def close(self):
        if self.handle:
            lib().ks_context_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ks_context_set_profiling(ctx: Context, on: bool):
    _check(lib().ks_context_set_profiling(ctx.handle, 1 if on else 0), "ks_context_set_profiling")


def ks_context_set_tuning(ctx: Context, ms_replicas_log2: int, quad_replicas_log2: int):
    _check(lib().ks_context_set_tuning(ctx.handle, ms_replicas_log2, quad_replicas_log2), "ks_context_set_tuning")


def ks_saliency_map(ctx: Context, volume, bins, scales, stream=None):
    """Dense Kadir-Brady map of a device volume (torch tensor (Z, Y, X)): returns
    (saliency float32, scale uint8) device tensors of the same shape."""
    import torch

    ptr, dt, dims = _volume_args(volume)
    sal = torch.empty(tuple(volume.shape), dtype=torch.float32, device=volume.device)
    scl = torch.empty(tuple(volume.shape), dtype=torch.uint8, device=volume.device)
    _check(lib().ks_saliency_map(ctx.handle, ptr, dt, dims, bins, _i2(scales), C.c_void_p(sal.data_ptr()),
                                 C.c_void_p(scl.data_ptr()), _stream_ptr(stream)), "ks_saliency_map")
    return sal, scl


def ks_context_set_options(ctx: Context, opts=None):
    """Selection thresholds and rank key for later ks_detect_device / ks_seed_traces
    calls on ctx (None: the defaults)."""
    _check(lib().ks_context_set_options(ctx.handle, None if opts is None else C.byref(opts)),
           "ks_context_set_options")


def _seed_array(seeds):
    a = np.ascontiguousarray(np.asarray(seeds, dtype=np.int32).reshape(-1, 3))
    return a, a.shape[0]


def ks_context_set_seeds(ctx: Context, seeds=None):
    """Start positions [(x, y, z), ...] for later ks_detect_device / ks_seed_traces
    calls on ctx, in place of the seed grid (None: the grid)."""
    if seeds is None:
        _check(lib().ks_context_set_seeds(ctx.handle, None, 0), "ks_context_set_seeds")
        return
    a, n = _seed_array(seeds)
    _check(lib().ks_context_set_seeds(ctx.handle, a.ctypes.data_as(C.POINTER(C.c_int32)), n),
           "ks_context_set_seeds")


def ks_context_autotune(ctx: Context, volume, bins, seed_spacing, scales, method, max_iter, reps=2, stream=None):
    """Times the search of this request under candidate tunings and keeps the
    fastest in ctx; returns (ms_replicas_log2, ms_small_replicas_log2, s_small,
    quad_replicas_log2)."""
    ptr, dt, dims = _volume_args(volume)
    out = (C.c_int32 * 4)()
    _check(lib().ks_context_autotune(ctx.handle, ptr, dt, dims, bins, seed_spacing, _i2(scales), method, max_iter,
                                     int(reps), out, _stream_ptr(stream)), "ks_context_autotune")
    return tuple(out)


def ks_context_set_ms_group(ctx: Context, scales_per_task: int = 0):
    _check(lib().ks_context_set_ms_group(ctx.handle, int(scales_per_task)), "ks_context_set_ms_group")


def ks_context_set_ms_chunks(ctx: Context, launches: int = 1):
    _check(lib().ks_context_set_ms_chunks(ctx.handle, int(launches)), "ks_context_set_ms_chunks")


def ks_context_set_overlap(ctx: Context, on: bool):
    _check(lib().ks_context_set_overlap(ctx.handle, int(bool(on))), "ks_context_set_overlap")


def ks_context_set_ms_update(ctx: Context, incremental_pct: int = 100):
    _check(lib().ks_context_set_ms_update(ctx.handle, incremental_pct), "ks_context_set_ms_update")


def ks_context_set_tuning_small(ctx: Context, ms_small_replicas_log2: int, s_small: int):
    _check(lib().ks_context_set_tuning_small(ctx.handle, ms_small_replicas_log2, s_small),
           "ks_context_set_tuning_small")


def ks_last_stats(ctx: Context) -> dict:
    st = RunStats()
    _check(lib().ks_last_stats(ctx.handle, C.byref(st)), "ks_last_stats")
    return {f: getattr(st, f) for f, _ in RunStats._fields_}


def ks_detect(volume: np.ndarray, bins, seed_spacing, scales, method, max_iter, capacity=1024):
    """Host volume (Z, Y, X) numpy array -> (regions, n_found)."""
    vol = np.ascontiguousarray(volume)
    z, y, x = vol.shape
    buf, out = _region_buffer(capacity)
    nf = C.c_int32()
    _check(lib().ks_detect(C.c_void_p(vol.ctypes.data), _NP_DTYPE[vol.dtype], _i3((x, y, z)), bins, seed_spacing,
                           _i2(scales), method, max_iter, out, int(capacity), C.byref(nf)), "ks_detect")
    return _regions(buf, nf.value, capacity), nf.value


def ks_detect_device(ctx: Context, volume, bins, seed_spacing, scales, method, max_iter, capacity=1024, stream=None):
    ptr, dt, dims = _volume_args(volume)
    buf, out = _region_buffer(capacity)
    nf = C.c_int32()
    _check(lib().ks_detect_device(ctx.handle, ptr, dt, dims, bins, seed_spacing, _i2(scales), method, max_iter, out,
                                  int(capacity), C.byref(nf), _stream_ptr(stream)), "ks_detect_device")
    return _regions(buf, nf.value, capacity), nf.value


def ks_detect_device_noalloc(ctx: Context, volume, bins, seed_spacing, scales, method, max_iter, capacity=1024,
                             stream=None):
    """ks_detect_device with its work memory in the library's static device array
    (no allocation by the call)."""
    ptr, dt, dims = _volume_args(volume)
    buf, out = _region_buffer(capacity)
    nf = C.c_int32()
    _check(lib().ks_detect_device_noalloc(ctx.handle, ptr, dt, dims, bins, seed_spacing, _i2(scales), method,
                                          max_iter, out, int(capacity), C.byref(nf), _stream_ptr(stream)),
           "ks_detect_device_noalloc")
    return _regions(buf, nf.value, capacity), nf.value


def ks_seed_traces(ctx: Context, volume, bins, seed_spacing, scales, method, max_iter, stream=None):
    ptr, dt, dims = _volume_args(volume)
    z, y, x = volume.shape
    n_est = C.c_int32()
    # first call with capacity 0 gives the trajectory count
    _check(lib().ks_seed_traces(ctx.handle, ptr, dt, dims, bins, seed_spacing, _i2(scales), method, max_iter, None, 0,
                                C.byref(n_est), _stream_ptr(stream)), "ks_seed_traces")
    out = (SeedTrace * max(n_est.value, 1))()
    n = C.c_int32()
    _check(lib().ks_seed_traces(ctx.handle, ptr, dt, dims, bins, seed_spacing, _i2(scales), method, max_iter, out,
                                n_est.value, C.byref(n), _stream_ptr(stream)), "ks_seed_traces")
    return np.ctypeslib.as_array(out)[:n.value].copy()


def ks_abmsod(ctx: Context, volume, bins, seed_spacing, radii, max_iter, threshold=0.0, stream=None):
    """ABMSOD candidates of a device volume (every start x every radius, in id
    order) as a structured array."""
    ptr, dt, dims = _volume_args(volume)
    n_est = C.c_int32()
    _check(lib().ks_abmsod(ctx.handle, ptr, dt, dims, bins, seed_spacing, _i2(radii), max_iter, float(threshold),
                           None, 0, C.byref(n_est), _stream_ptr(stream)), "ks_abmsod")
    out = (Ellipsoid * max(n_est.value, 1))()
    n = C.c_int32()
    _check(lib().ks_abmsod(ctx.handle, ptr, dt, dims, bins, seed_spacing, _i2(radii), max_iter, float(threshold),
                           out, n_est.value, C.byref(n), _stream_ptr(stream)), "ks_abmsod")
    return np.ctypeslib.as_array(out)[:n.value].copy()


def ks_bin_volume(ctx: Context, volume, bins, stream=None) -> np.ndarray:
    ptr, dt, dims = _volume_args(volume)
    out = np.empty(tuple(volume.shape), np.uint8)
    _check(lib().ks_bin_volume(ctx.handle, ptr, dt, dims, bins, C.c_void_p(out.ctypes.data), _stream_ptr(stream)),
           "ks_bin_volume")
    return out


def ks_histograms(ctx: Context, volume, bins, kind, xyz, scale=None, scale_range=(1, 1), stream=None) -> np.ndarray:
    """Window histograms through the search's device code.  KS_HIST_MS_MOVE takes
    xyz as (n, 6): P then Q per window."""
    ptr, dt, dims = _volume_args(volume)
    xyz = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1, 6 if kind == KS_HIST_MS_MOVE else 3)
    n = xyz.shape[0]
    K = scale_range[1] - scale_range[0] + 1
    if kind == KS_HIST_CUBE:
        out = np.zeros((n, bins), np.uint32)
    elif kind in (KS_HIST_MEANSHIFT, KS_HIST_MS_MOVE):
        out = np.zeros((n, 4, bins), np.int32)
    elif kind == KS_HIST_MS_INNER:
        out = np.zeros((n, 3, bins), np.uint32)
    elif kind == KS_HIST_OCTANTS:
        out = np.zeros((n, 8, K, bins), np.uint32)
    else:
        out = np.zeros((n, K, bins), np.uint32)
    sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.int32)
    _check(lib().ks_histograms(ctx.handle, ptr, dt, dims, bins, kind, _i2(scale_range), n,
                               C.c_void_p(xyz.ctypes.data), None if sc is None else C.c_void_p(sc.ctypes.data),
                               C.c_void_p(out.ctypes.data), _stream_ptr(stream)), "ks_histograms")
    return out


def ks_count_roots(ctx: Context, n: int, stream=None):
    """(sqrt(c), 1/sqrt(c)) for c in 0..n-1 as the mean-shift search computes them."""
    sq = np.empty(int(n), np.float64)
    rs = np.empty(int(n), np.float64)
    _check(lib().ks_count_roots(ctx.handle, int(n), C.c_void_p(sq.ctypes.data), C.c_void_p(rs.ctypes.data),
                                _stream_ptr(stream)), "ks_count_roots")
    return sq, rs


def make_request(volume, bins, seed_spacing, scales, method, max_iter, host=False, opts=None,
                 seeds=None) -> Request:
    """One batch or server request; seeds = [(x, y, z), ...] replaces the grid (the
    request keeps the array alive)."""
    r = Request()
    if opts is not None:
        r.options = opts
    if seeds is not None:
        a, n = _seed_array(seeds)
        r._seed_keep = a
        r.seeds = a.ctypes.data_as(C.POINTER(C.c_int32))
        r.n_seeds = n
    if host:
        vol = np.ascontiguousarray(volume)
        z, y, x = vol.shape
        r.volume = vol.ctypes.data
        r.dtype = _NP_DTYPE[vol.dtype]
    else:
        ptr, dt, _ = _volume_args(volume)
        z, y, x = volume.shape
        r.volume = ptr.value
        r.dtype = dt
    r.dims[0], r.dims[1], r.dims[2] = x, y, z
    r.bins, r.seed_spacing = bins, seed_spacing
    r.scales[0], r.scales[1] = scales
    r.method, r.max_iter = method, max_iter
    return r


def ks_detect_batch(ctx: Context, requests, capacity=1024, stream=None):
    """requests: list of Request (device volumes).  Returns a list of (regions, n_found)."""
    n = len(requests)
    reqs = (Request * max(n, 1))(*requests)
    bufs = [_region_buffer(capacity) for _ in range(n)]
    res = (Result * max(n, 1))()
    for i in range(n):
        res[i].regions = C.cast(bufs[i][1], C.POINTER(Region))
        res[i].capacity = int(capacity)
    _check(lib().ks_detect_batch(ctx.handle, n, reqs, res, _stream_ptr(stream)), "ks_detect_batch")
    return [(_regions(bufs[i][0], res[i].n_found, capacity), res[i].n_found) for i in range(n)]


def ks_context_autotune_batch(ctx: Context, requests, reps=2, stream=None):
    """Tunes the context for this batch; returns the chosen (ms_replicas_log2,
    ms_small_replicas_log2, s_small, quad_replicas_log2, ms_scales_per_task)."""
    n = len(requests)
    reqs = (Request * max(n, 1))(*requests)
    out = (C.c_int32 * 5)()
    _check(lib().ks_context_autotune_batch(ctx.handle, n, reqs, int(reps), out, _stream_ptr(stream)),
           "ks_context_autotune_batch")
    return tuple(out)


KS_ROOF_COPY, KS_ROOF_LDS_ADD64, KS_ROOF_LDS_ADD32, KS_ROOF_LDS_ADD64_SHARED4 = 0, 1, 2, 3


def ks_roofline(kind: int, device: int = 0) -> float:
    """Measured ceiling: bytes/s (copy) or lane-level LDS atomic adds/s."""
    r = C.c_double()
    _check(lib().ks_roofline(int(device), int(kind), C.byref(r)), "ks_roofline")
    return r.value


class Server:
    """Continuous-batching detection server (ks_server_*)."""

    def __init__(self, device: int = 0, hbm_budget: int = 8 << 30, max_slots: int = 8):
        h = C.c_void_p()
        _check(lib().ks_server_create(int(device), C.c_size_t(int(hbm_budget)), int(max_slots), C.byref(h)),
               "ks_server_create")
        self.handle = h
        self._limit = {}  # ticket -> max_regions of its request (0: none)

    def submit(self, volume: np.ndarray, bins, seed_spacing, scales, method, max_iter, opts=None, seeds=None,
               track=None, max_seeds=32, max_regions=0) -> int:
        """Queues a host volume; with track = an int id the request is a frame of
        that tracked sequence (started from the previous frame's regions);
        max_regions > 0 keeps only that many top regions for the poll."""
        r = make_request(volume, bins, seed_spacing, scales, method, max_iter, host=True, opts=opts, seeds=seeds)
        r.max_regions = int(max_regions)
        t = C.c_uint64()
        if track is None:
            _check(lib().ks_server_submit(self.handle, C.byref(r), C.byref(t)), "ks_server_submit")
        else:
            _check(lib().ks_server_submit_tracked(self.handle, C.byref(r), int(track), int(max_seeds), C.byref(t)),
                   "ks_server_submit_tracked")
        if max_regions:
            self._limit[t.value] = int(max_regions)
        return t.value

    def poll(self, ticket: int, capacity=1024):
        buf, out = _region_buffer(capacity)
        nf = C.c_int32()
        st = lib().ks_server_poll(self.handle, C.c_uint64(ticket), out, int(capacity), C.byref(nf))
        if st == KS_E_NOT_READY:
            return None
        _check(st, "ks_server_poll")
        limit = self._limit.pop(ticket, 0)
        written = min(nf.value, capacity, limit) if limit else min(nf.value, capacity)
        return _regions(buf, written, capacity), nf.value

    def drain(self):
        _check(lib().ks_server_drain(self.handle), "ks_server_drain")

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().ks_server_stats(self.handle, C.byref(st)), "ks_server_stats")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def reset_stats(self):
        _check(lib().ks_server_reset_stats(self.handle), "ks_server_reset_stats")

    def close(self):
        if self.handle:
            lib().ks_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
