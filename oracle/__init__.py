"""ctypes binding of the CPU oracle (libks_oracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the package smoke check and the
CPU-baseline leg of the benchmark.  The GPU library never imports, links or runs
anything here.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libks_oracle.so")
SRC = os.path.join(HERE, "ks_oracle.c")

QUADRANT, MEANSHIFT = 0, 1
STOP_NAMES = {0: "max_iter", 1: "zero_move", 2: "clamped", 3: "rejected"}


def compile_oracle(out: str = LIB_PATH) -> str:
    """gcc -O2 without FP contraction or host-specific code generation."""
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-o", out, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out


class Traj(C.Structure):
    _fields_ = [("traj", C.c_int64), ("x0", C.c_int32), ("y0", C.c_int32), ("z0", C.c_int32),
                ("x", C.c_int32), ("y", C.c_int32), ("z", C.c_int32), ("scale", C.c_int32),
                ("iters", C.c_int32), ("stop", C.c_int32), ("keep", C.c_int32), ("objective", C.c_double),
                ("h64", C.c_double), ("w64", C.c_double), ("y64", C.c_double), ("h_ref", C.c_double),
                ("y_ref", C.c_double)]


class Region(C.Structure):
    _fields_ = [("x", C.c_int32), ("y", C.c_int32), ("z", C.c_int32), ("scale", C.c_int32),
                ("saliency", C.c_double), ("entropy", C.c_double), ("pdf_change", C.c_double),
                ("key", C.c_double), ("seed", C.c_int64)]


class Ellipsoid(C.Structure):
    _fields_ = [("id", C.c_int64), ("x0", C.c_int32), ("y0", C.c_int32), ("z0", C.c_int32), ("radius", C.c_int32),
                ("x", C.c_double * 3), ("h", C.c_double * 6), ("rho", C.c_double), ("entropy", C.c_double),
                ("iters", C.c_int32), ("stop", C.c_int32)]


ABM_STOP = {"max_iter": 0, "converged": 1, "deteriorated": 2, "empty": 3, "degenerate": 4}
ABM_TOL = 0.01


class Stats(C.Structure):
    _fields_ = [("evals", C.c_int64), ("window_evals", C.c_int64), ("voxel_visits", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
            compile_oracle()
        L = C.CDLL(LIB_PATH)
        i32p = C.POINTER(C.c_int32)
        L.kso_bin_volume.argtypes = [C.c_void_p, C.c_int32, i32p, C.c_int32, C.c_void_p]
        L.kso_entropy64.argtypes = [C.c_void_p, C.c_int32]
        L.kso_entropy64.restype = C.c_double
        L.kso_entropy_ref.argtypes = [C.c_void_p, C.c_int32]
        L.kso_entropy_ref.restype = C.c_double
        L.kso_hist_cube.argtypes = [C.c_void_p, i32p, C.c_int32] + [C.c_int32] * 4 + [C.c_void_p]
        L.kso_hist_octant.argtypes = [C.c_void_p, i32p, C.c_int32] + [C.c_int32] * 5 + [C.c_void_p]
        L.kso_eval_quadrant.argtypes = [C.c_void_p, i32p, C.c_int32, i32p, C.c_int32, C.c_int32,
                                        C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.c_void_p]
        L.kso_eval_meanshift.argtypes = [C.c_void_p, i32p, C.c_int32, i32p, C.c_int32, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]
        L.kso_num_trajectories.argtypes = [i32p, C.c_int32, i32p, C.c_int32]
        L.kso_num_trajectories.restype = C.c_int64
        L.kso_run.argtypes = [C.c_void_p, C.c_int32, i32p, C.c_int32, i32p, C.c_int32, i32p, C.c_int32,
                              C.c_int32, C.c_double, C.c_double, C.c_void_p, C.c_int64, C.c_void_p,
                              C.POINTER(Stats)]
        L.kso_saliency_map.argtypes = [C.c_void_p, C.c_int32, i32p, C.c_int32, i32p, i32p, C.c_void_p,
                                       C.c_void_p, C.c_void_p]
        L.kso_bin_volume_window.argtypes = [C.c_void_p, C.c_int32, i32p, C.c_int32, C.c_int32, C.c_int32,
                                            C.c_void_p]
        L.kso_detect.argtypes = [C.c_void_p, C.c_int32, i32p, C.c_int32, i32p, C.c_int32, i32p, C.c_int32,
                                 C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_void_p, C.c_int32, i32p,
                                 C.POINTER(Stats)]
        L.kso_run_seeded.argtypes = [C.c_void_p, C.c_int32, i32p, C.c_int32, i32p, C.c_void_p, C.c_int64, i32p,
                                     C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_void_p, C.POINTER(Stats)]
        L.kso_detect_seeded.argtypes = [C.c_void_p, C.c_int32, i32p, C.c_int32, i32p, C.c_void_p, C.c_int64, i32p,
                                        C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_void_p,
                                        C.c_int32, i32p, C.POINTER(Stats)]
        L.kso_abmsod.argtypes = [C.c_void_p, C.c_int32, i32p, C.c_int32, i32p, C.c_int32, C.c_void_p, C.c_int64,
                                 i32p, C.c_int32, C.c_double, C.c_void_p, C.c_int64, C.c_void_p, C.POINTER(Stats)]
        L.kso_rank.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_int32, i32p]
        L.kso_set_readings.argtypes = [C.c_int32, C.c_int32]
        L.kso_set_abm_readings.argtypes = [C.c_int32, C.c_int32]
        _lib = L
    return _lib


@contextlib.contextmanager
def readings(sequential_sums=False, ln_n_form=False):
    """Runs the oracle under other readings of two points the paper leaves open
    (sums over bins in ascending order instead of the pairwise tree; H64 =
    ln N - S/N instead of (N ln N - S)/N), then restores the default ones."""
    lib().kso_set_readings(int(sequential_sums), int(ln_n_form))
    try:
        yield
    finally:
        lib().kso_set_readings(0, 0)


@contextlib.contextmanager
def abm_readings(convergence_stop=True, bandwidth_cap=True):
    """Runs the oracle's ABMSOD search with or without its two additions to
    Alg. 2 (the convergence stop; the bandwidth cap), then restores both."""
    lib().kso_set_abm_readings(int(convergence_stop), int(bandwidth_cap))
    try:
        yield
    finally:
        lib().kso_set_abm_readings(1, 1)


def _i3(v):
    return (C.c_int32 * 3)(*[int(a) for a in v])


def _dims(vol: np.ndarray):
    z, y, x = vol.shape
    return _i3((x, y, z))


_DT = {np.dtype(np.uint8): 0, np.dtype(np.uint16): 1, np.dtype(np.int16): 2}


def bin_volume(vol: np.ndarray, bins: int, window=None) -> np.ndarray:
    """Bin volume; with window = (lo, hi) the window-level binning (voxels outside
    get the value `bins`, ignored by every histogram)."""
    vol = np.ascontiguousarray(vol)
    out = np.empty(vol.shape, np.uint8)
    if window is None:
        lib().kso_bin_volume(vol.ctypes.data, _DT[vol.dtype], _dims(vol), bins, out.ctypes.data)
    else:
        lib().kso_bin_volume_window(vol.ctypes.data, _DT[vol.dtype], _dims(vol), bins, int(window[0]),
                                    int(window[1]), out.ctypes.data)
    return out


def _win(window):
    return None if window is None else (C.c_int32 * 2)(int(window[0]), int(window[1]))


def entropy64(counts) -> float:
    c = np.ascontiguousarray(counts, dtype=np.uint32)
    return lib().kso_entropy64(c.ctypes.data, c.size)


def entropy_ref(counts) -> float:
    c = np.ascontiguousarray(counts, dtype=np.uint32)
    return lib().kso_entropy_ref(c.ctypes.data, c.size)


def hist_cube(bv: np.ndarray, bins: int, p, s: int) -> np.ndarray:
    bv = np.ascontiguousarray(bv, dtype=np.uint8)
    out = np.zeros(bins, np.uint32)
    lib().kso_hist_cube(bv.ctypes.data, _dims(bv), bins, int(p[0]), int(p[1]), int(p[2]), int(s), out.ctypes.data)
    return out


def hist_octant(bv: np.ndarray, bins: int, p, j: int, k: int) -> np.ndarray:
    bv = np.ascontiguousarray(bv, dtype=np.uint8)
    out = np.zeros(bins, np.uint32)
    lib().kso_hist_octant(bv.ctypes.data, _dims(bv), bins, int(p[0]), int(p[1]), int(p[2]), int(j), int(k),
                          out.ctypes.data)
    return out


def eval_quadrant(bv: np.ndarray, bins: int, p, s_min: int, s_max: int):
    bv = np.ascontiguousarray(bv, dtype=np.uint8)
    S = s_max - s_min + 1
    eps = np.zeros((8, S), np.float64)
    kstar = np.zeros(8, np.int32)
    E = C.c_double()
    delta = np.zeros(3, np.float64)
    lib().kso_eval_quadrant(bv.ctypes.data, _dims(bv), bins, _i3(p), s_min, s_max, eps.ctypes.data,
                            kstar.ctypes.data, C.byref(E), delta.ctypes.data)
    return eps, kstar, E.value, delta


def eval_meanshift(bv: np.ndarray, bins: int, p, s: int):
    bv = np.ascontiguousarray(bv, dtype=np.uint8)
    counts = np.zeros(bins, np.uint32)
    msum = np.zeros((bins, 3), np.int64)
    delta = np.zeros(3, np.float64)
    rho = C.c_double()
    lib().kso_eval_meanshift(bv.ctypes.data, _dims(bv), bins, _i3(p), s, counts.ctypes.data, msum.ctypes.data,
                             delta.ctypes.data, C.byref(rho))
    return counts, msum, delta, rho.value


def num_trajectories(dims, spacing, scales, method) -> int:
    return lib().kso_num_trajectories(_i3(dims), spacing, (C.c_int32 * 2)(*scales), method)


TRAJ_FIELDS = [f[0] for f in Traj._fields_]


def _seeds(seeds):
    a = np.ascontiguousarray(np.asarray(seeds, dtype=np.int32).reshape(-1, 3))
    return a, a.shape[0]


def run(vol: np.ndarray, bins, spacing, scales, method, max_iter, ids=None, h_min=0.0, y_min=0.0, window=None,
        seeds=None):
    """Run trajectories (all, or the listed ids), from the seed grid or, with
    seeds = [(x, y, z), ...], from those positions.  Returns (structured array,
    stats dict)."""
    vol = np.ascontiguousarray(vol)
    z, y, x = vol.shape
    if seeds is not None:
        if ids is not None:
            raise ValueError("ids and seeds are exclusive")
        sa, ns = _seeds(seeds)
        n = ns * (scales[1] - scales[0] + 1 if method == MEANSHIFT else 1)
        out = (Traj * max(n, 1))()
        st = Stats()
        if lib().kso_run_seeded(vol.ctypes.data, _DT[vol.dtype], _dims(vol), bins, _win(window), sa.ctypes.data, ns,
                                (C.c_int32 * 2)(*scales), method, max_iter, h_min, y_min, out, C.byref(st)) != 0:
            raise ValueError("seed outside the volume")
        arr = np.ctypeslib.as_array(out)[:n].copy()
        return arr, {"evals": st.evals, "window_evals": st.window_evals, "voxel_visits": st.voxel_visits}
    if ids is None:
        n = num_trajectories((x, y, z), spacing, scales, method)
        idp = None
    else:
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        n = ids.size
        idp = ids.ctypes.data
    out = (Traj * max(n, 1))()
    st = Stats()
    lib().kso_run(vol.ctypes.data, _DT[vol.dtype], _dims(vol), bins, _win(window), spacing,
                  (C.c_int32 * 2)(*scales), method, max_iter, h_min, y_min, idp, n, out, C.byref(st))
    arr = np.ctypeslib.as_array(out)[:n].copy()
    return arr, {"evals": st.evals, "window_evals": st.window_evals, "voxel_visits": st.voxel_visits}


RANK_SALIENCY, RANK_PDF_CHANGE = 0, 1


def saliency_map(vol: np.ndarray, bins, scales, window=None):
    """Every-voxel Kadir-Brady map: (saliency float32, scale uint8, saliency64
    float64), each shaped like vol; scale 0 and saliency 0 where there is no
    entropy peak."""
    vol = np.ascontiguousarray(vol)
    sal = np.zeros(vol.shape, np.float32)
    scl = np.zeros(vol.shape, np.uint8)
    s64 = np.zeros(vol.shape, np.float64)
    lib().kso_saliency_map(vol.ctypes.data, _DT[vol.dtype], _dims(vol), bins, _win(window),
                           (C.c_int32 * 2)(*scales), sal.ctypes.data, scl.ctypes.data, s64.ctypes.data)
    return sal, scl, s64


def detect(vol: np.ndarray, bins, spacing, scales, method, max_iter, capacity=None, h_min=0.0, y_min=0.0,
           rank_by=RANK_SALIENCY, window=None, seeds=None):
    """Full detection from the seed grid or, with seeds = [(x, y, z), ...], from
    those positions; returns (structured array of regions, n_found, stats dict)."""
    vol = np.ascontiguousarray(vol)
    z, y, x = vol.shape
    if seeds is not None:
        sa, ns = _seeds(seeds)
        ntraj = ns * (scales[1] - scales[0] + 1 if method == MEANSHIFT else 1)
    else:
        ntraj = num_trajectories((x, y, z), spacing, scales, method)
    if capacity is None:
        capacity = max(1, ntraj)
    out = (Region * max(capacity, 1))()
    nf = C.c_int32()
    st = Stats()
    if seeds is not None:
        rc = lib().kso_detect_seeded(vol.ctypes.data, _DT[vol.dtype], _dims(vol), bins, _win(window), sa.ctypes.data,
                                     ns, (C.c_int32 * 2)(*scales), method, max_iter, h_min, y_min, rank_by, out,
                                     capacity, C.byref(nf), C.byref(st))
        if rc != 0:
            raise ValueError("seed outside the volume")
    else:
        lib().kso_detect(vol.ctypes.data, _DT[vol.dtype], _dims(vol), bins, _win(window), spacing,
                         (C.c_int32 * 2)(*scales), method, max_iter, h_min, y_min, rank_by, out, capacity,
                         C.byref(nf), C.byref(st))
    arr = np.ctypeslib.as_array(out)[:min(capacity, nf.value)].copy()
    return arr, nf.value, {"evals": st.evals, "window_evals": st.window_evals, "voxel_visits": st.voxel_visits}


def rank(traj: np.ndarray, rank_by=RANK_SALIENCY, capacity=None):
    """Step 8 alone on trajectory records of `run` (one run, or its shards
    concatenated in any order): (structured array of regions, n_found)."""
    t = np.ascontiguousarray(traj, dtype=np.dtype(Traj))
    n = t.shape[0]
    if capacity is None:
        capacity = max(1, n)
    out = (Region * max(capacity, 1))()
    nf = C.c_int32()
    if lib().kso_rank(t.ctypes.data, n, rank_by, out, capacity, C.byref(nf)) != 0:
        raise MemoryError("kso_rank")
    return np.ctypeslib.as_array(out)[:min(capacity, nf.value)].copy(), nf.value


def abmsod(vol: np.ndarray, bins, spacing, radii, max_iter, threshold=0.0, seeds=None, ids=None, window=None):
    """ABMSOD candidates (grid or seed list x radii, or the listed ids).  Returns
    (structured array with fields id, x0, y0, z0, radius, x[3], h[6], rho,
    entropy, iters, stop; stats dict)."""
    vol = np.ascontiguousarray(vol)
    z, y, x = vol.shape
    R = radii[1] - radii[0] + 1
    if seeds is not None:
        sa, ns = _seeds(seeds)
        sp_, nstart = sa.ctypes.data, ns
    else:
        sa, sp_, ns = None, None, 0
        nstart = num_trajectories((x, y, z), spacing, (1, 1), QUADRANT)
    if ids is None:
        n, idp = nstart * R, None
    else:
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        n, idp = ids.size, ids.ctypes.data
    out = (Ellipsoid * max(n, 1))()
    st = Stats()
    rc = lib().kso_abmsod(vol.ctypes.data, _DT[vol.dtype], _dims(vol), bins, _win(window), spacing, sp_, ns,
                          (C.c_int32 * 2)(*radii), max_iter, float(threshold), idp, n, out, C.byref(st))
    if rc != 0:
        raise ValueError("seed outside the volume or bad radii")
    arr = np.ctypeslib.as_array(out)[:n].copy()
    return arr, {"evals": st.evals, "window_evals": st.window_evals, "voxel_visits": st.voxel_visits}
