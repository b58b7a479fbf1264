"""Seeded synthetic volumes and workload descriptions.

The paper evaluates on PET volumes (128x128x34, Sec. 3.1) and brain MR volumes
(256x256x176, Sec. 3.2) that are not available here.  These generators produce
stand-ins with the same sizes, value ranges and structure: a few high-entropy
objects (spheres, an ellipsoidal myocardium-like shell, heterogeneous blobs) in a
low-entropy background.  They hold none of the detection arithmetic: both the
CPU oracle and the GPU library consume their output unchanged.

Arrays are returned with shape (Z, Y, X) in C order, so x is the fastest axis,
matching the dims = (X, Y, Z) convention of the C boundary.
"""
from __future__ import annotations

import dataclasses
from typing import List, Tuple

import numpy as np

U8, U16, I16 = 0, 1, 2
QUADRANT, MEANSHIFT = 0, 1
DTYPE_CODE = {np.dtype(np.uint8): U8, np.dtype(np.uint16): U16, np.dtype(np.int16): I16}


@dataclasses.dataclass
class Workload:
    """One detection request: the volume plus the search parameters."""
    name: str
    volume: np.ndarray  # (Z, Y, X)
    bins: int
    spacing: int
    scales: Tuple[int, int]
    method: int
    max_iter: int

    @property
    def dims(self) -> Tuple[int, int, int]:
        z, y, x = self.volume.shape
        return (x, y, z)

    @property
    def dtype_code(self) -> int:
        return DTYPE_CODE[self.volume.dtype]


def _grid(shape):
    z, y, x = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), np.arange(shape[2]), indexing="ij")
    return x, y, z


def spheres_volume(seed: int, dims=(64, 64, 64), n_spheres: int = 3) -> np.ndarray:
    """uint8: background N(40,5) clipped to [0,255]; spheres of radius 6..10 whose
    interiors are i.i.d. uniform over [0,255]; later spheres overwrite earlier ones."""
    rng = np.random.default_rng(seed)
    X, Y, Z = dims
    shape = (Z, Y, X)
    vol = np.clip(np.rint(rng.normal(40.0, 5.0, shape)), 0, 255).astype(np.uint8)
    x, y, z = _grid(shape)
    for _ in range(n_spheres):
        r = int(rng.integers(6, 11))
        c = [int(rng.integers(r, d - r)) for d in (X, Y, Z)]
        m = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 <= r * r
        vol[m] = rng.integers(0, 256, int(m.sum())).astype(np.uint8)
    return vol


def shell_volume(seed: int, dims=(128, 128, 64)) -> np.ndarray:
    """uint16 (12-bit) PET-like volume: an axis-aligned ellipsoidal shell with outer
    semi-axes (18,14,14) and thickness 4 at mean 2500 over a background of mean 300,
    Poisson noise, clipped to [0,4095]."""
    rng = np.random.default_rng(seed)
    X, Y, Z = dims
    shape = (Z, Y, X)
    outer = (18, 14, 14)
    inner = (14, 10, 10)
    c = [int(rng.integers(a + 8, d - a - 8)) for a, d in zip(outer, (X, Y, Z))]
    x, y, z = _grid(shape)
    qo = ((x - c[0]) / outer[0]) ** 2 + ((y - c[1]) / outer[1]) ** 2 + ((z - c[2]) / outer[2]) ** 2
    qi = ((x - c[0]) / inner[0]) ** 2 + ((y - c[1]) / inner[1]) ** 2 + ((z - c[2]) / inner[2]) ** 2
    mean = np.where((qo <= 1.0) & (qi > 1.0), 2500.0, 300.0)
    return np.clip(rng.poisson(mean), 0, 4095).astype(np.uint16)


def blobs_volume(seed: int, dims=(256, 256, 160)) -> np.ndarray:
    """int16 MR-like volume: Gaussian-smoothed (sigma 6) white noise min-max scaled to
    [0,1200], plus 1..4 spherical tumour blobs (radius 8..20) with interiors i.i.d.
    uniform over [200,3000]."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    X, Y, Z = dims
    shape = (Z, Y, X)
    bg = gaussian_filter(rng.normal(0.0, 1.0, shape), sigma=6.0, mode="reflect", truncate=4.0)
    lo, hi = float(bg.min()), float(bg.max())
    vol = np.rint((bg - lo) / (hi - lo) * 1200.0).astype(np.int16)
    x, y, z = _grid(shape)
    for _ in range(int(rng.integers(1, 5))):
        r = int(rng.integers(8, 21))
        c = [int(rng.integers(r, d - r)) for d in (X, Y, Z)]
        m = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 <= r * r
        vol[m] = rng.integers(200, 3001, int(m.sum())).astype(np.int16)
    return vol


# Per-type search parameters: (bins, spacing, scales, method, max_iter).
TYPE_PARAMS = {
    0: (32, 8, (3, 8), QUADRANT, 50),
    1: (64, 6, (4, 16), QUADRANT, 50),
    2: (64, 8, (4, 24), MEANSHIFT, 100),
}
TYPE_GEN = {0: spheres_volume, 1: shell_volume, 2: blobs_volume}
TYPE_DIMS = {0: (64, 64, 64), 1: (128, 128, 64), 2: (256, 256, 160)}


def spheres_64(seed: int = 0) -> Workload:
    """64^3 uint8, 3 spheres, 32 bins, spacing 8, scales 3..8, quadrant, 50 iterations."""
    return Workload("spheres64_u8_quadrant", spheres_volume(seed), *TYPE_PARAMS[0])


def pet_shell(method: int, seed: int = 1) -> Workload:
    """PET-like 128x128x64 uint16 shell, 64 bins, spacing 6, scales 4..16, 50 iterations."""
    name = "pet128x128x64_u16_" + ("quadrant" if method == QUADRANT else "meanshift")
    return Workload(name, shell_volume(seed), 64, 6, (4, 16), method, 50)


def mr_blobs(seed: int = 2) -> Workload:
    """MR-like 256x256x160 int16, 64 bins, spacing 8, scales 4..24, mean-shift, 100 iterations."""
    return Workload("mr256x256x160_i16_meanshift", blobs_volume(seed), *TYPE_PARAMS[2])


def typed_workload(kind: int, seed: int, dims, method_parity: int = 0) -> Workload:
    """A volume of generator type `kind` at `dims` with that type's parameters.  For
    type 1 (which runs both methods) odd `method_parity` selects mean-shift."""
    bins, sp, scales, method, max_iter = TYPE_PARAMS[kind]
    if kind == 1 and method_parity % 2 == 1:
        method = MEANSHIFT
    vol = TYPE_GEN[kind](seed, tuple(int(d) for d in dims))
    return Workload(f"type{kind}_{dims[0]}x{dims[1]}x{dims[2]}_s{seed}", vol, bins, sp, scales, method, max_iter)


def batch_specs(seed: int = 3, n: int = 64):
    """Uneven batch: per volume (kind, dims, volume seed, method parity).  Each dim is
    uniform: x,y in 64..192, z in 64..128; the type mix is 50/30/20."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        X = int(rng.integers(64, 193))
        Y = int(rng.integers(64, 193))
        Z = int(rng.integers(64, 129))
        kind = int(rng.choice(3, p=[0.5, 0.3, 0.2]))
        out.append((kind, (X, Y, Z), 1000 + i, i))
    return out


def batch_workloads(seed: int = 3, n: int = 64, only=None) -> List[Workload]:
    specs = batch_specs(seed, n)
    idx = range(n) if only is None else only
    return [typed_workload(specs[i][0], specs[i][2], specs[i][1], specs[i][3]) for i in idx]


def arrival_trace(rate: float, seed: int = 4, n: int = 256):
    """Poisson arrivals: (arrival time in s, kind, volume seed, method parity) for n
    requests at `rate` requests/s with the 50/30/20 type mix at native sizes."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n)
    kinds = rng.choice(3, size=n, p=[0.5, 0.3, 0.2])
    t = np.cumsum(gaps) - gaps[0]
    return [(float(t[i]), int(kinds[i]), 2000 + i, i) for i in range(n)]
