"""Independent numpy/scipy restatements used to pin the oracle.

Nothing here imports the oracle or the GPU library.  Histograms come from
np.bincount over array slices, entropies from scipy.stats.entropy, and the
mean-shift step from the per-voxel weights of Eq. 5 and the weighted mean of
Eq. 6 taken literally, voxel by voxel.
"""
from __future__ import annotations

import numpy as np
from scipy.stats import entropy as scipy_entropy


def clipped(bv: np.ndarray, lo, hi):
    """bv[z0:z1+1, y0:y1+1, x0:x1+1] for the box [lo, hi] (x,y,z) clipped to the volume,
    plus the clipped lower corner."""
    Z, Y, X = bv.shape
    l = [max(0, lo[0]), max(0, lo[1]), max(0, lo[2])]
    h = [min(X - 1, hi[0]), min(Y - 1, hi[1]), min(Z - 1, hi[2])]
    return bv[l[2]:h[2] + 1, l[1]:h[1] + 1, l[0]:h[0] + 1], l


def cube_counts(bv, bins, p, s):
    """Counts of bins 0..bins-1; values >= bins (outside a window level) are dropped."""
    sub, _ = clipped(bv, [p[0] - s, p[1] - s, p[2] - s], [p[0] + s, p[1] + s, p[2] + s])
    return np.bincount(sub.ravel(), minlength=bins + 1)[:bins]


def octant_counts(bv, bins, p, j, k):
    lo, hi = [], []
    for a in range(3):
        if (j >> a) & 1:
            lo.append(p[a]); hi.append(p[a] + k)
        else:
            lo.append(p[a] - k); hi.append(p[a])
    sub, _ = clipped(bv, lo, hi)
    return np.bincount(sub.ravel(), minlength=bins + 1)[:bins]


def H(counts) -> float:
    c = np.asarray(counts, dtype=np.float64)
    if c.sum() == 0:
        return 0.0
    return float(scipy_entropy(c))  # natural log, normalises the counts itself


def W(c_s, c_prev, s) -> float:
    if np.sum(c_s) == 0 or np.sum(c_prev) == 0:
        return 0.0
    p = np.asarray(c_s, np.float64) / np.sum(c_s)
    q = np.asarray(c_prev, np.float64) / np.sum(c_prev)
    return float(s * s / (2 * s - 1) * np.abs(p - q).sum())


def meanshift_step_literal(bv, bins, p, s):
    """Eq. 5 weights w(v) = sqrt(q_b / p_b) with q uniform (1/B), then Eq. 6 with a
    flat kernel: x_new = sum_v w(v) v / sum_v w(v), voxel by voxel.  Returns
    (x_new - P, Bhattacharyya coefficient sum_b sqrt(p_b q_b))."""
    sub, l = clipped(bv, [p[0] - s, p[1] - s, p[2] - s], [p[0] + s, p[1] + s, p[2] + s])
    zz, yy, xx = np.meshgrid(np.arange(sub.shape[0]) + l[2], np.arange(sub.shape[1]) + l[1],
                             np.arange(sub.shape[2]) + l[0], indexing="ij")
    b = sub.ravel()
    keep = b < bins  # voxels outside a window level do not take part
    b = b[keep]
    pb = np.bincount(b, minlength=bins) / b.size
    q = 1.0 / bins
    w = np.sqrt(q / pb[b])
    pos = np.stack([xx.ravel()[keep], yy.ravel()[keep], zz.ravel()[keep]], axis=1).astype(np.float64)
    x_new = (w[:, None] * pos).sum(axis=0) / w.sum()
    rho = float(np.sqrt(pb * q).sum())
    return x_new - np.asarray(p, np.float64), rho


def dense_kb(bv, bins, s_min, s_max):
    """Every-voxel Kadir-Brady search: for each voxel, entropies of the centred cubes
    s in [s_min-1, s_max+1], peaks over s in [s_min, s_max], best peak by H*W.
    Returns dict (x,y,z) -> (s*, H, W, Y, near_tie) for voxels with a peak."""
    Z, Y, X = bv.shape
    out = {}
    for z in range(Z):
        for y in range(Y):
            for x in range(X):
                p = (x, y, z)
                cs = {s: cube_counts(bv, bins, p, s) for s in range(s_min - 1, s_max + 2)}
                hs = {s: H(c) for s, c in cs.items()}
                best = None
                tie = False
                for s in range(s_min, s_max + 1):
                    d1, d2 = hs[s] - hs[s - 1], hs[s] - hs[s + 1]
                    if min(abs(d1), abs(d2)) < 1e-9:
                        tie = True
                    if d1 > 0 and d2 > 0:
                        w = W(cs[s], cs[s - 1], s)
                        yv = hs[s] * w
                        if best is None or yv > best[3]:
                            if best is not None and abs(yv - best[3]) < 1e-9:
                                tie = True
                            best = (s, hs[s], w, yv)
                if best is not None:
                    out[p] = best + (tie,)
    return out
