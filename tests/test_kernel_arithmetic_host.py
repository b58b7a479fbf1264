"""Host checks of two arithmetic shortcuts the HIP kernels take (no GPU, no
oracle: each check compares the shortcut with the plain operation it replaces).

* The sweep engine divides small integers with the hardware float reciprocal:
  floor((a + 1/2) * rcp(d)) for 0 <= a <= 1024, 1 <= d <= 1024.  (a + 1/2) / d
  lies at least 1/(2d) from an integer, so the quotient survives a reciprocal
  off by one ulp (the instruction's stated accuracy) and the rounding of the
  product.
* ABMSOD takes the Gaussian profile exp(-d/2) of its windows (Sec. 2.3, the
  kernel profile of Eq. 5 and Alg. 2) along a row by a two-term recurrence:
  d is a quadratic in the voxel's x, so g(x+1) = g(x) r(x) with
  r(x) = exp(-(d(x+1) - d(x))/2) and r(x+1) = r(x) exp(-H^-1_xx).  The pair is
  taken exactly at the row's first voxel inside the window and every 32 voxels
  after; the error must stay far below the sweep's 2^-40 fixed point.  The
  bandwidths are those the search can reach: start windows and the growth cap
  keep every half-extent sqrt(5 H_aa) within r_max + 1/2 <= 32.5 voxels.
"""
import math

import numpy as np


def test_small_division_by_float_reciprocal_is_exact():
    a = np.arange(0, 1025, dtype=np.float32)[:, None]
    d = np.arange(1, 1025, dtype=np.float32)[None, :]
    want = np.arange(0, 1025)[:, None] // np.arange(1, 1025)[None, :]
    rcp = np.float32(1.0) / d
    for r in (rcp, np.nextafter(rcp, np.float32(0.0)), np.nextafter(rcp, np.float32(np.inf))):
        prod = (a + np.float32(0.5)) * r          # float32 add (exact here), then a rounded float32 product
        assert prod.dtype == np.float32
        got = np.trunc(prod).astype(np.int64)     # the conversion to int truncates
        bad = np.argwhere(got != want)
        assert bad.size == 0, f"floor((a+1/2) rcp(d)) != a // d at (a, d) = {bad[:5].tolist()}"


def _quad_form(inv, u0, u1, u2):
    return (inv[0] * u0 * u0 + inv[1] * u1 * u1 + inv[2] * u2 * u2 +
            2.0 * (inv[3] * u0 * u1 + inv[4] * u0 * u2 + inv[5] * u1 * u2))


def _row_step_exponent(inv, u0, u1, u2):
    return -(inv[0] * (2.0 * u0 + 1.0) + 2.0 * (inv[3] * u1 + inv[4] * u2)) / 2.0


def test_row_weight_recurrence_stays_within_fixed_point():
    anchor = 32
    cap = 32.5 ** 2 / 5.0    # the largest diagonal entry of a bandwidth (voxel^2)
    rng = np.random.default_rng(20)
    worst, rows_in_window, long_rows = 0.0, 0, 0
    for _ in range(3000):
        # a positive definite bandwidth, from thin to the cap, in any orientation
        A = rng.normal(size=(3, 3))
        H = A @ A.T + np.eye(3) * rng.uniform(0.01, 0.5)
        H *= rng.uniform(0.05, cap) / np.max(np.diag(H))
        Hi = np.linalg.inv(H)
        inv = [Hi[0, 0], Hi[1, 1], Hi[2, 2], Hi[0, 1], Hi[0, 2], Hi[1, 2]]
        x = rng.uniform(20.0, 80.0, 3)
        c = rng.normal(size=3) * np.sqrt(np.diag(H))
        vy, vz = int(round(x[1] + c[1])), int(round(x[2] + c[2]))
        u1, u2 = vy - x[1], vz - x[2]
        q = math.exp(-inv[0])
        xs = range(int(x[0]) - 40, int(x[0]) + 41)
        inside = [vx for vx in xs if _quad_form(inv, vx - x[0], u1, u2) <= 5.0]
        if not inside:
            continue
        rows_in_window += 1
        long_rows += len(inside) > anchor
        at = inside[0]           # the kernel's precomputed anchor
        ga = math.exp(-_quad_form(inv, at - x[0], u1, u2) / 2.0)
        ra = math.exp(_row_step_exponent(inv, at - x[0], u1, u2))
        g = r = 0.0
        left = 0
        for vx in xs:
            u0 = vx - x[0]
            d = _quad_form(inv, u0, u1, u2)
            inw = d <= 5.0
            if inw and left <= 0:
                if vx == at:
                    g, r = ga, ra
                else:
                    g, r = math.exp(-d / 2.0), math.exp(_row_step_exponent(inv, u0, u1, u2))
                left = anchor
            if inw:
                exact = math.exp(-d / 2.0)
                worst = max(worst, abs(g - exact) / exact)
            if left > 0:
                g *= r
                r *= q
                left -= 1
    assert rows_in_window > 2000 and long_rows > 100, (rows_in_window, long_rows)   # re-anchored rows too
    # g <= 1 is summed as round(g 2^40): a quantum of 9.1e-13
    assert worst < 1e-13, worst
