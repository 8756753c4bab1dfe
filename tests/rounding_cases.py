"""Particle pairs that sit on the cut radius to the last bit.

For such a pair the plain float64 definition r2 = (dx*dx + dy*dy) + dz*dz
(every product and sum rounded) and an evaluation with fused multiply-add
classify the pair differently (r2 < R^2 or not).  The search is exact:
fused results are computed with rational arithmetic and rounded once.
"""
from fractions import Fraction

import numpy as np


def unfused_r2(dx, dy, dz):
    dx, dy, dz = np.float64(dx), np.float64(dy), np.float64(dz)
    s = dx * dx + dy * dy
    return s + dz * dz


def fused_r2(dx, dy, dz):
    """fma(dz, dz, fma(dy, dy, dx*dx)): each fma rounds once."""
    xx = np.float64(dx) * np.float64(dx)
    t = float(Fraction(float(dy)) * Fraction(float(dy)) + Fraction(float(xx)))
    return float(Fraction(float(dz)) * Fraction(float(dz)) + Fraction(t))


def find_straddle(xi, R, seed=0, tries=200000):
    """Returns (xj, dx, dy, dz) with xj - xi = (dx, dy, dz) in float64 such
    that the unfused r2 is below R^2 while the fused one is not, or the
    reverse."""
    R2 = np.float64(R) * np.float64(R)
    rng = np.random.default_rng(seed)
    xi = np.asarray(xi, dtype=np.float64)
    for _ in range(tries):
        d = rng.normal(size=3)
        d = d / np.linalg.norm(d) * R
        xj = xi + d
        # walk z by ulps across the sphere
        for k in range(-40, 41):
            xj2 = np.array([xj[0], xj[1], xj[2] + k * np.spacing(xj[2])])
            dd = xj2 - xi
            a = unfused_r2(*dd) < R2
            b = fused_r2(*dd) < R2
            if a != b:
                return xj2, dd, bool(a)
    return None


def straddle_workload(n_pairs=8, h=1.0 / 16.0):
    """Systems of two particles each, one straddling pair per system (both
    kinds: inside only without fusion, inside only with fusion)."""
    import lpgen
    p = lpgen.default_params(h)
    p.wall_z = -100.0
    states, offs, want = [], [0], []
    seed = 0
    kinds = {True: 0, False: 0}
    while len(want) < n_pairs:
        seed += 1
        xi = np.array([0.3 + 0.01 * seed, 0.4, 0.5])
        r = find_straddle(xi, p.R, seed=seed, tries=4000)
        if r is None:
            continue
        xj, dd, inside = r
        if kinds[inside] >= n_pairs // 2:
            continue
        kinds[inside] += 1
        pts = np.stack([xi, xj])
        z = np.zeros(2)
        states.append(lpgen.State(pts[:, 0].copy(), pts[:, 1].copy(),
                                  pts[:, 2].copy(), z.copy(), z.copy(), z.copy(),
                                  np.full(2, 1.0 / 0.45)))
        offs.append(offs[-1] + 2)
        want.append(inside)
    wl = lpgen.Workload("straddle", lpgen.State.concat(states),
                        np.array(offs), [p] * n_pairs, 1e-4, 1)
    return wl, want
