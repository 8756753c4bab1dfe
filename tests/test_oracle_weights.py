"""Pins of the oracle's weighted least-squares fit (Sec. 3.1 step 7 states
the fit as a weighted least-squares problem; the option LP_W_GAUSS takes
w = exp(-4 r^2 / R^2) per stencil row, r the distance to the fitted
particle, and w = exp(-12 h^2 / R^2) for a ghost row at offset h s).

- Exact data: any positive weights reproduce a quadratic exactly, so a
  weighted fit that scales the rows and right-hand sides inconsistently
  fails it.
- Arbitrary data: the fit equals LAPACK's SVD least-squares solver
  (numpy.linalg.lstsq) on the exported stencil's Taylor rows scaled by
  sqrt(w), weights computed here from the positions, so a wrong weight
  function, a wrong ghost distance, w instead of sqrt(w) on the rows, or a
  weight left off the right-hand side fails it.
- The weighted and the unit fits differ on such data (the option acts).
"""
import numpy as np
import pytest

import lpgen
import oracle
from lpgen import State

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

GAUSS = dict(weight=1)


def _state_from_points(pts):
    n = pts.shape[0]
    z = np.zeros(n)
    return State(pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2].copy(),
                 z.copy(), z.copy(), z.copy(), np.full(n, 1.0 / 0.45))


def _one(state, p, cfg=None):
    return oracle.Oracle(state, np.array([0, state.n]), [p], cfg)


def _quad_fields(rng, pts, nf=3):
    F, D = [], []
    for _ in range(nf):
        c0 = rng.normal()
        g = rng.normal(size=3)
        Hs = rng.normal(size=(3, 3))
        Hs = Hs + Hs.T
        F.append(c0 + pts @ g + 0.5 * np.einsum("ni,ij,nj->n", pts, Hs, pts))
        D.append((g[None, :] + pts @ Hs, Hs))
    return np.array(F), D


@pytest.mark.parametrize("layout", ["lattice", "random"])
def test_weighted_fit_reproduces_quadratics(layout):
    rng = np.random.default_rng({"lattice": 21, "random": 22}[layout])
    h = 0.05
    p = lpgen.default_params(h)
    p.wall_z = -100.0
    if layout == "random":
        pts = rng.uniform(0, 12 * h, size=(1728, 3))
    else:
        st0 = lpgen.lattice_column(12, 12, 12, h, seed=98, params=p)
        pts = np.stack([st0.x, st0.y, st0.z], 1)
    pts = pts + np.array([0.3, -0.2, 0.1])
    o = _one(_state_from_points(pts), p, GAUSS)
    nb = o.neighbours()
    F, D = _quad_fields(rng, pts)
    coef, flags = o.fit(F, [1] * 3, [0] * 3)
    ok = (nb.ghost_mask == 0) & (flags == 0)
    assert ok.sum() > 50
    for f, (grad, Hs) in enumerate(D):
        scale = np.max(np.abs(grad)) + np.max(np.abs(Hs))
        for a in range(3):
            assert np.max(np.abs(coef[f, a, ok] - grad[ok, a])) <= 1e-11 * scale
        for c, (a, b) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
            assert np.max(np.abs(coef[f, 3 + c, ok] - Hs[a, b])) <= 1e-10 * scale


def _taylor(e):
    return np.array([e[0], e[1], e[2], e[0] ** 2 / 2, e[1] ** 2 / 2, e[2] ** 2 / 2,
                     e[0] * e[1], e[0] * e[2], e[1] * e[2]])


@pytest.mark.parametrize("case", ["column", "cloud"])
def test_weighted_fit_matches_lapack_on_scaled_rows(case):
    if case == "column":
        wl = lpgen.column_small()
        st, p = wl.state, wl.params[0]
        step = 53
    else:
        h = 1.0 / 16.0
        p = lpgen.default_params(h)
        rng = np.random.default_rng(31)
        n = 900
        pts = rng.uniform(0, 0.9, size=(n, 3)) + np.array([0.0, 0.0, 0.001])
        st = _state_from_points(pts)
        step = 7
    rng = np.random.default_rng(9)
    f = rng.normal(size=st.n)
    ghost_value = 0.37
    o = _one(st, p, GAUSS)
    nb = o.neighbours()
    # ghost value f_i + ghost_value * 0 through ghost_zero = 0: ghosts carry f_i
    coef, flags = o.fit(np.stack([f, f + ghost_value]), [1, -1], [0, 1])
    ou = _one(st, p)
    cu, _ = ou.fit(f[None, :], [1], [0])
    pts = np.concatenate([np.stack([st.x, st.y, st.z], 1), nb.mirror_state[:3].T], 0)
    fa = np.concatenate([f, f[nb.mirror_src]])
    fb = np.concatenate([f + ghost_value, -(f + ghost_value)[nb.mirror_src]])
    R2 = p.R * p.R
    checked = ghosts = over = 0
    for i in range(0, st.n, step):
        if flags[i] & oracle.FLAG_LINEAR:
            continue
        ids = nb.sten_idx[i, :nb.sten_cnt[i]]
        d = pts[ids] - pts[i]
        w = np.exp(-4.0 * np.sum(d * d, 1) / R2)
        rows = [_taylor(e) for e in d / p.h]
        ba = list(fa[ids] - f[i])
        bb = list(fb[ids] - (f[i] + ghost_value))
        ws = list(w)
        for q in range(8):
            if nb.ghost_mask[i] >> q & 1:
                s = np.array([1.0 if q & 1 else -1.0, 1.0 if q & 2 else -1.0,
                              1.0 if q & 4 else -1.0])
                rows.append(_taylor(s))
                ba.append(0.0)                       # ghost carries f_i
                bb.append(0.0 - (f[i] + ghost_value))  # ghost value zero
                ws.append(np.exp(-12.0 * p.h * p.h / R2))
                ghosts += 1
        sw = np.sqrt(np.array(ws))
        A = np.array(rows) * sw[:, None]
        for fld, b in ((0, ba), (1, bb)):
            c = np.linalg.lstsq(A, np.array(b) * sw, rcond=None)[0]
            c[:3] /= p.h
            c[3:] /= p.h ** 2
            assert np.max(np.abs(coef[fld, :, i] - c)) <= 1e-10 * np.max(np.abs(c)), (i, fld)
        # the weights change the answer on non-polynomial data where the
        # unit fit leaves a residual (a 9-row fit interpolates, and ghost
        # rows of equal weight can be fitted exactly, whatever the weights)
        A0 = np.array(rows)
        c0 = np.linalg.lstsq(A0, np.array(ba), rcond=None)[0]
        if np.linalg.norm(A0 @ c0 - np.array(ba)) > 1e-6 * np.linalg.norm(ba):
            assert np.max(np.abs(coef[0, :, i] - cu[0, :, i])) > 1e-6 * np.max(np.abs(cu[0, :, i]))
            over += 1
        checked += 1
    assert over > 20
    assert checked > 40
    if case == "cloud":
        assert ghosts > 20
