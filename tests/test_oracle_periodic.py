"""Pins of the oracle's periodic boundaries (Sec. 3.1, boundary conditions:
states repeat across the faces of a periodic box along x and/or y).

A periodic system is the same as an infinite one made of copies of the box,
so the oracle on a periodic box must agree with the oracle on the open
system of 3 x 3 (or 3 x 1) explicit copies, for the particles of the
central copy: same candidate counts, stencil sizes and ghost masks, and
the same derivatives, pressure, viscosity and right-hand side (rounding
included: an image coordinate x + L is rounded once on either side).
A rigid shift of every particle along a periodic axis, wrapped into the
box, leaves every per-particle result unchanged up to rounding.
"""
import dataclasses

import numpy as np
import pytest

import lpgen
import oracle
from cases import CASES


def _tiled(wl):
    """Open system of explicit copies, the central one first (ids 0..n-1)."""
    p = wl.params[0]
    Lx, Ly = p.box_len
    sx = (0, -1, 1) if Lx > 0 else (0,)
    sy = (0, -1, 1) if Ly > 0 else (0,)
    parts = []
    for b in sy:
        for a in sx:
            st = wl.state.copy()
            st.x = st.x + a * Lx
            st.y = st.y + b * Ly
            parts.append(st)
    big = lpgen.State.concat(parts)
    q = dataclasses.replace(p, box_len=(0.0, 0.0))
    return big, np.array([0, big.n]), [q]


@pytest.mark.parametrize("case", ["periodic_xy", "periodic_x"])
@pytest.mark.parametrize("brute", [True, False])
def test_periodic_box_equals_explicit_copies(case, brute):
    wl = CASES[case]()
    n = wl.n
    o = oracle.Oracle(wl.state, wl.offsets, wl.params, brute=brute)
    big, off, prm = _tiled(wl)
    ob = oracle.Oracle(big, off, prm, brute=True)
    nb, nbb = o.neighbours(), ob.neighbours()
    cnt = np.diff(nb.cand_off)
    cntb = np.diff(nbb.cand_off)[:n]
    assert np.array_equal(cnt, cntb)
    assert np.array_equal(nb.sten_cnt, nbb.sten_cnt[:n])
    assert np.array_equal(nb.ghost_mask, nbb.ghost_mask[:n])
    # some stencils reach through a periodic face
    assert np.any(nbb.sten_idx[:n][np.arange(nbb.sten_idx.shape[1])[None, :] <
                                   nbb.sten_cnt[:n, None]] >= n)
    r, rb = o.evaluate(), ob.evaluate()
    for key in ("coef_u", "diag", "grad", "acc", "dVdt"):
        a, b = r[key], rb[key][..., :n]
        scale = max(np.max(np.abs(b)), 1e-300)
        assert np.max(np.abs(a - b)) <= 1e-13 * scale, key
    assert np.array_equal(r["flags"], rb["flags"][:n])


def test_periodic_shift_invariance():
    """Shift every particle by 0.37 h along x and 0.61 h along y, wrapped
    into the box: the right-hand side of every particle is unchanged."""
    wl = CASES["periodic_xy"]()
    p = wl.params[0]
    h = p.h
    st = wl.state.copy()
    st.x = st.x + 0.37 * h
    st.y = st.y + 0.61 * h
    oracle.wrap(st, wl.offsets, wl.params)
    assert np.all((st.x >= 0) & (st.x < p.box_len[0]))
    r0 = oracle.Oracle(wl.state, wl.offsets, wl.params).evaluate()
    r1 = oracle.Oracle(st, wl.offsets, wl.params).evaluate()
    for key in ("acc", "dVdt", "diag"):
        scale = np.max(np.abs(r0[key]))
        assert np.max(np.abs(r0[key] - r1[key])) <= 1e-9 * scale, key
    assert np.array_equal(r0["flags"], r1["flags"])


def test_periodic_sort_uses_the_box():
    """Morton cells of a periodic axis start at the box and wrap: the order
    of a state and of the same state shifted by one period agree."""
    wl = CASES["periodic_xy"]()
    p = wl.params[0]
    perm0, keys0 = oracle.sort_perm(wl.state, wl.offsets, wl.params)
    st = wl.state.copy()
    st.x = st.x + p.box_len[0]       # one period out: wrapped for the cells
    perm1, keys1 = oracle.sort_perm(st, wl.offsets, wl.params)
    assert np.array_equal(perm0, perm1) and np.array_equal(keys0, keys1)


def test_step_wraps_positions_into_the_box():
    wl = CASES["periodic_xy"]()
    p = wl.params[0]
    st = wl.state.copy()
    st.u = st.u + 50.0                 # 50 m/s: crosses the face in one step
    out, _, _ = oracle.step(st, wl.offsets, wl.params, 2e-3)
    assert np.all((out.x >= 0) & (out.x < p.box_len[0]))
    out2, _, _ = oracle.step2(st, wl.offsets, wl.params, 2e-3)
    assert np.all((out2.x >= 0) & (out2.x < p.box_len[0]))
