"""Pins of the adjoint of the oracle's second-order step
(oracle.adjoint.FrozenStep2 / step2_vjp) against the C oracle's step2:

- the torch re-expression of Heun's step reproduces oracle.step2;
- its reverse agrees with central differences of oracle.step2 (which
  re-sorts and re-selects the stencils of s and of the predictor at every
  evaluation) in seeded random directions of the state, at steps where
  neither set of stencils changes;
- the parameter cotangents agree with Richardson-extrapolated central
  differences in (mu_s, mu_2, I0).
"""
import numpy as np
import pytest

import lpgen
import oracle
from cases import CASES
from oracle import adjoint
from test_oracle_adjoint import _dot, _shift, _state_dir, _with_params


@pytest.mark.parametrize("case", ["column16_flow_ragged", "sheared_20x20x12",
                                  "ensemble_3", "lattice_exact", "periodic_xy",
                                  "periodic_x"])
def test_frozen_forward_reproduces_oracle_step2(case):
    wl = CASES[case]()
    ost, perm, _ = oracle.step2(wl.state, wl.offsets, wl.params, wl.dt)
    st = wl.state.take(perm)
    fs = adjoint.FrozenStep2(st, wl.offsets, wl.params, wl.dt)
    got = fs.run(st, adjoint.theta_of(wl.params))
    for a, b, c in zip(got.arrays(), ost.arrays(), st.arrays()):
        inc = np.max(np.abs(b - c))
        assert np.max(np.abs(a - b)) <= 1e-11 * inc + 4 * np.spacing(np.max(np.abs(b)))


def _structure2(st, wl):
    """What the second-order step holds fixed: the order, and the stencils,
    ghosts, mirrors and flags at s and at the predictor s*."""
    perm, _ = oracle.sort_perm(st, wl.offsets, wl.params)
    s = st.take(perm)
    s = lpgen.State(*[np.ascontiguousarray(a) for a in s.arrays()])
    out = [perm]
    o = oracle.Oracle(s, wl.offsets, wl.params)
    for stage in range(2):
        nb = o.neighbours()
        ev = o.evaluate()
        out += [nb.sten_cnt, nb.sten_idx, nb.ghost_mask, nb.mirror_src, ev["flags"]]
        if stage == 0:
            dt, a = wl.dt, ev["acc"]
            pred = lpgen.State(s.x + dt * s.u, s.y + dt * s.v, s.z + dt * s.w,
                               s.u + dt * a[0], s.v + dt * a[1], s.w + dt * a[2],
                               s.V + dt * ev["dVdt"])
            o = oracle.Oracle(pred, wl.offsets, wl.params)
    return out


def _fd_step2(wl, lam, v):
    ref = _structure2(wl.state, wl)
    for eps in (1e-6, 1e-7, 1e-8, 1e-9):
        sp, sm = _shift(wl.state, v, eps), _shift(wl.state, v, -eps)
        if all(all(np.array_equal(a, b) for a, b in zip(ref, _structure2(s, wl)))
               for s in (sp, sm)):
            fp, _, _ = oracle.step2(sp, wl.offsets, wl.params, wl.dt)
            fm, _, _ = oracle.step2(sm, wl.offsets, wl.params, wl.dt)
            return eps, _dot(lam, [(a - b) / (2 * eps)
                                   for a, b in zip(fp.arrays(), fm.arrays())])
    raise AssertionError("stencils change at every eps")


@pytest.mark.parametrize("case", ["column16_flow_ragged", "sheared_20x20x12",
                                  "periodic_xy"])
@pytest.mark.parametrize("part", ["positions", "velocities", "volumes"])
def test_step2_state_adjoint_matches_central_differences(case, part):
    wl = CASES[case]()
    lam = _state_dir(wl, 51)
    v = _state_dir(wl, 52)
    sel = {"positions": (0, 1, 2), "velocities": (3, 4, 5), "volumes": (6,)}[part]
    v = [d if k in sel else np.zeros(wl.n) for k, d in enumerate(v)]
    # particles clamped onto z = h/4 by the shear sit on structural
    # boundaries (octant sign, ghost margin): held in place
    free = wl.state.z != 0.25 * wl.params[0].h
    v = [d * free if k < 3 else d for k, d in enumerate(v)]
    g, _, _ = adjoint.step2_vjp(wl.state, wl.offsets, wl.params, wl.dt, lam)
    eps, fd = _fd_step2(wl, lam, v)
    ad = _dot(g, v)
    tol = 1e-6 if eps >= 1e-7 else 1e-4
    assert abs(fd - ad) <= tol * abs(fd), (eps, fd, ad)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_step2_parameter_adjoint_matches_central_differences(q):
    """The parameters reach the output through acc(s) and acc(s*), which
    also moves s*: differences of the whole step, element by element
    (no cancellation of large sums), Richardson over 2e-3 and 1e-3."""
    wl = CASES["column16_flow_ragged"]()
    lam = _state_dir(wl, 61)
    _, gth, _ = adjoint.step2_vjp(wl.state, wl.offsets, wl.params, wl.dt, lam)

    def d(eps):
        fp, _, _ = oracle.step2(wl.state, wl.offsets, _with_params(wl.params, q, eps), wl.dt)
        fm, _, _ = oracle.step2(wl.state, wl.offsets, _with_params(wl.params, q, -eps),
                                wl.dt)
        return _dot(lam, [(a - b) / (2 * eps) for a, b in zip(fp.arrays(), fm.arrays())])

    fd = (4.0 * d(1e-3) - d(2e-3)) / 3.0
    assert abs(gth[0, q]) > 0
    assert abs(fd - gth[0, q]) <= 1e-5 * abs(fd), (fd, gth[0, q])
