"""Pins of the FP64 adjoint oracle (oracle/adjoint.py) against the C oracle.

- The torch re-expression of the step reproduces the C oracle step.
- Its reverse agrees with central differences of the C oracle step (an
  independent implementation, re-sorting and re-selecting stencils at every
  evaluation) in seeded random directions, for the state and for the mu(I)
  parameters (mu_s, mu_2, I0).
- Over several steps with a runout loss, the composed adjoint agrees with
  central differences of the loss.
"""
import dataclasses

import numpy as np
import pytest

import lpgen
import oracle
from cases import CASES
from oracle import adjoint


def _state_dir(wl, seed):
    """Seeded direction with the scales of each field."""
    rng = np.random.default_rng(seed)
    n, h = wl.n, wl.params[0].h
    return [h * rng.standard_normal(n) for _ in range(3)] + \
           [0.1 * rng.standard_normal(n) for _ in range(3)] + \
           [0.01 * wl.state.V * rng.standard_normal(n)]


def _shift(st, v, eps):
    return lpgen.State(*[a + eps * d for a, d in zip(st.arrays(), v)])


def _dot(a, b):
    return sum(float(np.dot(x, y)) for x, y in zip(a, b))


def _with_params(params, q, delta):
    out = []
    for p in params:
        kw = {"mu_s": p.mu_s, "mu_2": p.mu_2, "I0": p.I0}
        key = ("mu_s", "mu_2", "I0")[q]
        kw[key] = kw[key] + delta
        out.append(dataclasses.replace(p, **kw))
    return out


@pytest.mark.parametrize("case", ["column16_flow_ragged", "sheared_20x20x12",
                                  "ensemble_3", "lattice_exact", "periodic_xy",
                                  "periodic_x"])
def test_frozen_forward_reproduces_oracle_step(case):
    wl = CASES[case]()
    ost, perm, _ = oracle.step(wl.state, wl.offsets, wl.params, wl.dt)
    st = wl.state.take(perm)
    fs = adjoint.FrozenStep(st, wl.offsets, wl.params, wl.dt)
    got = fs.run(st, adjoint.theta_of(wl.params))
    for a, b, c in zip(got.arrays(), ost.arrays(), st.arrays()):
        inc = np.max(np.abs(b - c))
        assert np.max(np.abs(a - b)) <= 1e-11 * inc + 4 * np.spacing(np.max(np.abs(b)))


def _structure(st, wl):
    """Everything the step holds fixed: order, stencils, ghosts, mirrors,
    fallback flags."""
    perm, _ = oracle.sort_perm(st, wl.offsets, wl.params)
    o = oracle.Oracle(st.take(perm), wl.offsets, wl.params)
    nb = o.neighbours()
    return (perm, nb.sten_cnt, nb.sten_idx, nb.ghost_mask, nb.mirror_src,
            o.evaluate()["flags"])


def _fd_step(wl, lam, v):
    """Central difference of <lam, step(s)> along v with the largest eps
    (1e-6 down to 1e-9) at which the step's discrete structure is the same
    at s + eps v and s - eps v as at s."""
    ref = _structure(wl.state, wl)
    for eps in (1e-6, 1e-7, 1e-8, 1e-9):
        sp, sm = _shift(wl.state, v, eps), _shift(wl.state, v, -eps)
        if all(all(np.array_equal(a, b) for a, b in zip(ref, _structure(s, wl)))
               for s in (sp, sm)):
            fp, _, _ = oracle.step(sp, wl.offsets, wl.params, wl.dt)
            fm, _, _ = oracle.step(sm, wl.offsets, wl.params, wl.dt)
            return eps, _dot(lam, [(a - b) / (2 * eps)
                                   for a, b in zip(fp.arrays(), fm.arrays())])
    raise AssertionError("stencils change at every eps")


@pytest.mark.parametrize("case", ["column16_flow_ragged", "sheared_20x20x12",
                                  "periodic_xy"])
@pytest.mark.parametrize("part", ["positions", "velocities", "volumes"])
def test_state_adjoint_matches_central_differences(case, part):
    wl = CASES[case]()
    lam = _state_dir(wl, 11)                       # dL/d(new state)
    v = _state_dir(wl, 12)                         # direction in the state
    sel = {"positions": (0, 1, 2), "velocities": (3, 4, 5), "volumes": (6,)}[part]
    v = [d if k in sel else np.zeros(wl.n) for k, d in enumerate(v)]
    # particles clamped onto z = h/4 by the shear sit exactly on structural
    # boundaries (octant sign dz = 0 with each other, |dz| = h/2 to their
    # own mirrors): they are held in place
    free = wl.state.z != 0.25 * wl.params[0].h
    v = [d * free if k < 3 else d for k, d in enumerate(v)]
    g, _, _ = adjoint.step_vjp(wl.state, wl.offsets, wl.params, wl.dt, lam)
    eps, fd = _fd_step(wl, lam, v)
    ad = _dot(g, v)
    tol = 1e-6 if eps >= 1e-7 else 1e-4
    assert abs(fd - ad) <= tol * abs(fd), (eps, fd, ad)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_parameter_adjoint_matches_central_differences(q):
    """d/d(mu_s, mu_2, I0) on a flow that visits the inertial branch (where
    mu(I) acts).  The parameters enter the step only through the
    acceleration a (u' = u + dt a, x' = x + dt u + dt^2 a / 2), so the
    differences are taken on the C oracle's a.  The sensitivity is small
    against a ~ g, so a 1e-6 step is swamped by rounding; the branch
    choice does not depend on the parameters, so a Richardson-extrapolated
    central difference with steps 2e-3 and 1e-3 is used instead."""
    wl = CASES["column16_flow_ragged"]()
    lam = _state_dir(wl, 21)
    _, gth, perm = adjoint.step_vjp(wl.state, wl.offsets, wl.params, wl.dt, lam)
    st = wl.state.take(perm)
    dt = wl.dt

    def dlam(eps):
        def acc(params):
            return oracle.Oracle(st, wl.offsets, params).evaluate()["acc"]
        da = (acc(_with_params(wl.params, q, eps)) -
              acc(_with_params(wl.params, q, -eps))) / (2 * eps)
        return sum(float(np.dot(dt * lam[3 + a] + 0.5 * dt * dt * lam[a], da[a]))
                   for a in range(3))

    fd = (4.0 * dlam(1e-3) - dlam(2e-3)) / 3.0
    assert abs(gth[0, q]) > 0
    assert abs(fd - gth[0, q]) <= 1e-5 * abs(fd), (fd, gth[0, q])


def test_trajectory_loss_gradient_matches_central_differences():
    """Three steps and the runout loss L = sum softplus((x - x*)/h): the
    composed adjoint (reverse over the steps, un-permuting at each) against
    central differences of L in the initial velocity field and mu_s."""
    wl = CASES["column16_flow_ragged"]()
    h = wl.params[0].h
    xs = 0.6
    steps = 3

    def loss(st):
        t = (st.x - xs) / h
        return float(np.sum(np.logaddexp(0.0, t)))

    def run(st0, params):
        st = st0
        states = []
        for _ in range(steps):
            states.append(st)
            st, _, _ = oracle.step(st, wl.offsets, params, wl.dt)
        return st, states

    stN, states = run(wl.state, wl.params)
    t = (stN.x - xs) / h
    lam = [1.0 / (1.0 + np.exp(-t)) / h] + [np.zeros(wl.n) for _ in range(6)]
    gth = np.zeros((1, 3))
    for st in reversed(states):
        lam, g, _ = adjoint.step_vjp(st, wl.offsets, wl.params, wl.dt, lam)
        gth += g
    v = _state_dir(wl, 31)
    dv = [np.zeros(wl.n)] * 3 + v[3:6] + [np.zeros(wl.n)]
    eps = 1e-6
    xp = run(_shift(wl.state, dv, eps), wl.params)[0].x
    xm = run(_shift(wl.state, dv, -eps), wl.params)[0].x
    # per-particle differences of the loss terms (no cancellation of the
    # large sum); what remains is the rounding of x, ~1e-5 of the result
    fd = float(np.sum(np.logaddexp(0.0, (xp - xs) / h) -
                      np.logaddexp(0.0, (xm - xs) / h))) / (2 * eps)
    ad = _dot(lam, dv)
    assert abs(fd - ad) <= 1e-4 * abs(fd), (fd, ad)

    # mu_s moves x by ~dt^2 a_mu per step, a few hundred ulps of x for a
    # small step in mu_s: the difference needs a large step, which the
    # smoothness in mu_s allows (Richardson over 0.02 and 0.01)
    def dmu(e):
        xp = run(wl.state, _with_params(wl.params, 0, e))[0].x
        xm = run(wl.state, _with_params(wl.params, 0, -e))[0].x
        return float(np.sum(np.logaddexp(0.0, (xp - xs) / h) -
                            np.logaddexp(0.0, (xm - xs) / h))) / (2 * e)

    fd = (4.0 * dmu(1e-2) - dmu(2e-2)) / 3.0
    assert abs(fd - gth[0, 0]) <= 1e-3 * abs(fd), (fd, gth[0, 0])
