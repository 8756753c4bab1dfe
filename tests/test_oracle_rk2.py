"""Pins of the oracle's second-order step (oracle.step2, Heun's method on
the right-hand side of Sec. 2.1) against properties of the time
integrator that do not depend on the step's own formula:

* order: one step of size h has a local error O(h^3) for Heun and O(h^2)
  for the explicit update of u and V in oracle.step (Sec. 3.1 step 8),
  measured against 16 Heun substeps of h / 16 on a flowing column;
* exactness: under a constant acceleration (isolated gas-regime particles:
  no pressure, no viscosity, only gravity) Heun's rule reproduces the
  parabola x + h u + h^2 g / 2, u + h g exactly.
"""
import numpy as np
import pytest

import lpgen
import oracle
from cases import CASES

pytestmark = pytest.mark.timeout(300)


def _sorted(wl):
    perm, _ = oracle.sort_perm(wl.state, wl.offsets, wl.params)
    st = wl.state.take(perm)
    return lpgen.State(*[np.ascontiguousarray(a) for a in st.arrays()])


def _steps(fn, wl, s, h, k):
    for _ in range(k):
        s, _, _ = fn(s, wl.offsets, wl.params, h, sort=False)
    return s


def _err(a, b, q):
    return [float(np.quantile(np.abs(x - y), q)) for x, y in zip(a.arrays(), b.arrays())]


def test_heun_local_error_is_third_order():
    """Halving h divides Heun's one-step error in u, w by about 8 and the
    first-order update's by about 4 (median and 90th percentile over
    particles, so that the few particles whose stencil or closure branch
    switches inside the step do not decide).  The percentile sees the
    predictor's volume: u depends on V through the pressure."""
    wl = CASES["column16_flow_ragged"]()
    s0 = _sorted(wl)
    errs = {}
    for h in (1e-4, 5e-5):
        ref = _steps(oracle.step2, wl, s0, h / 16, 16)
        e2, e1 = _steps(oracle.step2, wl, s0, h, 1), _steps(oracle.step, wl, s0, h, 1)
        errs[h] = [(_err(e2, ref, q), _err(e1, ref, q)) for q in (0.5, 0.9)]
    for qi in (0, 1):
        for k in (3, 5):   # u, w
            heun = np.log2(errs[1e-4][qi][0][k] / errs[5e-5][qi][0][k])
            euler = np.log2(errs[1e-4][qi][1][k] / errs[5e-5][qi][1][k])
            assert 2.6 < heun < 3.5, (qi, k, heun)
            assert 1.5 < euler < 2.5, (qi, k, euler)
    heun_v = np.log2(errs[1e-4][0][0][6] / errs[5e-5][0][0][6])
    assert heun_v > 2.6, heun_v


def test_free_fall_is_exact():
    """Particles 1 m apart and 1 m above the wall have no neighbour, no
    mirror and a gas-regime volume: acceleration g, dV/dt = 0; Heun's step
    is then exact for the position and velocity."""
    h = 1.0 / 16.0
    p = lpgen.default_params(h)
    g = np.array(p.g)
    ii, jj, kk = np.meshgrid(np.arange(3), np.arange(3), np.arange(2), indexing="ij")
    n = ii.size
    rng = np.random.default_rng(2)
    st = lpgen.State(ii.ravel() * 1.0, jj.ravel() * 1.0, 1.0 + kk.ravel() * 1.0,
                     rng.standard_normal(n), rng.standard_normal(n),
                     rng.standard_normal(n), np.full(n, 1.0 / (0.5 * p.phi_min)))
    off = np.array([0, n])
    dt = 1e-3
    new, perm, (r1, r2) = oracle.step2(st, off, [p], dt)
    s = st.take(perm)
    for r in (r1, r2):
        assert np.allclose(r["acc"], g[:, None], rtol=0, atol=1e-12)
        assert np.all(r["dVdt"] == 0.0)
    for a, (x, u, gk) in enumerate(zip((s.x, s.y, s.z), (s.u, s.v, s.w), g)):
        xe = x + dt * u + 0.5 * dt * dt * gk
        ue = u + dt * gk
        assert np.max(np.abs(new.arrays()[a] - xe)) <= 1e-14, a
        assert np.max(np.abs(new.arrays()[3 + a] - ue)) <= 1e-14, a
    assert np.array_equal(new.V, s.V)
