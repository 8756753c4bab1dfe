"""Pins of the optional reflecting wall (a reading: the paper states only
the mirror boundary): a particle that ends a step below the wall plane is
reflected across it (z -> 2 wall - z, w -> -w).  An isolated gas-regime
particle falling through the wall gives the closed form."""
import numpy as np
import pytest

import lpgen
import oracle


def _faller(wall=0.0):
    h = 1.0 / 16.0
    p = lpgen.default_params(h, wall_z=wall)
    # two particles far apart; the first falls through the wall in one step
    st = lpgen.State(np.array([0.0, 5.0]), np.array([0.0, 5.0]),
                     np.array([wall + 0.001, wall + 3.0]),
                     np.array([0.1, 0.0]), np.zeros(2), np.array([-2.0, 0.0]),
                     np.full(2, 1.0 / (0.5 * p.phi_min)))
    return st, np.array([0, 2]), [p], np.array(p.g)


@pytest.mark.parametrize("fn", [oracle.step, oracle.step2])
@pytest.mark.parametrize("wall", [0.0, 0.37])
def test_reflecting_wall_closed_form(fn, wall):
    st, off, prm, g = _faller(wall)
    dt = 1e-3
    out, perm, _ = fn(st, off, prm, dt, sort=False, cfg=dict(wall_reflect=1))
    z_free = st.z + dt * st.w + 0.5 * dt * dt * g[2]
    w_free = st.w + dt * g[2]
    assert z_free[0] < wall                      # it crossed the wall
    assert abs(out.z[0] - (2.0 * wall - z_free[0])) <= 1e-15
    assert abs(out.w[0] + w_free[0]) <= 1e-13
    assert abs(out.z[1] - z_free[1]) <= 1e-14 and abs(out.w[1] - w_free[1]) <= 1e-13
    # without the option the particle stays below the wall
    out0, _, _ = fn(st, off, prm, dt, sort=False)
    assert out0.z[0] < wall and abs(out0.w[0] - w_free[0]) <= 1e-13


def test_hydrostatic_mirror_pressure_supports_the_bottom_rows():
    """A 16^3 column at rest in quasi-static equilibrium: with the literal
    mirror (P(phi_src) at zero shear rate) the bottom row accelerates at
    about 2/3 g; with the hydrostatic wall pressure its acceleration is
    that of the interior rows (the small residual of the discrete
    equilibrium), as full support requires."""
    wl = lpgen.column_small()
    h = wl.params[0].h
    row = np.floor(wl.state.z / h).astype(int)
    res = {}
    for wp in (0, 1):
        r = oracle.Oracle(wl.state, wl.offsets, wl.params, cfg=dict(wall_pressure=wp)).evaluate()
        res[wp] = [float(r["acc"][2][row == k].mean()) for k in range(5)]
    interior = np.mean(res[1][2:])
    assert res[0][0] < -5.0
    assert abs(res[1][0] - interior) < 0.05 and abs(res[1][1] - interior) < 0.05
    assert abs(interior) < 0.5
