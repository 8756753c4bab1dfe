"""Pins of the reduced 1D layer model (oracle/layer1d.py) used to check the
3D periodic layer (the compression test of Sec. 4.1)."""
import numpy as np
import pytest

import lpgen
import oracle
from oracle import layer1d


def _p(dz=1e-3):
    return lpgen.validation_params(dz)


@pytest.mark.parametrize("phi", [0.40, 0.50, 0.58, 0.595])
@pytest.mark.parametrize("wz", [-30.0, -0.7, 0.0, 2.5])
def test_stress_is_the_3d_closure_in_one_dimension(phi, wz):
    """sigma_zz of the 1D model equals -P + eta gd_zz of the 3D oracle's
    closure for the velocity gradient diag(0, 0, w_z)."""
    p = _p()
    br, P, eta, _, _, gn, gd = oracle.closure_point(p, 1.0 / phi, np.diag([0.0, 0.0, wz]))
    want = -P + eta * gd[2, 2]
    got = float(layer1d.stress_zz(p, np.array([phi]), np.array([wz]))[0])
    assert abs(got - want) <= 1e-12 * max(abs(want), 1.0)
    assert abs(gn - abs(wz) / np.sqrt(3.0)) <= 1e-14 * max(abs(wz), 1.0)


def test_discrete_quasi_static_equilibrium_stays_at_rest():
    """Equal cell masses m stacked so that each cell's quasi-static pressure
    carries the weight above it (P_k = m g (N - k - 1/2)): nothing moves."""
    p = _p()
    N, m = 30, p.rho_s * 0.6 * 1e-3
    g = -p.g[2]
    P = m * g * (N - np.arange(N) - 0.5)
    phi = p.phi_max + P / (p.rho_s * p.beta)
    dz = m / (p.rho_s * phi)
    z = np.concatenate([[0.0], np.cumsum(dz)])
    s = layer1d.Layer1D(z, np.zeros(N + 1), np.full(N, m))
    for _ in range(2000):
        layer1d.step(p, s, 2e-6)
    assert np.max(np.abs(s.w)) <= 1e-9
    assert abs(s.height - z[-1]) <= 1e-12


def test_gas_layer_falls_freely():
    """Below phi_min there is no stress: every node but the wall's falls
    with w = -g t exactly (semi-implicit Euler is exact for the velocity)."""
    p = _p()
    s = layer1d.layer_from_profile(np.full(10, 0.2), 1e-3, p.rho_s, wall=0.5)
    dt, k = 1e-4, 50
    for _ in range(k):
        layer1d.step(p, s, dt)
    g = -p.g[2]
    assert np.allclose(s.w[1:], -g * dt * k, rtol=1e-12, atol=0)
    assert s.w[0] == 0.0


def test_layer_settles_at_the_quasi_static_height():
    """The compression layer (mean phi 0.5, 20 cells) comes to rest with
    phi close to phi_max everywhere: height H0 phi_mean / phi_max (the
    weight of the layer adds g H / beta ~ 2e-4 to phi), mass unchanged."""
    p = _p(0.03 / 20)
    H0, N = 0.03, 20
    zc = (np.arange(N) + 0.5) * H0 / N
    phi0 = lpgen.layer_profile(zc, H0)
    s = layer1d.layer_from_profile(phi0, H0 / N, p.rho_s)
    m0 = s.m.copy()
    ts, hs = layer1d.run(p, s, 4e-6, 0.06, 0.005)
    want = H0 * np.mean(phi0) / p.phi_max
    assert abs(hs[-1] - want) <= 2e-3 * want, (hs[-1], want)
    assert abs(hs[-2] - hs[-1]) <= 1e-4 * want      # at rest
    assert np.array_equal(s.m, m0)
