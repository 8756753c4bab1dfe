"""Reduced 1D model of a granular layer on a wall (the verification model
of the paper's granular-layer compression test, Sec. 4.1).

TEST INFRASTRUCTURE ONLY: used by ``tests/`` and the validation leg of
``bench.py``; the HIP library never imports it.

A layer of infinite transverse extent has u = (0, 0, w(z, t)), so the
governing equations of Sec. 2.1 reduce to one dimension:

  d(1/phi)/dt = (1/phi) dw/dz,     rho_s phi dw/dt = d(sigma_zz)/dz - rho_s phi g,

with the stress of Sec. 2.1 (sigma = -P I + eta gd, gd = D - div/3 I):
D = diag(0, 0, w_z), so gd_zz = 2 w_z / 3, |gd| = sqrt(gd:gd / 2) =
|w_z| / sqrt(3), and sigma_zz = -P + (2/3) eta w_z.  The closure is the
one of Sec. 2.2 and 2.2.1 with the readings of the method (the same
regimes as the 3D step): gas (phi <= phi_min) P = eta = 0; inertial
(phi <= phi_max) P = rho_s (2 a d |gd| / (phi_c - phi))^2, a = phi_c -
phi_min, I = (phi_c - phi)/a, mu(I) = mu_s + (mu_2 - mu_s)/(I0/I + 1),
eta = mu P / |gd| (written as rho_s mu k^2 |gd| with k = 2 a d /
(phi_c - phi), finite at |gd| = 0); quasi-static P = rho_s (alpha + beta
phi), eta = 0.

Discretisation (plain Lagrangian finite volumes, independent of the LP
fits): N cells of fixed mass per unit area m_k = rho_s phi_k dz_k between
nodes z_0 = wall (held at rest) < z_1 < ... < z_N (free top, sigma = 0
above).  Cell strain rate (w_{k+1} - w_k)/(z_{k+1} - z_k), cell stress as
above, node acceleration (sigma_k - sigma_{k-1}) / M_k - g with the node
mass M_k = (m_{k-1} + m_k)/2 (m_{N-1}/2 at the top), and semi-implicit
Euler steps (w first, then z with the new w).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Layer1D:
    z: np.ndarray          # node heights, N + 1 (z[0] = wall)
    w: np.ndarray          # node velocities, N + 1
    m: np.ndarray          # cell masses per unit area, N

    def phi(self, rho_s: float) -> np.ndarray:
        return self.m / (rho_s * np.diff(self.z))

    @property
    def height(self) -> float:
        return float(self.z[-1] - self.z[0])


def layer_from_profile(phi_cells: np.ndarray, dz: float, rho_s: float,
                       wall: float = 0.0) -> Layer1D:
    """Layer of cells of height dz and solid fractions phi_cells, at rest."""
    n = len(phi_cells)
    z = wall + dz * np.arange(n + 1, dtype=np.float64)
    return Layer1D(z, np.zeros(n + 1), rho_s * np.asarray(phi_cells, dtype=np.float64) * dz)


def stress_zz(p, phi: np.ndarray, wz: np.ndarray) -> np.ndarray:
    """sigma_zz of the closure for solid fraction phi and strain rate w_z."""
    gdn = np.abs(wz) / np.sqrt(3.0)
    gas = phi <= p.phi_min
    inert = (~gas) & (phi <= p.phi_max)
    quasi = ~(gas | inert)
    a = p.phi_c - p.phi_min
    wd = np.where(inert, p.phi_c - phi, 1.0)
    k = 2.0 * a * p.d / wd
    P_in = p.rho_s * (k * gdn) ** 2
    I = wd / a
    mu = p.mu_s + (p.mu_2 - p.mu_s) / (p.I0 / I + 1.0)
    eta_in = p.rho_s * mu * k * k * gdn
    P = np.where(inert, P_in, np.where(quasi, p.rho_s * (p.alpha + p.beta * phi), 0.0))
    eta = np.where(inert, eta_in, 0.0)
    return -P + (2.0 / 3.0) * eta * wz


def step(p, s: Layer1D, dt: float) -> None:
    """One semi-implicit Euler step in place (the wall node stays at rest)."""
    g = -p.g[2]
    dz = np.diff(s.z)
    phi = s.m / (p.rho_s * dz)
    wz = np.diff(s.w) / dz
    sig = stress_zz(p, phi, wz)
    acc = np.empty_like(s.w)
    M = 0.5 * (s.m[:-1] + s.m[1:])
    acc[1:-1] = (sig[1:] - sig[:-1]) / M - g
    acc[-1] = (0.0 - sig[-1]) / (0.5 * s.m[-1]) - g
    acc[0] = 0.0
    s.w += dt * acc
    s.w[0] = 0.0
    s.z += dt * s.w


def run(p, s: Layer1D, dt: float, t_end: float, every: float):
    """Steps to t_end; returns (times, heights) sampled every `every` s."""
    ts, hs = [0.0], [s.height]
    nsteps = int(round(t_end / dt))
    per = max(1, int(round(every / dt)))
    for k in range(1, nsteps + 1):
        step(p, s, dt)
        if k % per == 0:
            ts.append(k * dt)
            hs.append(s.height)
    return np.array(ts), np.array(hs)
