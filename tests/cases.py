"""Seeded parity workloads shared by the oracle and GPU tests (inputs
only: lpgen states, never results)."""
import numpy as np

import lpgen


def _with_flow(wl):
    """Smooth velocities and a density field visiting all three regimes."""
    st = wl.state
    st.u = 0.3 * np.sin(3.1 * st.y / wl.params[0].h * 0.0625 + 1.0) * np.cos(2.0 * st.z)
    st.v = 0.2 * np.cos(2.3 * st.x) * np.sin(1.7 * st.z + 0.4)
    st.w = 0.25 * np.sin(2.9 * st.x + 1.1 * st.y)
    st.V = 1.0 / (0.47 + 0.15 * np.sin(4.0 * st.z / (wl.params[0].h * 16) + 2.0 * st.y))
    return wl


def _ragged(wl, drop=37):
    """Drops `drop` seeded particles so the count is not a tile multiple."""
    rng = np.random.default_rng(5)
    keep = np.sort(rng.choice(wl.n, wl.n - drop, replace=False))
    wl.state = wl.state.take(keep)
    wl.offsets = np.array([0, wl.state.n])
    return wl


def _exact_lattice(nx=12, ny=10, nz=9):
    """Unjittered lattice: many exactly equal distances, so every stencil
    cut is decided by the id tie-break."""
    h = 1.0 / 16.0
    p = lpgen.default_params(h)
    st = lpgen.lattice_column(nx, ny, nz, h, seed=7, jitter=0.0, params=p)
    return lpgen.Workload("lattice_exact", st, np.array([0, st.n]), [p], 1e-4, 1)


def _sparse_cloud(n=1500, seed=11):
    """Seeded random cloud of 1500 particles in a 1.5 m box on the wall,
    about 7 neighbours each within R: many particles have fewer than 9 rows
    (linear fallback), uncovered octants (ghosts) and gas-regime volumes."""
    h = 1.0 / 16.0
    p = lpgen.default_params(h)
    u = lpgen.uniform01(seed, np.arange(7 * n, dtype=np.uint64)).reshape(7, n)
    side = 1.5
    st = lpgen.State(side * u[0], side * u[1], side * u[2] + 0.001,
                     0.2 * (u[3] - 0.5), 0.2 * (u[4] - 0.5), 0.2 * (u[5] - 0.5),
                     1.0 / (0.30 + 0.32 * u[6]))
    return lpgen.Workload("sparse_cloud", st, np.array([0, n]), [p], 1e-4, 1)


def _periodic_layer(nx=12, ny=10, nz=8, axes=(True, True), seed=13):
    """Layer periodic along x and/or y (box [0, nx h) x [0, ny h)) with
    velocities and volumes that are smooth across the periodic faces, so
    that stencils there reach through them."""
    h = 1.0 / 16.0
    Lx, Ly = nx * h, ny * h
    p = lpgen.default_params(h, box_lo=(0.0, 0.0),
                             box_len=(Lx if axes[0] else 0.0, Ly if axes[1] else 0.0))
    st = lpgen.lattice_column(nx, ny, nz, h, seed=seed, params=p)
    kx, ky = 2.0 * np.pi / Lx, 2.0 * np.pi / Ly
    st.u = 0.3 * np.sin(kx * st.x) * np.cos(2.0 * st.z)
    st.v = 0.2 * np.cos(ky * st.y + 0.3) * np.sin(1.7 * st.z + 0.4)
    st.w = 0.25 * np.sin(kx * st.x + ky * st.y)
    st.V = 1.0 / (0.47 + 0.15 * np.sin(4.0 * st.z / (h * 16) + ky * st.y))
    name = "periodic_xy" if all(axes) else "periodic_x"
    return lpgen.Workload(name, st, np.array([0, st.n]), [p], 1e-4, 1)


CASES = {
    "column16": lambda: lpgen.column_small(),
    "lattice_exact": lambda: _with_flow(_exact_lattice()),
    "column16_flow_ragged": lambda: _ragged(_with_flow(lpgen.column_small())),
    "sheared_20x20x12": lambda: lpgen.column_sheared(nx=20, ny=20, nz=12),
    "ensemble_3": lambda: _with_flow(lpgen.ensemble(n_sys=3, n_lo=600, n_hi=3000)),
    "sparse_cloud": lambda: _sparse_cloud(),
    "periodic_xy": lambda: _periodic_layer(),
    "periodic_x": lambda: _periodic_layer(12, 9, 11, axes=(True, False), seed=17),
}
