"""Seeded synthetic inputs for the Lagrangian-particle granular-flow step.

This module is shared by the CPU oracle and the HIP path.  It holds no part
of the method's arithmetic: it only draws random numbers, lays particles on
a jittered lattice and fills the physical-parameter record.  Everything here
is plain numpy.

Workloads are the granular-column collapse problems of the paper's
validation section (Sec. 4.2, axisymmetric collapsing column), at the sizes
of the benchmark configurations:

* ``column_small``   16 x 16 x 16   = 4,096 particles,   h = 1/16 m
* ``column_bench``   64 x 64 x 128  = 524,288 particles, h = 0.5/64 m
* ``column_sheared`` 128 x 128 x 64 = 1,048,576 particles after a seeded
  smooth shear (uneven stencils)
* ``column_adjoint`` 32 x 32 x 128  = 131,072 particles
* ``ensemble``       64 independent columns of seeded size and parameters

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  The generator is counter
based: draw ``k`` of stream ``seed`` is ``mix(seed + (k + 1) * GAMMA)``, so
any draw can be produced independently and in any order.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
BASE_SEED = 220614061


def splitmix64(seed: int, k: np.ndarray) -> np.ndarray:
    """Draws ``k`` (uint64 array of counters) of the SplitMix64 stream ``seed``."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (k + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, k: np.ndarray) -> np.ndarray:
    """U[0,1) doubles with 53 random bits: (draw >> 11) * 2^-53."""
    return (splitmix64(seed, k) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


@dataclasses.dataclass
class Params:
    """Physical parameters of one granular system (one column).

    ``rho_s`` is the grain material density (the paper's phi_s), ``d`` the
    grain diameter, ``mu_s, mu_2, I0`` the mu(I) friction-law constants,
    ``phi_c, phi_min, phi_max`` the critical, minimum and quasi-static
    threshold solid fractions, ``alpha, beta`` the quasi-static pressure
    constants of P = rho_s (alpha + beta phi), ``g`` gravity, ``h`` the
    inter-particle spacing, ``R`` the neighbour radius and ``wall_z`` the
    height of the solid wall plane z = wall_z.  ``box_lo`` and ``box_len``
    give the periodic box along x and y: an axis with ``box_len`` > 0 is
    periodic with period ``box_len`` over [box_lo, box_lo + box_len); 0
    leaves it open.
    """
    rho_s: float = 2450.0
    d: float = 5e-4
    mu_s: float = 0.38
    mu_2: float = 0.64
    I0: float = 0.279
    phi_c: float = 0.60
    phi_min: float = 0.35
    phi_max: float = 0.59
    alpha: float = -1200.0 * 0.59
    beta: float = 1200.0
    g: tuple = (0.0, 0.0, -9.81)
    h: float = 1.0 / 16.0
    R: float = 2.5 / 16.0
    wall_z: float = 0.0
    box_lo: tuple = (0.0, 0.0)
    box_len: tuple = (0.0, 0.0)

    def as_vector(self) -> np.ndarray:
        """Flat float64 record in the order rho_s, d, mu_s, mu_2, I0, phi_c,
        phi_min, phi_max, alpha, beta, gx, gy, gz, h, R, wall_z, x_lo, y_lo,
        Lx, Ly."""
        return np.array([self.rho_s, self.d, self.mu_s, self.mu_2, self.I0,
                         self.phi_c, self.phi_min, self.phi_max, self.alpha,
                         self.beta, self.g[0], self.g[1], self.g[2], self.h,
                         self.R, self.wall_z, self.box_lo[0], self.box_lo[1],
                         self.box_len[0], self.box_len[1]], dtype=np.float64)


def default_params(h: float, **kw) -> Params:
    """Material constants of the benchmark columns with spacing ``h``; the
    neighbour radius is 2.5 h."""
    beta = kw.pop("beta", 1200.0)
    phi_max = kw.pop("phi_max", 0.59)
    p = Params(h=h, R=2.5 * h, beta=beta, phi_max=phi_max,
               alpha=-beta * phi_max, **kw)
    return p


@dataclasses.dataclass
class State:
    """Structure-of-arrays particle state (float64, host)."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    V: np.ndarray

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def arrays(self) -> List[np.ndarray]:
        return [self.x, self.y, self.z, self.u, self.v, self.w, self.V]

    def copy(self) -> "State":
        return State(*[a.copy() for a in self.arrays()])

    def take(self, idx: np.ndarray) -> "State":
        return State(*[a[idx] for a in self.arrays()])

    @staticmethod
    def concat(states: List["State"]) -> "State":
        return State(*[np.concatenate([s.arrays()[k] for s in states])
                       for k in range(7)])


@dataclasses.dataclass
class Workload:
    """A batch of independent systems: particles of system s occupy
    ``offsets[s]:offsets[s+1]``; ``params[s]`` holds its constants."""
    name: str
    state: State
    offsets: np.ndarray
    params: List[Params]
    dt: float
    steps: int

    @property
    def n(self) -> int:
        return self.state.n

    @property
    def n_sys(self) -> int:
        return len(self.params)


def lattice_column(nx: int, ny: int, nz: int, h: float, seed: int,
                   jitter: float = 0.05, x0: float = 0.0, y0: float = 0.0,
                   params: Optional[Params] = None) -> State:
    """Column of particles at ((i+1/2)h, (j+1/2)h, (k+1/2)h) + (x0, y0, 0),
    id = i + nx (j + ny k), each coordinate jittered by U(-jitter h,
    jitter h) drawn in id order, x then y then z (draw 3 id + axis).

    Velocity is zero.  The specific volume V = 1/phi follows the hydrostatic
    profile phi = phi_max exp(|g| (H - z) / beta) with H = nz h, which is the
    quasi-static equilibrium of the pressure law P = rho_s beta (phi - phi_max)
    under gravity.
    """
    p = params if params is not None else default_params(h)
    n = nx * ny * nz
    ids = np.arange(n, dtype=np.int64)
    i = ids % nx
    j = (ids // nx) % ny
    k = ids // (nx * ny)
    draws = uniform01(seed, np.arange(3 * n, dtype=np.uint64)).reshape(n, 3)
    jit = (2.0 * draws - 1.0) * (jitter * h)
    x = x0 + (i + 0.5) * h + jit[:, 0]
    y = y0 + (j + 0.5) * h + jit[:, 1]
    z = (k + 0.5) * h + jit[:, 2]
    H = nz * h
    gmag = abs(p.g[2])
    phi = p.phi_max * np.exp(gmag * (H - z) / p.beta)
    V = 1.0 / phi
    zero = np.zeros(n)
    return State(x, y, z, zero.copy(), zero.copy(), zero.copy(), V)


def smooth_field(seed: int, pts: np.ndarray, wavelength: float,
                 modes: int = 8) -> np.ndarray:
    """Seeded smooth vector field f(x) = sum_q c_q cos(kappa_q . x + theta_q)
    per component, |kappa_q| = 2 pi / wavelength, direction uniform on the
    sphere, c_q ~ U(-1,1), theta_q ~ U(0, 2 pi), each component normalised to
    max |f_a| = 1 over ``pts``.  Draw order: component a, mode q, then
    (cos-polar u, azimuth, amplitude, phase) = draws 4 (modes a + q) + 0..3.
    """
    out = np.zeros_like(pts)
    kmag = 2.0 * math.pi / wavelength
    for a in range(3):
        acc = np.zeros(pts.shape[0])
        for q in range(modes):
            base = 4 * (modes * a + q)
            d = uniform01(seed, np.arange(base, base + 4, dtype=np.uint64))
            ct = 2.0 * d[0] - 1.0
            st = math.sqrt(max(0.0, 1.0 - ct * ct))
            ph = 2.0 * math.pi * d[1]
            kvec = kmag * np.array([st * math.cos(ph), st * math.sin(ph), ct])
            c = 2.0 * d[2] - 1.0
            th = 2.0 * math.pi * d[3]
            acc += c * np.cos(pts @ kvec + th)
        m = np.max(np.abs(acc))
        out[:, a] = acc / m if m > 0 else acc
    return out


def column_small(seed: int = BASE_SEED + 1) -> Workload:
    """16^3 = 4,096-particle column, h = 1/16 m (a 1 m cube) on the wall z=0;
    one RHS evaluation plus 10 explicit steps of dt = 1e-4 s."""
    h = 1.0 / 16.0
    p = default_params(h)
    st = lattice_column(16, 16, 16, h, seed, params=p)
    return Workload("column_16x16x16", st, np.array([0, st.n]), [p], 1e-4, 10)


def column_bench(seed: int = BASE_SEED + 2, nx: int = 64, ny: int = 64,
                 nz: int = 128) -> Workload:
    """64 x 64 x 128 = 524,288-particle column (0.5 x 0.5 x 1.0 m, aspect 2),
    h = 0.5/64 m; 100 steps of dt = 2e-5 s."""
    h = 0.5 / 64.0
    p = default_params(h)
    st = lattice_column(nx, ny, nz, h, seed, params=p)
    return Workload(f"column_{nx}x{ny}x{nz}", st, np.array([0, st.n]), [p],
                    2e-5, 100)


def column_sheared(seed: int = BASE_SEED + 3, nx: int = 128, ny: int = 128,
                   nz: int = 64) -> Workload:
    """128 x 128 x 64 = 1,048,576 particles, h = 0.5/64 m, after a seeded
    smooth shear of wavelength 8h: u = 0.5 m/s f(x) and positions displaced
    by 2h f(x) (z clamped to >= h/4), which opens free surfaces and spreads
    the stencil sizes; 20 steps of dt = 2e-5 s."""
    h = 0.5 / 64.0
    p = default_params(h)
    st = lattice_column(nx, ny, nz, h, seed, params=p)
    pts = np.stack([st.x, st.y, st.z], axis=1)
    f = smooth_field(seed + 1000, pts, 8.0 * h)
    st.u = 0.5 * f[:, 0]
    st.v = 0.5 * f[:, 1]
    st.w = 0.5 * f[:, 2]
    st.x = st.x + 2.0 * h * f[:, 0]
    st.y = st.y + 2.0 * h * f[:, 1]
    st.z = np.maximum(st.z + 2.0 * h * f[:, 2], 0.25 * h)
    return Workload(f"sheared_{nx}x{ny}x{nz}", st, np.array([0, st.n]), [p],
                    2e-5, 20)


def column_adjoint(seed: int = BASE_SEED + 4, nx: int = 32, ny: int = 32,
                   nz: int = 128) -> Workload:
    """32 x 32 x 128 = 131,072-particle column, h = 0.5/64 m (0.25 x 0.25 x
    1.0 m at x in [0, 0.25]); 50 steps of dt = 5e-5 s."""
    h = 0.5 / 64.0
    p = default_params(h)
    st = lattice_column(nx, ny, nz, h, seed, params=p)
    return Workload(f"adjoint_{nx}x{ny}x{nz}", st, np.array([0, st.n]), [p],
                    5e-5, 50)


def ensemble(seed: int = BASE_SEED + 5, n_sys: int = 64,
             n_lo: int = 8000, n_hi: int = 200000) -> Workload:
    """``n_sys`` independent columns.  Per column c, four draws in order:
    N_c = n_lo + floor(U (n_hi - n_lo + 1)), aspect A_c = 0.5 + 3.5 U,
    mu_s = 0.3 + 0.15 U, I0 = 0.2 + 0.15 U; mu_2 = mu_s + 0.26;
    nx = ny = round((N_c / A_c)^(1/3)), nz = round(A_c nx), h = 0.5/64 m.
    Columns are placed side by side in x (2 m apart) and never interact."""
    h = 0.5 / 64.0
    states, params, offs = [], [], [0]
    for c in range(n_sys):
        d = uniform01(seed, np.arange(4 * c, 4 * c + 4, dtype=np.uint64))
        Nc = n_lo + int(math.floor(d[0] * (n_hi - n_lo + 1)))
        Ac = 0.5 + 3.5 * d[1]
        mu_s = 0.3 + 0.15 * d[2]
        I0 = 0.2 + 0.15 * d[3]
        nx = max(2, int(round((Nc / Ac) ** (1.0 / 3.0))))
        nz = max(2, int(round(Ac * nx)))
        p = default_params(h, mu_s=mu_s, mu_2=mu_s + 0.26, I0=I0)
        st = lattice_column(nx, nx, nz, h, seed + 7919 * (c + 1), params=p,
                            x0=2.0 * c)
        states.append(st)
        params.append(p)
        offs.append(offs[-1] + st.n)
    return Workload(f"ensemble_{n_sys}", State.concat(states),
                    np.array(offs, dtype=np.int64), params, 2e-5, 20)


def cloud_graded(seed: int = BASE_SEED + 70, n: int = 1 << 20, side_h: int = 96,
                 ratio: float = 0.1) -> Workload:
    """Seeded random cloud whose number density falls exponentially with
    height, from that of the h = 0.5/64 m lattice at the wall to `ratio`
    of it at the top, so that stencils span from full (60 rows) to a few
    neighbours plus ghost rows: the uneven stencils of a free surface.
    Box side_h h square; per particle three draws in id order (x, y, and
    the height by the inverse of the truncated exponential law); solid
    fraction 0.59 times the relative density (quasi-static at the bottom,
    gas at the top); a seeded smooth flow of 0.5 m/s (wavelength 8h);
    dt = 2e-5 s."""
    h = 0.5 / 64.0
    p = default_params(h)
    side = side_h * h
    # n = side^2 rho0 lam (1 - ratio) with rho0 = 1/h^3
    lam = n * h ** 3 / (side * side * (1.0 - ratio))
    top = -lam * math.log(ratio)
    u = uniform01(seed, np.arange(3 * n, dtype=np.uint64)).reshape(n, 3)
    x = side * u[:, 0]
    y = side * u[:, 1]
    z = -lam * np.log1p(-u[:, 2] * (1.0 - ratio)) + 0.25 * h
    rel = np.exp(-(z - 0.25 * h) / lam)
    zero = np.zeros(n)
    st = State(x, y, z, zero.copy(), zero.copy(), zero.copy(), 1.0 / (0.59 * rel))
    f = smooth_field(seed + 1, np.stack([x, y, z], axis=1), 8.0 * h)
    st.u, st.v, st.w = 0.5 * f[:, 0], 0.5 * f[:, 1], 0.5 * f[:, 2]
    assert top > 0.0
    return Workload(f"graded_cloud_{n}", st, np.array([0, n]), [p], 2e-5, 20)


def with_shear_velocity(wl: Workload, seed: int = BASE_SEED + 60,
                        amplitude: float = 0.5, wavelength_h: float = 8.0) -> Workload:
    """Copy of ``wl`` whose initial velocity is the seeded smooth field of
    ``smooth_field`` (wavelength ``wavelength_h`` times the first system's
    h, ``amplitude`` m/s per component), positions and volumes unchanged:
    the divergence of this flow takes particles out of the quasi-static
    branch within a few steps."""
    st = wl.state.copy()
    pts = np.stack([st.x, st.y, st.z], axis=1)
    f = smooth_field(seed, pts, wavelength_h * wl.params[0].h)
    st.u = amplitude * f[:, 0]
    st.v = amplitude * f[:, 1]
    st.w = amplitude * f[:, 2]
    return Workload(wl.name + "_sheared_velocity", st, wl.offsets, wl.params,
                    wl.dt, wl.steps)


def validation_params(h: float, **kw) -> Params:
    """Grain constants of the paper's validation runs (Sec. 4): mu_s =
    tan 30 deg, mu_2 = tan 50 deg, I0 = 2.65, d = 0.32 mm, rho_s = 2600
    kg/m^3; phi_c = 0.60, phi_min = 0.35; the quasi-static law as in
    default_params; R = 2.5 h."""
    base = dict(mu_s=math.tan(math.radians(30.0)), mu_2=math.tan(math.radians(50.0)),
                I0=2.65, d=0.32e-3, rho_s=2600.0)
    base.update(kw)
    return default_params(h, **base)


def layer_profile(z: np.ndarray, H0: float, phi_bottom: float = 0.51,
                  phi_top: float = 0.49) -> np.ndarray:
    """Initial solid fraction of the compression layer: linear in height
    from phi_bottom at the wall to phi_top at z = H0 (mean 0.5, so that
    compaction to phi_c = 0.6 would leave 5/6 of the height)."""
    return phi_bottom + (phi_top - phi_bottom) * np.asarray(z) / H0


def layer_periodic(seed: int = BASE_SEED + 40, nx: int = 12, nz: int = 40,
                   H0: float = 0.03) -> Workload:
    """Granular layer of height H0 = 0.03 m on the wall z = 0, periodic in
    x and y (box nx h x nx h, h = H0 / nz), at rest, with the solid
    fraction of layer_profile (zero pressure: the inertial branch at zero
    shear rate) and the grain constants of validation_params: the
    compression test of the paper's Sec. 4.1.  dt = 5e-6 s; 0.05 s of
    physical time settle it."""
    h = H0 / nz
    L = nx * h
    p = validation_params(h, box_lo=(0.0, 0.0), box_len=(L, L))
    st = lattice_column(nx, nx, nz, h, seed, params=p)
    st.V = 1.0 / layer_profile(st.z, H0)
    return Workload(f"layer_{nx}x{nx}x{nz}", st, np.array([0, st.n]), [p], 5e-6, 10000)


def column_cylinder(seed: int = BASE_SEED + 50, r_i: float = 0.05, h_i: float = 0.03,
                    h: float = 1.25e-3) -> Workload:
    """Axisymmetric column of radius r_i and height h_i (aspect a =
    h_i / r_i = 0.6 by default) standing on the wall z = 0 and released
    at rest: the collapse test of the paper's Sec. 4.2.1.  Jittered lattice
    of spacing h on [-r_i, r_i]^2 x [0, h_i] (lattice_column), keeping the
    particles with x^2 + y^2 <= r_i^2 (lattice order); hydrostatic
    quasi-static solid fraction; grain constants of validation_params.
    dt = 0.2 h / 35 m/s (the quasi-static sound speed is sqrt(beta))."""
    n = int(round(2.0 * r_i / h))
    nz = int(round(h_i / h))
    p = validation_params(h)
    st = lattice_column(n, n, nz, h, seed, x0=-r_i, y0=-r_i, params=p)
    keep = np.nonzero(st.x * st.x + st.y * st.y <= r_i * r_i)[0]
    st = st.take(keep)
    dt = 0.2 * h / math.sqrt(p.beta)
    return Workload(f"cylinder_a{h_i / r_i:.2f}_h{h * 1e3:.2f}mm", st,
                    np.array([0, st.n]), [p], dt, int(math.ceil(0.17 / dt)))


WORKLOADS = {
    "column_small": column_small,
    "column_bench": column_bench,
    "column_sheared": column_sheared,
    "column_adjoint": column_adjoint,
    "ensemble": ensemble,
    "layer_periodic": layer_periodic,
}
