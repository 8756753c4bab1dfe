"""FP64 adjoint of the oracle step with frozen stencils (plain PyTorch, CPU).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and nothing else.

The step of ``oracle.step`` is re-expressed with torch float64 CPU
operations on the stencils, ghost masks, mirror sources and fallback flags
that the C oracle computed for the state (those are piecewise constant in
the state, so they are held fixed, as the derivative of the step requires):

  mirrors (Sec. 3.1 step 9) -> Taylor rows xi = (x_k - x_i)/h and ghost rows
  (Sec. 3.1 steps 5-7) -> least squares for u, v, w (normal equations) ->
  mu(I) closure (Sec. 2.2, 2.2.1) -> least squares for P and eta -> Form E
  right-hand side (Sec. 2.1) -> explicit update (Sec. 3.1 steps 8, 10).

Its reverse is torch.autograd's exact chain rule through these operations.
Conventions at the non-smooth points: the shear-rate norm has zero
derivative where it is zero; branch and stencil choices are constant.
``tests/test_oracle_adjoint.py`` pins the forward against the C oracle and
the reverse against central differences of the C oracle step.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np
import torch

from lpgen import Params, State

from . import Oracle, sort_perm, SKIN_DEFAULT

# parameter record order (16 doubles per system)
_RHO, _D, _MUS, _MU2, _I0, _PHIC, _PHIMIN, _PHIMAX, _ALPHA, _BETA = range(10)
_GX, _H, _WALL = 10, 13, 15
_XLO, _YLO, _LX, _LY = 16, 17, 18, 19
# second-derivative index of the pair (a, b)
_HIDX = ((3, 6, 7), (6, 4, 8), (7, 8, 5))
_SIGNS = torch.tensor([[(1.0 if (o & 1) else -1.0), (1.0 if (o & 2) else -1.0),
                        (1.0 if (o & 4) else -1.0)] for o in range(8)],
                      dtype=torch.float64)


def _taylor(ex, ey, ez):
    return torch.stack([ex, ey, ez, 0.5 * ex * ex, 0.5 * ey * ey, 0.5 * ez * ez,
                        ex * ey, ex * ez, ey * ez], dim=-1)


def theta_of(params: Sequence[Params]) -> np.ndarray:
    """(mu_s, mu_2, I0) of every system, n_sys x 3."""
    return np.array([[p.mu_s, p.mu_2, p.I0] for p in params], dtype=np.float64)


class FrozenStep:
    """One oracle step of a state that is already in the step's particle
    order, as a differentiable torch function of (state, theta)."""

    def __init__(self, state: State, offsets, params: Sequence[Params], dt: float,
                 cfg=None, brute=None):
        o = Oracle(state, offsets, params, cfg, brute)
        nb = o.neighbours()
        ev = o.evaluate()
        self.n = n = state.n
        self.dt = float(dt)
        self.ref = ev
        off = np.asarray(offsets, dtype=np.int64)
        sys = np.zeros(n, dtype=np.int64)
        for s in range(len(params)):
            sys[off[s]:off[s + 1]] = s
        self.sys = torch.from_numpy(sys)
        self.prm = torch.tensor(np.stack([p.as_vector() for p in params]),
                                dtype=torch.float64)
        m = nb.sten_idx.shape[1]
        cnt = nb.sten_cnt.astype(np.int64)
        self.mask = torch.from_numpy(np.arange(m)[None, :] < cnt[:, None])
        idx = np.where(self.mask.numpy(), nb.sten_idx, 0).astype(np.int64)
        self.sten = torch.from_numpy(idx)
        gm = nb.ghost_mask.astype(np.int64)
        self.gmask = torch.from_numpy(((gm[:, None] >> np.arange(8)[None, :]) & 1)
                                      .astype(bool))
        self.msrc = torch.from_numpy(nb.mirror_src.astype(np.int64))
        # periodic axes: the copy of each stencil point nearest to the
        # particle (shift -L when x_j - x_i > L/2, +L below -L/2), frozen
        pts = np.concatenate([np.arange(n), nb.mirror_src.astype(np.int64)])
        prm = self.prm.numpy()
        self.shift = []
        for coord, lcol in ((state.x, _LX), (state.y, _LY)):
            L = prm[sys, lcol][:, None]
            c = np.asarray(coord, dtype=np.float64)
            d = c[pts][idx] - c[:, None]
            sh = np.where((L > 0) & (d > 0.5 * L), -L,
                          np.where((L > 0) & (d < -0.5 * L), L, 0.0))
            self.shift.append(torch.from_numpy(np.ascontiguousarray(sh)))
        self.lin = torch.from_numpy((ev["flags"] & 1).astype(bool))
        nrows = cnt + self.gmask.numpy().sum(axis=1)
        self.few = torch.from_numpy(nrows < 3)

    def _per(self, col):
        return self.prm[self.sys, col]

    def _solve(self, A, B):
        """Least squares for each particle: A (n, m, 9), B (n, m, k) ->
        (n, 9, k); the linear fallback keeps 3 columns (others 0)."""
        G = A.transpose(1, 2) @ A
        R = A.transpose(1, 2) @ B
        eye = torch.eye(9, dtype=torch.float64)
        keep3 = torch.zeros(9, 9, dtype=torch.float64)
        keep3[:3, :3] = 1.0
        lin = self.lin[:, None, None]
        G = torch.where(lin, G * keep3 + eye * (1.0 - keep3), G)
        R = torch.where(lin, R * (torch.arange(9) < 3)[None, :, None], R)
        few = self.few[:, None, None]
        G = torch.where(few, eye.expand_as(G), G)
        R = torch.where(few, torch.zeros_like(R), R)
        return torch.linalg.solve(G, R)

    def forward(self, x, y, z, u, v, w, V, theta):
        acc, dVdt = self.rhs(x, y, z, u, v, w, V, theta)
        dt = self.dt
        un = u + dt * acc[0]
        vn = v + dt * acc[1]
        wn = w + dt * acc[2]
        xn = self.wrap(x + dt * (0.5 * (u + un)), 0)
        yn = self.wrap(y + dt * (0.5 * (v + vn)), 1)
        zn = z + dt * (0.5 * (w + wn))
        Vn = V + dt * dVdt
        return xn, yn, zn, un, vn, wn, Vn

    def wrap(self, c, axis):
        """Coordinate along axis 0 (x) or 1 (y) mapped into the periodic box
        (a shift by a constant: derivative 1)."""
        lo = self._per(_XLO + axis)
        L = self._per(_LX + axis)
        per = L > 0
        c = torch.where(per & (c >= lo + L), c - L, c)
        return torch.where(per & (c < lo), c + L, c)

    def rhs(self, x, y, z, u, v, w, V, theta):
        """Acceleration (3 tensors) and dV/dt of Sec. 2.1 (Form E) on the
        frozen stencils."""
        n = self.n
        h = self._per(_H)
        wall = self._per(_WALL)
        ms = self.msrc
        # mirrors: (x, y, 2 wall - z), (u, v, -w), same V
        X = torch.cat([x, x[ms]])
        Y = torch.cat([y, y[ms]])
        Z = torch.cat([z, 2.0 * wall[ms] - z[ms]])
        Ua = torch.cat([u, u[ms]])
        Va = torch.cat([v, v[ms]])
        Wa = torch.cat([w, -w[ms]])
        S, mk = self.sten, self.mask
        mkf = mk.to(torch.float64)
        ex = ((X[S] + self.shift[0]) - x[:, None]) / h[:, None]
        ey = ((Y[S] + self.shift[1]) - y[:, None]) / h[:, None]
        ez = (Z[S] - z[:, None]) / h[:, None]
        As = _taylor(ex, ey, ez) * mkf[..., None]
        Ag = _taylor(_SIGNS[:, 0], _SIGNS[:, 1], _SIGNS[:, 2])[None, :, :] * \
            self.gmask.to(torch.float64)[..., None]
        A = torch.cat([As, Ag], dim=1)
        zg = torch.zeros(n, 8, dtype=torch.float64)

        def rhs(fa, fi, ghost):
            return torch.cat([(fa[S] - fi[:, None]) * mkf, ghost], dim=1)

        Bu = torch.stack([rhs(Ua, u, zg), rhs(Va, v, zg), rhs(Wa, w, zg)], dim=2)
        cu = self._solve(A, Bu)                       # (n, 9, 3)
        inv = torch.stack([1.0 / h] * 3 + [1.0 / (h * h)] * 6, dim=1)  # (n, 9)
        coef = cu * inv[:, :, None]                   # coef[i, q, f]
        # closure at the reals
        Gm = coef[:, :3, :].transpose(1, 2)           # Gm[i, a, b] = d u_a / d x_b
        div = Gm[:, 0, 0] + Gm[:, 1, 1] + Gm[:, 2, 2]
        D = 0.5 * (Gm + Gm.transpose(1, 2))
        gd = D - (div / 3.0)[:, None, None] * torch.eye(3, dtype=torch.float64)
        ss = (gd * gd).sum(dim=(1, 2))
        pos = ss > 0
        gn = torch.where(pos, torch.sqrt(0.5 * torch.where(pos, ss, torch.ones_like(ss))),
                         torch.zeros_like(ss))
        phi = 1.0 / V
        rho, d = self._per(_RHO), self._per(_D)
        phic, phimin, phimax = self._per(_PHIC), self._per(_PHIMIN), self._per(_PHIMAX)
        alpha, beta = self._per(_ALPHA), self._per(_BETA)
        mus, mu2, I0 = theta[self.sys, 0], theta[self.sys, 1], theta[self.sys, 2]
        gas = phi <= phimin
        inert = (~gas) & (phi <= phimax)
        quasi = ~(gas | inert)
        aa = phic - phimin
        wd = torch.where(inert, phic - phi, torch.ones_like(phi))
        k = 2.0 * aa * d / wd
        P_in = rho * (k * gn) * (k * gn)
        I = wd / aa
        mu = mus + (mu2 - mus) / (I0 / I + 1.0)
        E_in = rho * mu * k * k * gn
        P_qs = rho * (alpha + beta * phi)
        zero = torch.zeros_like(phi)
        P = torch.where(inert, P_in, torch.where(quasi, P_qs, zero))
        eta = torch.where(inert, E_in, zero)
        # mirrors: the source's density at zero shear rate; ghosts: 0
        phs = 1.0 / V[ms]
        rs = self.prm[self.sys[ms]]
        Pm = torch.where(phs > rs[:, _PHIMAX], rs[:, _RHO] * (rs[:, _ALPHA] + rs[:, _BETA] * phs),
                         torch.zeros_like(phs))
        Pa = torch.cat([P, Pm])
        Ea = torch.cat([eta, torch.zeros_like(Pm)])
        gP_gh = (-P)[:, None].expand(n, 8) * self.gmask.to(torch.float64)
        gE_gh = (-eta)[:, None].expand(n, 8) * self.gmask.to(torch.float64)
        B2 = torch.stack([rhs(Pa, P, gP_gh), rhs(Ea, eta, gE_gh)], dim=2)
        c2 = self._solve(A, B2)                       # (n, 9, 2)
        gP = c2[:, :3, 0] / h[:, None]
        gE = c2[:, :3, 1] / h[:, None]
        # Form E right-hand side
        acc = []
        for a in range(3):
            lap = sum(coef[:, _HIDX[b][b], a] for b in range(3))
            gdiv = sum(coef[:, _HIDX[a][b], b] for b in range(3))
            tg = sum(gd[:, a, b] * gE[:, b] for b in range(3))
            force = -gP[:, a] + tg + eta * (0.5 * lap + gdiv / 6.0)
            acc.append(V * force / rho + self._per(_GX + a))
        dVdt = V * div
        return acc, dVdt

    def run(self, state: State, theta: np.ndarray) -> State:
        t = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
             for a in state.arrays()]
        out = self.forward(*t, torch.from_numpy(np.asarray(theta, dtype=np.float64)))
        return State(*[o.detach().numpy() for o in out])

    def vjp(self, state: State, theta: np.ndarray, lam: Sequence[np.ndarray]):
        """dL/d(state) and dL/dtheta for dL/d(new state) = lam."""
        t = [torch.tensor(np.asarray(a, dtype=np.float64), requires_grad=True)
             for a in state.arrays()]
        th = torch.tensor(np.asarray(theta, dtype=np.float64), requires_grad=True)
        out = self.forward(*t, th)
        g = torch.autograd.grad(out, t + [th],
                                grad_outputs=[torch.from_numpy(np.asarray(l, dtype=np.float64))
                                              for l in lam],
                                allow_unused=True)
        res = [np.zeros(state.n) if gi is None else gi.numpy() for gi in g[:7]]
        gth = np.zeros_like(theta) if g[7] is None else g[7].numpy()
        return res, gth


class FrozenStep2(FrozenStep):
    """One second-order oracle step (oracle.step2: Heun's rule on the
    right-hand side f = (u, acc, dVdt)) of a state already in the step's
    order, differentiable in (state, theta): stencils of s and of the
    predictor s* = s + dt f(s) (as the C oracle selects them) held fixed."""

    def __init__(self, state: State, offsets, params: Sequence[Params], dt: float,
                 cfg=None, brute=None):
        super().__init__(state, offsets, params, dt, cfg, brute)
        ev = self.ref
        a, d = ev["acc"], ev["dVdt"]
        pred = State(state.x + dt * state.u, state.y + dt * state.v,
                     state.z + dt * state.w, state.u + dt * a[0],
                     state.v + dt * a[1], state.w + dt * a[2], state.V + dt * d)
        self.stage2 = FrozenStep(pred, offsets, params, dt, cfg, brute)

    def forward(self, x, y, z, u, v, w, V, theta):
        dt = self.dt
        a1, d1 = self.rhs(x, y, z, u, v, w, V, theta)
        pos, vel = (x, y, z), (u, v, w)
        ps = [p + dt * q for p, q in zip(pos, vel)]
        vs = [q + dt * a for q, a in zip(vel, a1)]
        Vs = V + dt * d1
        a2, d2 = self.stage2.rhs(*ps, *vs, Vs, theta)
        half = 0.5 * dt
        xn = [p + half * (q + qs) for p, q, qs in zip(pos, vel, vs)]
        xn = [self.wrap(xn[0], 0), self.wrap(xn[1], 1), xn[2]]
        un = [q + half * (b1 + b2) for q, b1, b2 in zip(vel, a1, a2)]
        return (*xn, *un, V + half * (d1 + d2))


def _order(state, offsets, params, skin, sort):
    if sort:
        return sort_perm(state, offsets, params, skin)[0]
    return np.arange(state.n, dtype=np.int32)


def step2_vjp(state: State, offsets, params: Sequence[Params], dt: float,
              lam: Sequence[np.ndarray], skin: float = SKIN_DEFAULT, brute=None,
              sort: bool = True):
    """Adjoint of oracle.step2 (Morton re-sort, Heun step) at `state`, with
    the conventions of step_vjp."""
    perm = _order(state, offsets, params, skin, sort)
    st = state.take(perm)
    st = State(*[np.ascontiguousarray(a) for a in st.arrays()])
    fs = FrozenStep2(st, offsets, params, dt, brute=brute)
    g, gth = fs.vjp(st, theta_of(params), lam)
    out = []
    for a in g:
        b = np.empty_like(a)
        b[perm] = a
        out.append(b)
    return out, gth, perm


def step_vjp(state: State, offsets, params: Sequence[Params], dt: float,
             lam: Sequence[np.ndarray], skin: float = SKIN_DEFAULT, brute=None,
             sort: bool = True):
    """Adjoint of oracle.step (Morton re-sort, RHS, update) at `state`:
    lam is dL/d(new state) in the step's output order; returns
    (dL/d(state) in the input order, dL/dtheta (n_sys x 3), perm).  With
    ``sort`` false the step keeps the given order (perm is the identity),
    as oracle.step(sort=False) does."""
    perm = _order(state, offsets, params, skin, sort)
    st = state.take(perm)
    st = State(*[np.ascontiguousarray(a) for a in st.arrays()])
    fs = FrozenStep(st, offsets, params, dt, brute=brute)
    g, gth = fs.vjp(st, theta_of(params), lam)
    out = []
    for a in g:
        b = np.empty_like(a)
        b[perm] = a
        out.append(b)
    return out, gth, perm
