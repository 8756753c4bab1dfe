"""Gradients through LP trajectories with torch.autograd.

``simulate`` runs ``steps`` LP steps (each: re-sort by the context's cells,
then one step; lp_build_cells + lp_step, or lp_step2 for the second-order
step) and returns the final state as torch tensors that take part in
autograd.  The backward pass runs the library's lp_step_adjoint (or
lp_step2_adjoint) step by step in reverse.  Only every
``checkpoint_every``-th state is kept during the forward pass; each segment
is recomputed from its checkpoint during the backward pass, which
reproduces the forward states exactly (the steps are deterministic).

Gradients flow to the initial state (x, y, z, u, v, w, V) and to the
friction-law parameters theta = (mu_s, mu_2, I0) of every system.  All
arithmetic runs in the HIP library; this module only sequences calls.
"""
from __future__ import annotations

import dataclasses
from typing import Sequence

from . import Context, DeviceState


def _params_with(params: Sequence, theta_host) -> list:
    out = []
    for p, t in zip(params, theta_host):
        out.append(dataclasses.replace(p, mu_s=float(t[0]), mu_2=float(t[1]),
                                       I0=float(t[2])))
    return out


def _torch():
    import torch
    return torch


def _make_function():
    torch = _torch()

    class _Trajectory(torch.autograd.Function):
        @staticmethod
        def forward(fctx, ctx: Context, offsets, params, dt, steps, every, order, theta,
                    *state):
            ctx.set_systems(offsets, _params_with(params, theta.detach().cpu().tolist()))
            st = DeviceState([a.detach().clone() for a in state])
            step = ctx.lp_step2 if order == 2 else ctx.lp_step
            ckpts = {}
            for k in range(steps):
                if k % every == 0:
                    ckpts[k] = st.clone()
                ctx.lp_build_cells(st, want_perm=False)
                step(st, dt)
            fctx.lp = (ctx, dt, steps, every, order, ckpts, theta.device, theta.dtype)
            return tuple(st.t)

        @staticmethod
        def backward(fctx, *gout):
            ctx, dt, steps, every, order, ckpts, tdev, tdt = fctx.lp
            step = ctx.lp_step2 if order == 2 else ctx.lp_step
            adjoint = ctx.lp_step2_adjoint if order == 2 else ctx.lp_step_adjoint
            ref = next(iter(ckpts.values())).t[0]
            lam = DeviceState([torch.zeros_like(ref) if g is None else
                               g.detach().to(torch.float64).contiguous()
                               for g in gout])
            dtheta = torch.zeros(ctx.n_sys, 3, dtype=torch.float64, device=ref.device)
            for k0 in sorted(ckpts, reverse=True):
                k1 = min(k0 + every, steps)
                st = ckpts[k0].clone()
                inputs = []
                for _ in range(k0, k1):
                    inputs.append(st.clone())
                    ctx.lp_build_cells(st, want_perm=False)
                    step(st, dt)
                for s_in in reversed(inputs):
                    lam = adjoint(s_in, dt, lam, dtheta)
            fctx.lp = None
            return (None, None, None, None, None, None, None,
                    dtheta.to(device=tdev, dtype=tdt)) + tuple(lam.t)

    return _Trajectory


_FN = None


def simulate(ctx: Context, offsets, params: Sequence, state: Sequence, theta, dt: float,
             steps: int, checkpoint_every: int = 10, order: int = 1):
    """Final state (7 tensors, the order after the last re-sort) of `steps`
    steps from `state` (7 float64 device tensors) with friction-law
    parameters `theta` (n_sys x 3 tensor: mu_s, mu_2, I0); differentiable
    with respect to both.  order 1: the explicit step (lp_step); order 2:
    the second-order step (lp_step2)."""
    global _FN
    if _FN is None:
        _FN = _make_function()
    if steps < 1 or checkpoint_every < 1:
        raise ValueError("steps and checkpoint_every must be positive")
    if order not in (1, 2):
        raise ValueError("order must be 1 or 2")
    return _FN.apply(ctx, list(offsets), list(params), float(dt), int(steps),
                     int(checkpoint_every), int(order), theta, *state)
