"""Gradients through LP trajectories with torch.autograd.

``simulate`` runs ``steps`` LP steps (lp_step, or lp_step2 for the
second-order step) and returns the final state as torch tensors that take
part in autograd.  The first step of every checkpointed segment re-sorts the
state and rebuilds the neighbour list (a forced re-sort of the step
record); the other steps re-sort only when the list's skin runs out, as
plain lp_step calls do.  Only the state at the start of each segment is
kept during the forward pass.  The backward pass recomputes a segment from
its checkpoint with step records (which reproduces the forward steps
exactly: the steps, the re-sorts and the lists are deterministic) and runs
the library's lp_step_adjoint (or lp_step2_adjoint) on each recorded step
in reverse, reusing that step's neighbour list.  A segment whose steps span
two lists (a re-sort inside it) is recomputed once more for the part before
the re-sort.

Gradients flow to the initial state (x, y, z, u, v, w, V) and to the
friction-law parameters theta = (mu_s, mu_2, I0) of every system.  The
backward pass sets the context's systems to those of its forward pass (and
restores the previous ones afterwards), so other runs on the same context
in between do not change it.  All arithmetic runs in the HIP library; this
module only sequences calls.
"""
from __future__ import annotations

import dataclasses
from typing import Sequence

from . import Context, DeviceState, StepRecord


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
            run_params = _params_with(params, theta.detach().cpu().tolist())
            ctx.set_systems(offsets, run_params)
            st = DeviceState([a.detach().clone() for a in state])
            step = ctx.lp_step2 if order == 2 else ctx.lp_step
            rec = StepRecord(st.n)
            ckpts = {}
            for k in range(steps):
                if k % every == 0:
                    ckpts[k] = st.clone()
                rec.s.force_sort = 1 if k % every == 0 else 0
                step(st, dt, rec=rec)
            fctx.lp = (ctx, list(offsets), run_params, dt, steps, every, order, ckpts,
                       theta.device, theta.dtype)
            return tuple(st.t)

        @staticmethod
        def backward(fctx, *gout):
            (ctx, offsets, run_params, dt, steps, every, order, ckpts, tdev,
             tdt) = fctx.lp
            step = ctx.lp_step2 if order == 2 else ctx.lp_step
            adjoint = ctx.lp_step2_adjoint if order == 2 else ctx.lp_step_adjoint
            ref = next(iter(ckpts.values())).t[0]
            lam = DeviceState([torch.zeros_like(ref) if g is None else
                               g.detach().to(torch.float64).contiguous()
                               for g in gout])
            dtheta = torch.zeros(len(run_params), 3, dtype=torch.float64,
                                 device=ref.device)
            saved = (getattr(ctx, "offsets", None), getattr(ctx, "params", None))
            ctx.set_systems(offsets, run_params)
            try:
                for k0 in sorted(ckpts, reverse=True):
                    end = min(k0 + every, steps)
                    while end > k0:
                        # recompute [k0, end) with records; the steps from
                        # the last re-sort on share the context's current
                        # list, so their adjoints run now
                        st = ckpts[k0].clone()
                        inputs, recs = [], []
                        for k in range(k0, end):
                            inputs.append(st.clone())
                            rec = StepRecord(st.n, force_sort=(k == k0))
                            step(st, dt, rec=rec)
                            recs.append(rec)
                        start = k0
                        for k in range(end - 1, k0, -1):
                            if recs[k - k0].resorted:
                                start = k
                                break
                        for k in range(end - 1, start - 1, -1):
                            lam = adjoint(inputs[k - k0], dt, lam, dtheta,
                                          rec=recs[k - k0])
                        end = start
            finally:
                if saved[0] is not None:
                    ctx.set_systems(saved[0], saved[1])
            fctx.lp = None
            return (None, None, None, None, None, None, None,
                    dtheta.to(device=tdev, dtype=tdt)) + tuple(lam.t)

    return _Trajectory


_FN = None


def simulate(ctx: Context, offsets, params: Sequence, state: Sequence, theta, dt: float,
             steps: int, checkpoint_every: int = 10, order: int = 1):
    """Final state (7 tensors, in the order of the last step) of `steps`
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
