"""Batching of uneven stencils by size class (rows, ghosts included: at
most 16, at most 32, more), each class dispatched with its own lanes per
particle: steps of both kinds and the second-order adjoint with the class
dispatch forced (LP_DEBUG_CLASSES: lanes 1, 2, 4) against the oracle on
every case; the autotuned plan on uneven stencils, its class counts
against the exported stencils (exact), and steps with it against the
oracle."""
import numpy as np
import pytest

import oracle
from cases import CASES
from oracle import adjoint
from test_gpu_parity import _incr_ok, _log, _relerr, lp  # noqa: F401

pytestmark = pytest.mark.gpu


def _step_check(lp, wl, ctx, kind):
    import torch
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    (ctx.lp_step2 if kind == "step2" else ctx.lp_step)(st, wl.dt, perm)
    ctx.sync_status()
    fn = oracle.step2 if kind == "step2" else oracle.step
    want, operm, _ = fn(wl.state, wl.offsets, wl.params, wl.dt)
    assert np.array_equal(perm.cpu().numpy(), operm)
    old = wl.state.take(operm)
    for k, (a, b, c) in enumerate(zip(st.to_host().arrays(), want.arrays(), old.arrays())):
        ok, e = _incr_ok(a, b, c)
        assert ok, (lp.DeviceState.NAMES[k], e)


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("kind", ["step", "step2"])
def test_class_dispatch_step_parity(lp, case, kind):
    wl = CASES[case]()
    _log("case %s %s n=%d (size classes forced)" % (case, kind, wl.n))
    ctx = lp.make_context(wl, debug_flags=lp.LP_DEBUG_CLASSES)
    assert ctx.lp_fit_plan()["size_classes"]
    _step_check(lp, wl, ctx, kind)


@pytest.mark.parametrize("case", ["sparse_cloud", "sheared_20x20x12", "column16_flow_ragged"])
def test_class_dispatch_step2_adjoint_parity(lp, case):
    import torch

    from test_gpu_adjoint import _dev, _lam
    wl = CASES[case]()
    lam = _lam(wl, 53)
    want, wth, operm = adjoint.step2_vjp(wl.state, wl.offsets, wl.params, wl.dt, lam)
    ctx = lp.make_context(wl, debug_flags=lp.LP_DEBUG_CLASSES)
    st = lp.DeviceState.from_host(wl.state)
    dth = torch.zeros(len(wl.params), 3, dtype=torch.float64, device="cuda")
    got, perm = ctx.lp_step2_adjoint(st, wl.dt, _dev(lam), dth, want_perm=True)
    ctx.sync_status()
    assert np.array_equal(perm.cpu().numpy(), operm)
    for k, (a, b) in enumerate(zip(got.to_host().arrays(), want)):
        assert _relerr(a, b) <= 1e-10, lp.DeviceState.NAMES[k]


@pytest.mark.parametrize("case", ["sparse_cloud", "sheared_20x20x12", "column16"])
def test_autotuned_plan_and_class_counts(lp, case):
    import torch
    wl = CASES[case]()
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    ctx.lp_autotune(st)
    plan = ctx.lp_fit_plan()
    _log("case %s plan %s" % (case, plan))
    assert sum(plan["class_particles"]) == wl.n
    for key in ("class_lanes_pass1", "class_lanes_pass2"):
        assert all(x in (1, 2, 4) for x in plan[key])
    # class counts from the exported stencils of the same state (the
    # autotune sorts a copy as lp_build_cells does)
    chk = lp.make_context(wl)
    s2 = lp.DeviceState.from_host(wl.state)
    chk.lp_build_cells(s2, want_perm=False)
    nb = chk.lp_neighbors(s2, candidates=False)
    rows = nb["sten_cnt"].to(torch.int64) + torch.stack(
        [(nb["ghost_mask"].to(torch.int64) >> o) & 1 for o in range(8)]).sum(0)
    want = [int((rows <= 16).sum()), int(((rows > 16) & (rows <= 32)).sum()),
            int((rows > 32).sum())]
    assert plan["class_particles"] == want
    # steps with the chosen plan
    _step_check(lp, wl, ctx, "step")
