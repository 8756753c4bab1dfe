"""GPU parity of the refined-FP32 mode (precision LP_FP32_REFINED): float32
Gram factor, one float64 residual correction per fit, float64 Householder
refit above the condition threshold.  The target is the same FP64 oracle;
every state array must agree within 1e-5 of the oracle's increment (the
achieved error is printed per array)."""
import numpy as np
import pytest

import lpgen
import oracle
from cases import CASES
from test_gpu_parity import (_incr_ok, _log, _relerr, _trajectory_gpu,
                             _trajectory_oracle, lp)  # noqa: F401

pytestmark = pytest.mark.gpu
TOL_REFINED = 1e-5


def _step_check(lp, wl, tol, **cfg):
    import torch
    ctx = lp.make_context(wl, precision=lp.LP_FP32_REFINED, **cfg)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ctx.lp_step(st, wl.dt, perm)
    ctx.sync_status()
    _log("stats %s" % ctx.stats())
    ost, operm, _ = oracle.step(wl.state, wl.offsets, wl.params, wl.dt,
                                brute=wl.n <= 20000)
    assert np.array_equal(perm.cpu().numpy(), operm)
    old = wl.state.take(operm)
    worst = 0.0
    for k, (a, b, c) in enumerate(zip(st.to_host().arrays(), ost.arrays(),
                                      old.arrays())):
        ok, e = _incr_ok(a, b, c, tol=tol)
        _log("  %s increment rel err %.3e" % (lp.DeviceState.NAMES[k], e))
        worst = max(worst, e)
        assert ok, (lp.DeviceState.NAMES[k], e)
    return worst


@pytest.mark.parametrize("case", list(CASES))
def test_refined_step_parity(lp, case):
    wl = CASES[case]()
    _log("case %s n=%d (refined fp32)" % (case, wl.n))
    _step_check(lp, wl, TOL_REFINED)


def test_refined_full_size_column(lp):
    """The 524,288-particle benchmark column in refined mode."""
    wl = lpgen.column_bench()
    _log("column_bench n=%d (refined fp32)" % wl.n)
    _step_check(lp, wl, TOL_REFINED)


def test_refined_threshold_sends_every_stencil_to_fp64(lp):
    """With the condition threshold at its minimum every stencil is refitted
    by float64 Householder QR, so the result meets the FP64 bar."""
    wl = CASES["sheared_20x20x12"]()
    _log("sheared, refined with cond_max -> 1 (all stencils FP64)")
    _step_check(lp, wl, 1e-10, cond_max=1.0 + 1e-12)


def test_refined_trajectory(lp):
    """Five refined steps with the list reused, particle by particle against
    the oracle trajectory."""
    wl = CASES["sheared_20x20x12"]()
    got, stats = _trajectory_gpu(lp, wl, 5, precision=lp.LP_FP32_REFINED)
    _log("stats %s" % stats)
    want = _trajectory_oracle(wl, 5)
    for k, (a, b, c) in enumerate(zip(got.arrays(), want.arrays(),
                                      wl.state.arrays())):
        ok, e = _incr_ok(a, b, c, tol=TOL_REFINED, ulps=64)
        _log("  %s increment rel err %.3e" % (lp.DeviceState.NAMES[k], e))
        assert ok, (lp.DeviceState.NAMES[k], e)


def test_refined_matches_fp64_path_closely(lp):
    """Refined and FP64 GPU steps agree far inside the refined tolerance on
    a smooth flow (the correction step recovers near-FP64 accuracy)."""
    import torch
    wl = CASES["column16_flow_ragged"]()
    out = []
    for prec in (lp.LP_FP64, lp.LP_FP32_REFINED):
        ctx = lp.make_context(wl, precision=prec)
        st = lp.DeviceState.from_host(wl.state)
        ctx.lp_step(st, wl.dt, torch.empty(wl.n, dtype=torch.int32, device="cuda"))
        ctx.sync_status()
        out.append(st.to_host())
    for k, (a, b) in enumerate(zip(out[1].arrays(), out[0].arrays())):
        e = _relerr(a, b)
        _log("  %s refined vs fp64 rel err %.3e" % (lp.DeviceState.NAMES[k], e))
        assert e <= 1e-9
