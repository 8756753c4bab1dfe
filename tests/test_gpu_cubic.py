"""GPU parity of the cubic (19-unknown) fits (fit_order = 3; a wavefront
per particle) against the oracle's cubic fits, which are pinned by exact
cubic reproduction, convergence orders and their fallbacks: derivatives
and steps within 1e-10, fallback flags exact.  Both sides use m_max = 56
(stencil plus ghost rows fill at most one wavefront)."""
import numpy as np
import pytest

import lpgen
import oracle
from cases import CASES
from test_gpu_parity import (TOL, _fields, _gpu_sorted, _incr_ok, _log, _oracle_sorted,
                             _relerr, lp)  # noqa: F401

pytestmark = pytest.mark.gpu
CUBIC = dict(fit_order=3, m_max=56)


@pytest.mark.parametrize("case", list(CASES))
def test_cubic_fit_derivs_parity(lp, case):
    import torch
    wl = CASES[case]()
    _log("case %s n=%d (cubic fits)" % (case, wl.n))
    ctx, st, _ = _gpu_sorted(lp, wl, **CUBIC)
    _, ost = _oracle_sorted(wl)
    ctx.lp_neighbors(st, candidates=False, stencils=False, ghosts=False)
    F = _fields(ost)
    ms, gz = [1, 1, -1], [0, 0, 1]
    coef, flags = ctx.lp_fit_derivs(st, torch.tensor(F, device="cuda"), ms, gz)
    ctx.sync_status()
    o = oracle.Oracle(ost, wl.offsets, wl.params, cfg=CUBIC)
    ocoef, oflags = o.fit(F, ms, gz)
    gc = coef.cpu().numpy()
    for f in range(3):
        for q in range(9):
            e = _relerr(gc[f, q], ocoef[f, q])
            assert e <= TOL, (f, q, e)
    gf = flags.cpu().numpy()
    assert np.array_equal(gf & 17, oflags & 17)
    _log("  quadratic fallbacks %d, linear %d" % (np.sum(gf & 16 != 0), np.sum(gf & 1)))


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("kind", ["step", "step2"])
def test_cubic_step_parity(lp, case, kind):
    import torch
    wl = CASES[case]()
    _log("case %s %s n=%d (cubic fits)" % (case, kind, wl.n))
    ctx = lp.make_context(wl, **CUBIC)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    (ctx.lp_step2 if kind == "step2" else ctx.lp_step)(st, wl.dt, perm)
    ctx.sync_status()
    fn = oracle.step2 if kind == "step2" else oracle.step
    want, operm, _ = fn(wl.state, wl.offsets, wl.params, wl.dt, cfg=CUBIC)
    assert np.array_equal(perm.cpu().numpy(), operm)
    old = wl.state.take(operm)
    for k, (a, b, c) in enumerate(zip(st.to_host().arrays(), want.arrays(), old.arrays())):
        ok, e = _incr_ok(a, b, c)
        assert ok, (lp.DeviceState.NAMES[k], e)


def test_cubic_rheology_rhs_parity(lp):
    """Closure and cubic P, eta fits from the oracle's cubic velocity
    derivatives; flags carry the fit's fallback bits."""
    import torch
    wl = CASES["column16_flow_ragged"]()
    ctx, st, _ = _gpu_sorted(lp, wl, **CUBIC)
    _, ost = _oracle_sorted(wl)
    ctx.lp_neighbors(st, candidates=False, stencils=False, ghosts=False)
    r = oracle.Oracle(ost, wl.offsets, wl.params, cfg=CUBIC).evaluate()
    g = ctx.lp_rheology_rhs(st, torch.tensor(r["coef_u"], device="cuda"))
    ctx.sync_status()
    for name, q in (("acc", None), ("dVdt", None), ("grad", None)):
        e = _relerr(g[name].cpu().numpy(), r[name])
        assert e <= TOL, (name, e)
    assert np.array_equal(g["flags"].cpu().numpy() & 23, r["flags"] & 23)


def test_full_size_column_cubic_step_parity(lp):
    """The 524,288-particle benchmark column, one step with cubic fits,
    every particle against the oracle."""
    import torch
    wl = lpgen.column_bench()
    _log("column_bench n=%d (cubic fits)" % wl.n)
    ctx = lp.make_context(wl, **CUBIC)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ctx.lp_step(st, wl.dt, perm)
    ctx.sync_status()
    want, operm, _ = oracle.step(wl.state, wl.offsets, wl.params, wl.dt, cfg=CUBIC,
                                 brute=False)
    assert np.array_equal(perm.cpu().numpy(), operm)
    old = wl.state.take(operm)
    for k, (a, b, c) in enumerate(zip(st.to_host().arrays(), want.arrays(), old.arrays())):
        ok, e = _incr_ok(a, b, c)
        _log("  %s increment rel err %.3e" % (lp.DeviceState.NAMES[k], e))
        assert ok


def test_cubic_configuration_errors(lp):
    wl = CASES["column16"]()
    with pytest.raises(lp.LPError) as e:
        lp.make_context(wl, fit_order=3)            # m_max 60 > 56
    assert e.value.status == 1
    ctx = lp.make_context(wl, **CUBIC)
    st = lp.DeviceState.from_host(wl.state)
    with pytest.raises(lp.LPError) as e:
        ctx.lp_step_adjoint(st, wl.dt, st)
    assert e.value.status == 1
