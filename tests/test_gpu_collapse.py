"""GPU parity of the options the column-collapse runs use (the paper's
Sec. 4.2.1 test): min_real_rows (a stencil with fewer real rows than 9
takes the linear fit) on every parity case for both step kinds, and a few
steps of the a = 0.6 cylinder itself (120,631 particles) with the
reflecting wall, the hydrostatic mirror pressure, a fallback tolerance of
5e-2 and min_real_rows 9, against the oracle with the same options."""
import numpy as np
import pytest

import lpgen
import oracle
from cases import CASES
from test_gpu_parity import _incr_ok, _log, lp  # noqa: F401

pytestmark = pytest.mark.gpu
COLLAPSE = dict(wall_reflect=1, wall_pressure=1, fallback_tol=5e-2, min_real_rows=9)


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("kind", ["step", "step2"])
def test_min_real_rows_step_parity(lp, case, kind):
    import torch
    wl = CASES[case]()
    _log("case %s %s n=%d (min_real_rows 9)" % (case, kind, wl.n))
    ctx = lp.make_context(wl, min_real_rows=9)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    (ctx.lp_step2 if kind == "step2" else ctx.lp_step)(st, wl.dt, perm)
    ctx.sync_status()
    fn = oracle.step2 if kind == "step2" else oracle.step
    want, operm, _ = fn(wl.state, wl.offsets, wl.params, wl.dt, cfg=dict(min_real_rows=9))
    assert np.array_equal(perm.cpu().numpy(), operm)
    old = wl.state.take(operm)
    for k, (a, b, c) in enumerate(zip(st.to_host().arrays(), want.arrays(), old.arrays())):
        ok, e = _incr_ok(a, b, c)
        assert ok, (lp.DeviceState.NAMES[k], e)


@pytest.mark.parametrize("case", ["sparse_cloud", "column16_flow_ragged"])
def test_min_real_rows_fit_flags_exact(lp, case):
    """lp_fit_derivs with min_real_rows 9 on both fit paths: flags exact,
    coefficients within 1e-10."""
    import torch
    from test_gpu_parity import _fields, _gpu_sorted, _oracle_sorted, _relerr
    wl = CASES[case]()
    for cfg in ({}, dict(debug_flags=lp.LP_DEBUG_QR_FIT)):
        ctx, st, _ = _gpu_sorted(lp, wl, min_real_rows=9, **cfg)
        _, ost = _oracle_sorted(wl)
        ctx.lp_neighbors(st, candidates=False, stencils=False, ghosts=False)
        F = _fields(ost)
        coef, flags = ctx.lp_fit_derivs(st, torch.tensor(F, device="cuda"), [1, 1, -1],
                                        [0, 0, 1])
        ctx.sync_status()
        ocoef, oflags = oracle.Oracle(ost, wl.offsets, wl.params,
                                      dict(min_real_rows=9)).fit(F, [1, 1, -1], [0, 0, 1])
        assert np.array_equal(flags.cpu().numpy() & 1, oflags & 1)
        gc = coef.cpu().numpy()
        for f in range(3):
            for q in range(9):
                assert _relerr(gc[f, q], ocoef[f, q]) <= 1e-10, (f, q)


@pytest.mark.parametrize("kind", ["step", "step2"])
def test_collapse_configuration_steps(lp, kind):
    """Three steps of the a = 0.6 cylinder with the collapse options,
    particle by particle against the oracle (permutations composed)."""
    import torch
    wl = lpgen.column_cylinder()
    _log("cylinder n=%d dt=%.3e %s" % (wl.n, wl.dt, kind))
    ctx = lp.make_context(wl, **COLLAPSE)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ids = np.arange(wl.n)
    ost = wl.state
    oids = np.arange(wl.n)
    fn = oracle.step2 if kind == "step2" else oracle.step
    step = ctx.lp_step2 if kind == "step2" else ctx.lp_step
    for k in range(3):
        old = ost
        step(st, wl.dt, perm)
        ctx.sync_status()
        ids = ids[perm.cpu().numpy()]
        ost, operm, _ = fn(ost, wl.offsets, wl.params, wl.dt, cfg=COLLAPSE, brute=False)
        oids = oids[operm]
        old = old.take(operm)
        # compare by particle identity
        g = st.to_host()
        pos = np.empty(wl.n, dtype=np.int64)
        pos[ids] = np.arange(wl.n)
        for q, (a, b, c) in enumerate(zip(g.arrays(), ost.arrays(), old.arrays())):
            a_by_id = a[pos[oids]]
            ok, e = _incr_ok(a_by_id, b, c)
            _log("  step %d %s rel %.3e" % (k, lp.DeviceState.NAMES[q], e))
            assert ok, (k, lp.DeviceState.NAMES[q], e)
