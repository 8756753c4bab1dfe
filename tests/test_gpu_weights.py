"""GPU parity of the Gaussian-weighted fits (LP_W_GAUSS: the weighted
least-squares fit of Sec. 3.1 step 7 with w = exp(-4 r^2 / R^2) per stencil
row and exp(-12 h^2 / R^2) per ghost row) against the oracle with the same
weights, on every parity case: lp_fit_derivs with both fit paths (normal
equations and forced Householder refits, flags exact), lp_rheology_rhs, and
lp_step with 1, 2 and 4 lanes per particle, refined FP32 and cubic fits.  Bars as in
the unit-weight parity tests (1e-10 FP64, 1e-5 refined FP32)."""
import sys

import numpy as np
import pytest

import lpgen
import oracle
from cases import CASES

pytestmark = pytest.mark.gpu
TOL = 1e-10
GAUSS = dict(weight=1)


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2206_14061_amd as lp_mod
    lp_mod._lib.load()
    return lp_mod


def _relerr(a, b):
    sc = np.max(np.abs(b)) if b.size else 0.0
    d = np.max(np.abs(a - b)) if b.size else 0.0
    return d / sc if sc > 0 else d


def _incr_ok(new, want, old, tol=TOL, ulps=8):
    if want.size == 0:
        return True, 0.0
    d = np.max(np.abs(new - want))
    inc = np.max(np.abs(want - old))
    floor = ulps * np.spacing(np.max(np.abs(old)) + np.max(np.abs(want)))
    return d <= tol * inc + floor, d / inc if inc > 0 else d


def _sorted(lp, wl, **cfg):
    ctx = lp.make_context(wl, weight=lp.LP_W_GAUSS, **cfg)
    st = lp.DeviceState.from_host(wl.state)
    ctx.lp_build_cells(st, want_perm=False)
    perm, _ = oracle.sort_perm(wl.state, wl.offsets, wl.params)
    ost = wl.state.take(perm)
    ost = lpgen.State(*[np.ascontiguousarray(a) for a in ost.arrays()])
    return ctx, st, ost


def _fields(st):
    x, y, z = st.x, st.y, st.z
    return np.stack([np.sin(3.0 * x + 1.0) * np.cos(2.0 * y) + z * z,
                     np.exp(0.5 * x) * np.sin(2.5 * z) - 0.3 * y,
                     np.cos(1.7 * x * y + z)])


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("path", ["gram", "qr"])
def test_weighted_fit_derivs_parity(lp, case, path):
    import torch
    wl = CASES[case]()
    _log("gauss fit case %s path %s n=%d" % (case, path, wl.n))
    cfg = {} if path == "gram" else dict(debug_flags=lp.LP_DEBUG_QR_FIT)
    ctx, st, ost = _sorted(lp, wl, **cfg)
    ctx.lp_neighbors(st, candidates=False, stencils=False, ghosts=False)
    F = _fields(ost)
    ms, gz = [1, 1, -1], [0, 0, 1]
    coef, flags = ctx.lp_fit_derivs(st, torch.tensor(F, device="cuda"), ms, gz)
    ctx.sync_status()
    ocoef, oflags = oracle.Oracle(ost, wl.offsets, wl.params, GAUSS).fit(F, ms, gz)
    # the weights act: the unit-weight fit differs
    ucoef, _ = oracle.Oracle(ost, wl.offsets, wl.params).fit(F, ms, gz)
    assert _relerr(ucoef, ocoef) > 1e-6
    gc = coef.cpu().numpy()
    for f in range(3):
        for q in range(9):
            e = _relerr(gc[f, q], ocoef[f, q])
            assert e <= TOL, (f, q, e)
    assert np.array_equal(flags.cpu().numpy() & 1, oflags & 1)


@pytest.mark.parametrize("case", list(CASES))
def test_weighted_rheology_rhs_parity(lp, case):
    import torch
    wl = CASES[case]()
    _log("gauss rhs case %s n=%d" % (case, wl.n))
    ctx, st, ost = _sorted(lp, wl)
    ctx.lp_neighbors(st, candidates=False, stencils=False, ghosts=False)
    r = oracle.Oracle(ost, wl.offsets, wl.params, GAUSS).evaluate()
    g = ctx.lp_rheology_rhs(st, torch.tensor(r["coef_u"].reshape(27, -1), device="cuda"))
    ctx.sync_status()
    for name in ("dVdt", "acc", "diag", "grad"):
        got, want = g[name].cpu().numpy(), r[name]
        for q in range(want.shape[0] if want.ndim == 2 else 1):
            a = got[q] if want.ndim == 2 else got
            b = want[q] if want.ndim == 2 else want
            assert _relerr(a, b) <= TOL, (name, q)
    assert np.array_equal(g["flags"].cpu().numpy() & 7, r["flags"] & 7)


# path: (bar, GPU options, oracle options beyond the weights)
_PATHS = {"gram": (TOL, {}, {}), "qr": (TOL, dict(debug_flags=2), {}),
          "lanes2": (TOL, dict(debug_flags=4), {}), "lanes4": (TOL, dict(debug_flags=8), {}),
          "refined": (1e-5, dict(precision=1), {}),
          "cubic": (TOL, dict(fit_order=3, m_max=56), dict(fit_order=3, m_max=56))}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("path", list(_PATHS))
def test_weighted_step_parity(lp, case, path):
    import torch
    wl = CASES[case]()
    _log("gauss step case %s path %s n=%d" % (case, path, wl.n))
    tol, cfg, ocfg = _PATHS[path]
    ctx = lp.make_context(wl, weight=lp.LP_W_GAUSS, **cfg)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ctx.lp_step(st, wl.dt, perm)
    ctx.sync_status()
    ost, operm, _ = oracle.step(wl.state, wl.offsets, wl.params, wl.dt,
                                cfg=dict(GAUSS, **ocfg))
    assert np.array_equal(perm.cpu().numpy(), operm)
    old = wl.state.take(operm)
    for k, (a, b, c) in enumerate(zip(st.to_host().arrays(), ost.arrays(), old.arrays())):
        ok, e = _incr_ok(a, b, c, tol=tol)
        assert ok, (lp.DeviceState.NAMES[k], e)


def test_weighted_step_parity_full_column(lp):
    """The 524,288-particle column, one weighted step, every particle."""
    import torch
    wl = lpgen.column_bench()
    _log("gauss step column_bench n=%d" % wl.n)
    ctx = lp.make_context(wl, weight=lp.LP_W_GAUSS)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ctx.lp_step(st, wl.dt, perm)
    ctx.sync_status()
    ost, operm, _ = oracle.step(wl.state, wl.offsets, wl.params, wl.dt, cfg=GAUSS,
                                brute=False)
    assert np.array_equal(perm.cpu().numpy(), operm)
    old = wl.state.take(operm)
    for k, (a, b, c) in enumerate(zip(st.to_host().arrays(), ost.arrays(), old.arrays())):
        ok, e = _incr_ok(a, b, c)
        assert ok, (lp.DeviceState.NAMES[k], e)
