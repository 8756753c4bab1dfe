"""The fits with each tile's neighbours staged in LDS against the same
fits reading every neighbour from global memory (LP_DEBUG_GLOBAL_GATHER):
the rows, their order and their arithmetic are the same, so the states
agree to rounding.  Both paths are checked against the oracle elsewhere;
here the staged path is also shown to be the one taken (no unstaged
tiles), including at the full 524,288-particle column."""
import numpy as np
import pytest

import lpgen
from cases import CASES
from test_gpu_parity import _log, lp  # noqa: F401

pytestmark = pytest.mark.gpu


def _run(lp, wl, steps, order=1, **cfg):
    ctx = lp.make_context(wl, **cfg)
    st = lp.DeviceState.from_host(wl.state)
    for _ in range(steps):
        (ctx.lp_step2 if order == 2 else ctx.lp_step)(st, wl.dt)
    ctx.sync_status()
    return st.to_host(), ctx.stats()


def _compare(a, b, tag, rtol=1e-12):
    for q, (x, y) in enumerate(zip(a.arrays(), b.arrays())):
        scale = max(float(np.max(np.abs(y))), 1e-300)
        d = float(np.max(np.abs(x - y))) if x.size else 0.0
        _log("%s array %d: max |staged - global| = %.3g (scale %.3g)" % (tag, q, d, scale))
        np.testing.assert_allclose(x, y, rtol=rtol, atol=0.1 * rtol * scale,
                                   err_msg="%s %d" % (tag, q))


@pytest.mark.parametrize("case", ["column16", "column16_flow_ragged", "lattice_exact",
                                  "sheared_20x20x12", "ensemble_3", "sparse_cloud",
                                  "periodic_xy", "periodic_x"])
@pytest.mark.parametrize("order", [1, 2])
def test_staged_matches_global(lp, case, order):
    wl = CASES[case]()
    print("case", case, "order", order, "n", wl.n, flush=True)
    got, st_s = _run(lp, wl, 2, order)
    ref, st_g = _run(lp, wl, 2, order, debug_flags=lp.LP_DEBUG_GLOBAL_GATHER)
    _log("stats staged %s global %s" % (st_s, st_g))
    assert st_s["tiles"] == (wl.n + 255) // 256
    assert st_s["unstaged_tiles"] == 0
    assert st_g["unstaged_tiles"] == st_g["tiles"]
    _compare(got, ref, case)


@pytest.mark.parametrize("case", ["column16_flow_ragged", "sheared_20x20x12", "ensemble_3",
                                  "periodic_xy"])
def test_staged_matches_global_refined(lp, case):
    """The refined FP32 fits read staged rows in both sweeps (float32
    moments, float64 residuals).  The float32 sums may round differently
    where the compiler schedules the two paths differently; one float64
    correction leaves that at the square of float32 rounding, so the states
    agree to 1e-10."""
    wl = CASES[case]()
    print("case", case, "refined n", wl.n, flush=True)
    got, st_s = _run(lp, wl, 2, precision=lp.LP_FP32_REFINED)
    ref, st_g = _run(lp, wl, 2, precision=lp.LP_FP32_REFINED,
                     debug_flags=lp.LP_DEBUG_GLOBAL_GATHER)
    _log("stats staged %s global %s" % (st_s, st_g))
    assert st_s["unstaged_tiles"] == 0
    assert st_g["unstaged_tiles"] == st_g["tiles"]
    _compare(got, ref, case, rtol=1e-10)


@pytest.mark.parametrize("opt", ["wall_pressure", "wall_reflect"])
def test_staged_wall_options(lp, opt):
    """Mirror rows read the pressure a mirror carries from the staged
    copy, including the hydrostatic wall-pressure option."""
    wl = CASES["column16_flow_ragged"]()
    got, _ = _run(lp, wl, 2, **{opt: 1})
    ref, _ = _run(lp, wl, 2, debug_flags=lp.LP_DEBUG_GLOBAL_GATHER, **{opt: 1})
    _compare(got, ref, opt)


def test_staged_full_column(lp):
    """One step of the 64 x 64 x 128 column (524,288 particles): all but a
    few tiles (at most 1 %, those with more than 1664 distinct list
    sources) are staged, and the state agrees with the global-gather
    step's to rounding."""
    wl = lpgen.column_bench()
    print("case column_bench n", wl.n, flush=True)
    got, st_s = _run(lp, wl, 1)
    ref, st_g = _run(lp, wl, 1, debug_flags=lp.LP_DEBUG_GLOBAL_GATHER)
    _log("stats staged %s" % st_s)
    assert st_s["tiles"] == 2048 and st_s["unstaged_tiles"] <= 20
    _compare(got, ref, "column_bench")


def test_mixed_staged_tiles(lp):
    """A 24^3 column with h = 1.25 lattice spacings (about 145 list entries
    per particle): some inner tiles have more than 1664 distinct list
    sources and are not staged, the others are.  In one launch both kinds
    match the global-gather step to rounding, and the step matches the
    oracle's."""
    import dataclasses

    import oracle
    import torch
    from test_gpu_parity import _incr_ok

    wl = lpgen.column_bench(nx=24, ny=24, nz=24)
    h = wl.params[0].h * 1.25
    wl.params = [dataclasses.replace(p, h=h, R=2.5 * h) for p in wl.params]
    print("case column 24^3, h x1.25, n", wl.n, flush=True)
    got, st_s = _run(lp, wl, 1)
    ref, _ = _run(lp, wl, 1, debug_flags=lp.LP_DEBUG_GLOBAL_GATHER)
    _log("stats %s" % st_s)
    assert 0 < st_s["unstaged_tiles"] < st_s["tiles"]
    _compare(got, ref, "mixed")
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ctx.lp_step(st, wl.dt, perm)
    ctx.sync_status()
    ost, operm, _ = oracle.step(wl.state, wl.offsets, wl.params, wl.dt)
    assert np.array_equal(perm.cpu().numpy(), operm)
    old = wl.state.take(operm)
    for k, (a, b, c) in enumerate(zip(st.to_host().arrays(), ost.arrays(), old.arrays())):
        ok, e = _incr_ok(a, b, c)
        assert ok, (lp.DeviceState.NAMES[k], e)
