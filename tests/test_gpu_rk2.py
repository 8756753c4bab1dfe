"""GPU parity of the second-order step lp_step2 (Heun's method on the
right-hand side of Sec. 2.1) against oracle.step2, itself pinned by its
temporal order and by exact free fall: permutation exact, increments of
position, velocity and volume within 1e-10 of the oracle's."""
import numpy as np
import pytest

import lpgen
import oracle
from cases import CASES
from test_gpu_parity import TOL, _incr_ok, _log, _relerr, lp  # noqa: F401

pytestmark = pytest.mark.gpu


def _check(lp, got, want, old, tol=TOL):
    for k, (a, b, c) in enumerate(zip(got.arrays(), want.arrays(), old.arrays())):
        ok, e = _incr_ok(a, b, c, tol=tol)
        _log("  %s increment rel err %.3e" % (lp.DeviceState.NAMES[k], e))
        assert ok, (lp.DeviceState.NAMES[k], e)


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("path", ["gram", "qr"])
def test_step2_parity(lp, case, path):
    import torch
    wl = CASES[case]()
    _log("case %s path %s n=%d (second-order step)" % (case, path, wl.n))
    cfg = {} if path == "gram" else dict(debug_flags=lp.LP_DEBUG_QR_FIT)
    ctx = lp.make_context(wl, **cfg)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ctx.lp_step2(st, wl.dt, perm)
    ctx.sync_status()
    want, operm, _ = oracle.step2(wl.state, wl.offsets, wl.params, wl.dt)
    assert np.array_equal(perm.cpu().numpy(), operm)
    _check(lp, st.to_host(), want, wl.state.take(operm))


def test_step2_and_step_alternate_on_one_state(lp):
    """lp_step2, lp_step, lp_step2 on one state without a re-sort (one list
    build): each result against the oracle's step of the same kind applied
    to the oracle's previous result."""
    import torch
    wl = CASES["column16_flow_ragged"]()
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ctx.stats()
    ref, sort = wl.state, True
    for kind in ("step2", "step", "step2"):
        old = ref
        if kind == "step2":
            ctx.lp_step2(st, wl.dt, perm)
            ref, operm, _ = oracle.step2(ref, wl.offsets, wl.params, wl.dt, sort=sort)
        else:
            ctx.lp_step(st, wl.dt, perm)
            ref, operm, _ = oracle.step(ref, wl.offsets, wl.params, wl.dt, sort=sort)
        ctx.sync_status()
        assert np.array_equal(perm.cpu().numpy(), operm), kind
        _log("%s:" % kind)
        _check(lp, st.to_host(), ref, old.take(operm))
        sort = False
    assert ctx.stats()["rebuilds"] == 1


def test_step2_rebuilds_inside_a_run(lp):
    """A skin of 30 dt max|u| / R: the second-order step re-sorts once some
    particle has moved 0.4 of the skin (12 steps of the fastest particle),
    which leaves the predictor 3 steps of room; over 30 steps the list is
    rebuilt at least once after the first build, no predictor leaves it,
    and every step matches the oracle (which re-sorts when the GPU did)."""
    import torch
    wl = CASES["column16_flow_ragged"]()
    p = wl.params[0]
    vmax = float(np.max(np.sqrt(wl.state.u ** 2 + wl.state.v ** 2 + wl.state.w ** 2)))
    skin = 30.0 * wl.dt * vmax / p.R
    _log("skin %.4g" % skin)
    ctx = lp.make_context(wl, skin=skin)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ctx.stats()
    ref = wl.state
    rebuilds = 0
    for step in range(30):
        ctx.lp_step2(st, wl.dt, perm)
        ctx.sync_status()
        sorted_now = ctx.stats()["rebuilds"] > 0
        rebuilds += int(sorted_now)
        old = ref
        ref, operm, _ = oracle.step2(ref, wl.offsets, wl.params, wl.dt, skin=skin,
                                     sort=sorted_now)
        assert np.array_equal(perm.cpu().numpy(), operm), step
        if sorted_now or step % 10 == 9:
            _log("step %d%s:" % (step, " (re-sorted)" if sorted_now else ""))
            _check(lp, st.to_host(), ref, old.take(operm))
    _log("rebuilds %d" % rebuilds)
    assert rebuilds >= 2


def test_predictor_outside_the_list_is_reported(lp):
    """A step so long that the predictor moves some particle more than half
    the skin latches an error that lp_sync_status reports as LP_E_STATE;
    every kernel stays within its buffers (the stencils are still selected
    from the list) and the context keeps working."""
    wl = CASES["column16_flow_ragged"]()
    p = wl.params[0]
    speed = np.sqrt(wl.state.u ** 2 + wl.state.v ** 2 + wl.state.w ** 2)
    dt = 0.75 * 0.1 * p.R / float(np.max(speed))    # 0.75 of the skin
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    ctx.lp_step2(st, dt)
    with pytest.raises(lp.LPError) as e:
        ctx.sync_status()
    assert e.value.status == 5
    assert "skin" in str(e.value)
    st = lp.DeviceState.from_host(wl.state)
    ctx.lp_build_cells(st, want_perm=False)
    ctx.lp_step2(st, wl.dt)
    ctx.sync_status()


def test_step2_needs_a_skin(lp):
    wl = CASES["column16"]()
    ctx = lp.make_context(wl, skin=0.0)
    st = lp.DeviceState.from_host(wl.state)
    with pytest.raises(lp.LPError) as e:
        ctx.lp_step2(st, wl.dt)
    assert e.value.status == 1
    with pytest.raises(lp.LPError) as e:
        lp.make_context(wl).lp_step2(st, 0.0)
    assert e.value.status == 1


def test_full_size_column_step2_parity(lp):
    """The 64 x 64 x 128 benchmark column (524,288 particles): one
    second-order step, every particle against the oracle."""
    import torch
    wl = lpgen.column_bench()
    _log("column_bench n=%d (second-order step)" % wl.n)
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ctx.lp_step2(st, wl.dt, perm)
    ctx.sync_status()
    want, operm, _ = oracle.step2(wl.state, wl.offsets, wl.params, wl.dt, brute=False)
    assert np.array_equal(perm.cpu().numpy(), operm)
    old = wl.state.take(operm)
    _check(lp, st.to_host(), want, old)
    for k, (a, b) in enumerate(zip(st.to_host().arrays(), want.arrays())):
        assert _relerr(a, b) <= TOL, lp.DeviceState.NAMES[k]
