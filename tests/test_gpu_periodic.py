"""Periodic boundaries on the GPU (Sec. 3.1, boundary conditions) against
the oracle, which is pinned against explicit copies of the box: particles
drifting through the periodic faces over several steps with re-sorts,
captured step sequences, and the error for positions beyond one period."""
import numpy as np
import pytest

import oracle
from cases import CASES
from test_gpu_parity import _incr_ok, _log, lp  # noqa: F401

pytestmark = pytest.mark.gpu


def _drifting(case, drift=(2.0, -1.5)):
    """The case moved by (0.47 h, -0.47 h) (wrapped into the box, so that
    rows of particles sit at the faces) and given a uniform drift."""
    wl = CASES[case]()
    h = wl.params[0].h
    wl.state.x = wl.state.x + 0.47 * h
    wl.state.y = wl.state.y - 0.47 * h
    oracle.wrap(wl.state, wl.offsets, wl.params)
    wl.state.u = wl.state.u + drift[0]
    wl.state.v = wl.state.v + drift[1]
    wl.dt = 1e-3
    return wl


@pytest.mark.parametrize("case", ["periodic_xy", "periodic_x"])
@pytest.mark.parametrize("kind", ["step", "step2"])
def test_drift_through_periodic_faces(lp, case, kind):
    """Fourteen steps of 1 ms with a uniform drift of (2, -1.5) m/s
    (skin 0.3, so that the second-order predictor stays inside the list):
    particles leave through one face and re-enter through the opposite
    one, and the list is rebuilt on the way; every step matches the
    oracle's (which re-sorts when the GPU did) and positions stay in the
    box."""
    import torch
    wl = _drifting(case)
    p = wl.params[0]
    skin = 0.3
    ctx = lp.make_context(wl, skin=skin)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ctx.stats()
    ref, wraps, rebuilds = wl.state, 0, 0
    for k in range(14):
        (ctx.lp_step2 if kind == "step2" else ctx.lp_step)(st, wl.dt, perm)
        ctx.sync_status()
        sorted_now = ctx.stats()["rebuilds"] > 0
        rebuilds += int(sorted_now)
        fn = oracle.step2 if kind == "step2" else oracle.step
        old = ref
        ref, operm, _ = fn(ref, wl.offsets, wl.params, wl.dt, skin=skin, sort=sorted_now)
        assert np.array_equal(perm.cpu().numpy(), operm), k
        got = st.to_host()
        prev = old.take(operm)
        wraps += int(np.sum(np.abs(got.x - prev.x) > 0.5 * p.box_len[0]))
        for a, (x, y, z) in enumerate(zip(got.arrays(), ref.arrays(), prev.arrays())):
            if a < 2 and p.box_len[a] > 0:
                # compare increments through the nearest copy
                L = p.box_len[a]
                x = np.where(x - z > L / 2, x - L, np.where(x - z < -L / 2, x + L, x))
                y = np.where(y - z > L / 2, y - L, np.where(y - z < -L / 2, y + L, y))
            ok, e = _incr_ok(x, y, z)
            assert ok, (k, lp.DeviceState.NAMES[a], e)
        for a in range(2):
            if p.box_len[a] > 0:
                c = got.arrays()[a]
                assert np.all((c >= p.box_lo[a]) & (c < p.box_lo[a] + p.box_len[a]))
    _log("%s %s: %d face crossings, %d list builds" % (case, kind, wraps, rebuilds))
    assert wraps > 0 and rebuilds >= 2


def test_periodic_graph_replays_match_eager_steps(lp):
    """Captured steps on the drifting periodic layer (wraps and re-sorts
    inside the graph) equal eager steps bit for bit, particle by id."""
    import torch
    from test_gpu_graph import _by_id, _eager, _same
    wl = _drifting("periodic_xy")
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    ids = torch.arange(wl.n, dtype=torch.int32, device="cuda")
    for rep in range(1, 3):
        ctx.lp_step_graph(st, wl.dt, 5, ids)
        ctx.sync_status()
        got = _by_id(st, ids.cpu().numpy())
        want, wstats = _eager(lp, wl, 5 * rep, wl.state)
        _log("replay %d: eager stats %s" % (rep, wstats))
        assert _same(got, want), rep
        torch.cuda.synchronize()


def test_position_beyond_one_period_is_reported(lp):
    wl = CASES["periodic_xy"]()
    p = wl.params[0]
    st0 = wl.state.copy()
    st0.x[5] = p.box_lo[0] + 2.5 * p.box_len[0]
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(st0)
    ctx.lp_build_cells(st, want_perm=False)
    with pytest.raises(lp.LPError) as e:
        ctx.sync_status()
    assert e.value.status == 1 and "periodic" in str(e.value)


def test_too_short_period_is_rejected(lp):
    import dataclasses
    wl = CASES["periodic_xy"]()
    p = wl.params[0]
    bad = dataclasses.replace(p, box_len=(2.0 * p.R, p.box_len[1]))
    ctx = lp.Context()
    ctx.reserve(wl.n)
    with pytest.raises(lp.LPError) as e:
        ctx.set_systems(list(wl.offsets), [bad])
    assert e.value.status == 1
