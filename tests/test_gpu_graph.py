"""Captured step sequences (lp_step_graph) against eager lp_step calls.

The captured steps decide re-sorts on the device with the same rule as
lp_step, so a replay of k steps reproduces k eager steps particle by
particle (identity tracked by the ids the graph permutes, and by composing
lp_step's permutations).  Every replay is checked, with eager work and
synchronisations between replays."""
import numpy as np
import pytest

import lpgen
from cases import CASES
from test_gpu_parity import _log, lp  # noqa: F401

pytestmark = pytest.mark.gpu


def _eager(lp, wl, steps, start, **cfg):
    """`steps` eager lp_step calls from `start`; state by original id."""
    import torch
    ctx = lp.make_context(wl, **cfg)
    st = lp.DeviceState.from_host(start)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ids = np.arange(wl.n)
    for _ in range(steps):
        ctx.lp_step(st, wl.dt, perm)
        ids = ids[perm.cpu().numpy()]
    ctx.sync_status()
    host = st.to_host()
    out = [np.empty(wl.n) for _ in range(7)]
    for a, src in zip(out, host.arrays()):
        a[ids] = src
    return lpgen.State(*out), ctx.stats()


def _by_id(st, ids):
    host = st.to_host()
    out = [np.empty(len(ids)) for _ in range(7)]
    for a, src in zip(out, host.arrays()):
        a[ids] = src
    return lpgen.State(*out)


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a.arrays(), b.arrays()))


@pytest.mark.parametrize("case,skin", [("column16_flow_ragged", 0.1),
                                       ("column16_flow_ragged", 0.002),
                                       ("ensemble_3", 0.002)])
def test_graph_replays_match_eager_steps(lp, case, skin):
    """Three replays of a 6-step graph (skin 0.002 forces re-sorts inside
    the graph) against 6, 12 and 18 eager steps."""
    import torch
    wl = CASES[case]()
    k = 6
    ctx = lp.make_context(wl, skin=skin)
    st = lp.DeviceState.from_host(wl.state)
    ids = torch.arange(wl.n, dtype=torch.int32, device="cuda")
    for rep in range(1, 4):
        ctx.lp_step_graph(st, wl.dt, k, ids)
        ctx.sync_status()
        got = _by_id(st, ids.cpu().numpy())
        stats = ctx.stats()
        want, wstats = _eager(lp, wl, k * rep, wl.state, skin=skin)
        _log("%s skin %g replay %d: graph %s / eager %s" % (case, skin, rep, stats, wstats))
        assert _same(got, want), rep
        # unrelated eager work on the same stream between replays
        junk = torch.randn(1 << 16, device="cuda", dtype=torch.float64)
        assert torch.isfinite(junk.sum()).item()
        torch.cuda.synchronize()


def test_graph_rebuilds_inside_capture(lp):
    """With a tiny skin the captured steps re-sort on the device: the ids
    stay a permutation and the device counter records the rebuilds."""
    import torch
    wl = CASES["column16_flow_ragged"]()
    ctx = lp.make_context(wl, skin=0.0005)
    st = lp.DeviceState.from_host(wl.state)
    ids = torch.arange(wl.n, dtype=torch.int32, device="cuda")
    ctx.stats()
    ctx.lp_step_graph(st, wl.dt, 8, ids)
    ctx.sync_status()
    stats = ctx.stats()
    _log("stats %s" % stats)
    assert stats["rebuilds"] >= 2
    got = np.sort(ids.cpu().numpy())
    assert np.array_equal(got, np.arange(wl.n))


def test_graph_recaptures_on_new_arguments(lp):
    """A different dt or step count captures a new graph; results still
    match eager steps."""
    import torch
    wl = CASES["column16_flow_ragged"]()
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    ids = torch.arange(wl.n, dtype=torch.int32, device="cuda")
    ctx.lp_step_graph(st, wl.dt, 3, ids)
    ctx.lp_step_graph(st, wl.dt, 2, ids)
    ctx.sync_status()
    got = _by_id(st, ids.cpu().numpy())
    want, _ = _eager(lp, wl, 5, wl.state)
    assert _same(got, want)


def test_ensemble_systems_evolve_as_if_alone(lp):
    """The 64-column ensemble of the batching benchmark (6.7M particles,
    per-column mu(I) parameters) in one context: after two steps, columns
    0, 17 and 63 equal the same columns stepped in contexts of their own,
    bit for bit (systems never interact, and each column's particles are
    ordered and computed the same way in both)."""
    import torch
    wl = lpgen.ensemble()
    _log("ensemble n=%d systems=%d" % (wl.n, len(wl.params)))
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    for _ in range(2):
        ctx.lp_step(st, wl.dt)
    ctx.sync_status()
    full = st.to_host()
    for c in (0, 17, 63):
        a, b = int(wl.offsets[c]), int(wl.offsets[c + 1])
        one = lpgen.Workload("col", wl.state.take(np.arange(a, b)),
                             np.array([0, b - a]), [wl.params[c]], wl.dt, 2)
        ctx1 = lp.make_context(one)
        s1 = lp.DeviceState.from_host(one.state)
        for _ in range(2):
            ctx1.lp_step(s1, wl.dt)
        ctx1.sync_status()
        alone = s1.to_host()
        for k, (x, y) in enumerate(zip(full.arrays(), alone.arrays())):
            assert np.array_equal(x[a:b], y), (c, k)
        _log("  column %d (%d particles): identical" % (c, b - a))


def test_graph_replay_after_a_list_without_tile_map(lp):
    """lp_build_cells between replays builds a new list without a tile map;
    the next replay (no recapture) first builds the map for it, so the
    captured staged fits read the current list: replay, re-sort, replay
    equals the same eager sequence exactly."""
    import torch
    wl = CASES["column16_flow_ragged"]()
    k = 4

    def run(graph):
        ctx = lp.make_context(wl)
        st = lp.DeviceState.from_host(wl.state)
        ids = torch.arange(wl.n, dtype=torch.int32, device="cuda")
        perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")

        def steps():
            nonlocal ids
            if graph:
                ctx.lp_step_graph(st, wl.dt, k, ids)
            else:
                for _ in range(k):
                    ctx.lp_step(st, wl.dt, perm)
                    ids = ids[perm.long()]

        steps()
        ids = ids[ctx.lp_build_cells(st).long()]
        # the new list has no tile map yet
        s = ctx.stats()
        assert s["unstaged_tiles"] == s["tiles"] > 0
        steps()
        ctx.sync_status()
        stats = ctx.stats()
        return _by_id(st, ids.cpu().numpy()), stats

    got, gstats = run(True)
    want, wstats = run(False)
    _log("graph %s / eager %s" % (gstats, wstats))
    assert gstats["unstaged_tiles"] == 0 and wstats["unstaged_tiles"] == 0
    assert _same(got, want)
