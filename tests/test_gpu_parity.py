"""GPU parity: every entry point of the HIP library against the FP64 CPU
oracle on identical seeded inputs.

Integer results (permutation, candidate sets, stencil sets, ghost masks,
fallback and branch flags) must match bit for bit.  Floating-point arrays
must satisfy ||gpu - oracle||_inf <= 1e-10 ||oracle||_inf per array (FP64
mode).  Inputs come from lpgen or from the oracle, never from the GPU.
"""
import sys

import numpy as np
import pytest

import lpgen
import oracle
from cases import CASES

pytestmark = pytest.mark.gpu
TOL = 1e-10


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
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    sc = np.max(np.abs(b)) if b.size else 0.0
    d = np.max(np.abs(a - b)) if b.size else 0.0
    return d / sc if sc > 0 else d


def _incr_ok(new, want, old, tol=TOL, ulps=8):
    """Increment check: |new - want| <= tol ||want - old||_inf plus a few
    ulps of the coordinate magnitude (the GPU may fuse x + dt*(...) into
    one rounding where the oracle rounds twice).  Returns (ok, measure)."""
    new, want, old = (np.asarray(a, dtype=np.float64) for a in (new, want, old))
    if want.size == 0:
        return True, 0.0
    d = np.max(np.abs(new - want))
    inc = np.max(np.abs(want - old))
    floor = ulps * np.spacing(np.max(np.abs(old)) + np.max(np.abs(want)))
    lim = tol * inc + floor
    return d <= lim, d / inc if inc > 0 else d


def _gpu_sorted(lp, wl, **cfg):
    """GPU context with the workload's state Morton-sorted on the device."""
    ctx = lp.make_context(wl, **cfg)
    st = lp.DeviceState.from_host(wl.state)
    perm = ctx.lp_build_cells(st)
    return ctx, st, perm


def _oracle_sorted(wl):
    perm, _ = oracle.sort_perm(wl.state, wl.offsets, wl.params)
    st = wl.state.take(perm)
    return perm, lpgen.State(*[np.ascontiguousarray(a) for a in st.arrays()])


@pytest.mark.parametrize("case", list(CASES))
def test_build_cells_permutation_bit_exact(lp, case):
    wl = CASES[case]()
    _log("case %s n=%d systems=%d" % (case, wl.n, wl.n_sys))
    ctx, st, perm = _gpu_sorted(lp, wl)
    ctx.sync_status()
    operm, ost = _oracle_sorted(wl)
    assert np.array_equal(perm.cpu().numpy(), operm)
    got = st.to_host()
    for a, b in zip(got.arrays(), ost.arrays()):
        assert np.array_equal(a, b)


def _check_neighbours(lp, wl, **cfg):
    ctx, st, perm = _gpu_sorted(lp, wl, **cfg)
    _, ost = _oracle_sorted(wl)
    o = oracle.Oracle(ost, wl.offsets, wl.params, brute=(wl.n <= 16384))
    nb = o.neighbours()
    g = ctx.lp_neighbors(st)
    ctx.sync_status()
    assert g["n_mirror"] == nb.n_mirror
    assert np.array_equal(g["cand_off"].cpu().numpy(), nb.cand_off)
    assert np.array_equal(g["cand_idx"].cpu().numpy(), nb.cand_idx)
    assert np.array_equal(g["ghost_mask"].cpu().numpy(), nb.ghost_mask)
    cnt = g["sten_cnt"].cpu().numpy()
    assert np.array_equal(cnt, nb.sten_cnt)
    gi = g["sten_idx"].cpu().numpy()
    oi = np.where(np.arange(nb.sten_idx.shape[1])[None, :] < nb.sten_cnt[:, None],
                  nb.sten_idx, np.iinfo(np.int32).max)
    oi = np.sort(oi, axis=1)
    oi[oi == np.iinfo(np.int32).max] = -1
    assert np.array_equal(gi, oi)
    return ctx


@pytest.mark.parametrize("case", list(CASES))
def test_neighbours_stencils_ghosts_bit_exact(lp, case):
    wl = CASES[case]()
    _log("case %s n=%d" % (case, wl.n))
    ctx = _check_neighbours(lp, wl)
    _log("stats %s" % ctx.stats())


@pytest.mark.parametrize("case", ["column16_flow_ragged", "sheared_20x20x12",
                                  "lattice_exact"])
def test_sorted_stencil_path_bit_exact(lp, case):
    """The exact sorted-candidate path (used for overflowing cut buckets)
    gives the same stencils when forced for every particle."""
    wl = CASES[case]()
    _log("case %s n=%d (sorted stencil path)" % (case, wl.n))
    _check_neighbours(lp, wl, debug_flags=lp.LP_DEBUG_SORTED_STENCIL)


@pytest.mark.parametrize("case", ["sheared_20x20x12", "ensemble_3"])
def test_mirror_numbering_through_the_block_scan(lp, case):
    """Mirror ids from the separate scan of the per-tile wall counts (the
    path above 2048 tiles) are those of the in-kernel prefix sums: both
    bit-exact against the oracle on workloads of several tiles."""
    wl = CASES[case]()
    _log("case %s n=%d (mirror scan)" % (case, wl.n))
    _check_neighbours(lp, wl, debug_flags=lp.LP_DEBUG_MIRROR_SCAN)


def test_mirror_numbering_paths_agree_on_the_full_column(lp):
    """128 tiles of the 524,288-particle column: mirror count, candidate
    lists and stencils equal with either way of numbering the mirrors."""
    wl = lpgen.column_bench()
    got = []
    for flags in (0, lp.LP_DEBUG_MIRROR_SCAN):
        ctx, st, _ = _gpu_sorted(lp, wl, debug_flags=flags)
        g = ctx.lp_neighbors(st)
        ctx.sync_status()
        got.append({k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in g.items()})
        del ctx, st
    _log("mirrors %d" % got[0]["n_mirror"])
    assert got[0]["n_mirror"] > 0
    for k in got[0]:
        assert np.array_equal(np.asarray(got[0][k]), np.asarray(got[1][k])), k


def test_steps_on_unaligned_state_arrays(lp):
    """State arrays that start 8 bytes past a 16-byte boundary take the
    one-particle form of the state copy; the trajectory equals the one on
    aligned arrays bit for bit (odd particle count: the paired form's last
    particle too)."""
    import torch
    wl = CASES["column16_flow_ragged"]()
    assert wl.n % 2 == 1
    got = []
    for shift in (0, 1):
        arrs = []
        for a in wl.state.arrays():
            buf = torch.empty(wl.n + 1, dtype=torch.float64, device="cuda")
            t = buf[shift:shift + wl.n]
            t.copy_(torch.as_tensor(a))
            arrs.append(t)
        assert all((t.data_ptr() % 16 == 8) == (shift == 1) for t in arrs)
        ctx = lp.make_context(wl)
        st = lp.DeviceState(arrs)
        for _ in range(3):
            ctx.lp_step(st, wl.dt)
        ctx.sync_status()
        _log("shift %d stats %s" % (shift, ctx.stats()))
        got.append(st.to_host())
    for a, b in zip(got[0].arrays(), got[1].arrays()):
        assert np.array_equal(a, b)


def test_other_entry_points_between_steps_leave_the_step_unchanged(lp):
    """Stencils, fits of other fields and a rheology RHS between two steps
    (with many refits: cond_max = 3) leave the second step as it is without
    them, bit for bit and with the same refit count: the counters a step
    relies on (refit list, sorted-path list, displacement maximum) start
    from zero whatever ran before."""
    import torch
    wl = CASES["column16_flow_ragged"]()
    got = []
    for extra in (False, True):
        ctx = lp.make_context(wl, cond_max=3.0)
        st = lp.DeviceState.from_host(wl.state)
        ctx.lp_step(st, wl.dt)
        ctx.lp_build_cells(st, want_perm=False)
        if extra:
            ctx.lp_neighbors(st)
            F = torch.stack([st.t[3], st.t[4], st.t[5]])
            coef, _ = ctx.lp_fit_derivs(st, F, [1, 1, -1], [0, 0, 0])
            ctx.lp_rheology_rhs(st, coef)
        ctx.sync_status()
        before = ctx.stats()
        for _ in range(2):
            ctx.lp_step(st, wl.dt)
        ctx.sync_status()
        after = ctx.stats()
        _log("extra %s stats before %s after %s" % (extra, before, after))
        got.append((st.to_host(), after["qr_refits"], after["rebuilds"]))
    assert got[0][1] > 0
    assert got[0][1:] == got[1][1:]
    for a, b in zip(got[0][0].arrays(), got[1][0].arrays()):
        assert np.array_equal(a, b)


def _fields(st):
    x, y, z = st.x, st.y, st.z
    return np.stack([np.sin(3.0 * x + 1.0) * np.cos(2.0 * y) + z * z,
                     np.exp(0.5 * x) * np.sin(2.5 * z) - 0.3 * y,
                     np.cos(1.7 * x * y + z)])


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("path", ["gram", "qr"])
def test_fit_derivs_parity(lp, case, path):
    wl = CASES[case]()
    _log("case %s path %s n=%d" % (case, path, wl.n))
    import torch
    cfg = {} if path == "gram" else dict(debug_flags=lp.LP_DEBUG_QR_FIT)
    ctx, st, _ = _gpu_sorted(lp, wl, **cfg)
    _, ost = _oracle_sorted(wl)
    ctx.lp_neighbors(st, candidates=False, stencils=False, ghosts=False)
    F = _fields(ost)
    ms, gz = [1, 1, -1], [0, 0, 1]
    coef, flags = ctx.lp_fit_derivs(st, torch.tensor(F, device="cuda"), ms, gz)
    ctx.sync_status()
    o = oracle.Oracle(ost, wl.offsets, wl.params)
    ocoef, oflags = o.fit(F, ms, gz)
    gc = coef.cpu().numpy()
    for f in range(3):
        for q in range(9):
            e = _relerr(gc[f, q], ocoef[f, q])
            assert e <= TOL, (f, q, e)
    assert np.array_equal(flags.cpu().numpy() & 1, oflags & 1)


@pytest.mark.parametrize("case", list(CASES))
def test_rheology_rhs_parity(lp, case):
    """Closure, second fit and RHS from the oracle's velocity derivatives."""
    wl = CASES[case]()
    _log("case %s n=%d" % (case, wl.n))
    import torch
    ctx, st, _ = _gpu_sorted(lp, wl)
    _, ost = _oracle_sorted(wl)
    ctx.lp_neighbors(st, candidates=False, stencils=False, ghosts=False)
    o = oracle.Oracle(ost, wl.offsets, wl.params)
    r = o.evaluate()
    g = ctx.lp_rheology_rhs(st, torch.tensor(r["coef_u"].reshape(27, -1), device="cuda"))
    ctx.sync_status()
    for name in ("dVdt", "acc", "diag", "grad"):
        got = g[name].cpu().numpy()
        want = r[name]
        for q in range(want.shape[0] if want.ndim == 2 else 1):
            a = got[q] if want.ndim == 2 else got
            b = want[q] if want.ndim == 2 else want
            e = _relerr(a, b)
            assert e <= TOL, (name, q, e)
    gf = g["flags"].cpu().numpy()
    assert np.array_equal(gf & 7, r["flags"] & 7)


_STEP_PATHS = {"gram": {}, "qr": dict(debug_flags=1 << 1),
               "lanes2": dict(debug_flags=1 << 2), "lanes4": dict(debug_flags=1 << 3)}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("path", list(_STEP_PATHS))
def test_step_parity(lp, case, path):
    """lp_step against the oracle step: permutation exact; increments of
    position, velocity and volume within 1e-10 of the oracle's.  Paths:
    Gram fits, forced Householder refits, 2 and 4 lanes per particle."""
    wl = CASES[case]()
    _log("case %s path %s n=%d" % (case, path, wl.n))
    import torch
    cfg = _STEP_PATHS[path]
    ctx = lp.make_context(wl, **cfg)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ctx.lp_step(st, wl.dt, perm)
    ctx.sync_status()
    ost, operm, _ = oracle.step(wl.state, wl.offsets, wl.params, wl.dt)
    assert np.array_equal(perm.cpu().numpy(), operm)
    old = wl.state.take(operm)
    got = st.to_host()
    for k, (a, b, c) in enumerate(zip(got.arrays(), ost.arrays(), old.arrays())):
        ok, e = _incr_ok(a, b, c)
        assert ok, (lp.DeviceState.NAMES[k], e)


@pytest.mark.parametrize("m_max", [9, 20, 64])
def test_step_parity_other_stencil_caps(lp, m_max):
    """The stencil cap m_max (9 = the unknowns, 64 = the largest supported)
    changes which candidates are kept; the step still matches the oracle
    run with the same cap."""
    import torch
    wl = CASES["column16_flow_ragged"]()
    _log("m_max %d" % m_max)
    ctx = lp.make_context(wl, m_max=m_max)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ctx.lp_step(st, wl.dt, perm)
    ctx.sync_status()
    ost, operm, _ = oracle.step(wl.state, wl.offsets, wl.params, wl.dt,
                                cfg=dict(m_max=m_max))
    assert np.array_equal(perm.cpu().numpy(), operm)
    old = wl.state.take(operm)
    for k, (a, b, c) in enumerate(zip(st.to_host().arrays(), ost.arrays(), old.arrays())):
        ok, e = _incr_ok(a, b, c)
        assert ok, (lp.DeviceState.NAMES[k], e)


def test_qr_refit_rows_beyond_one_wavefront(lp):
    """The QR refit holds stencil row k in lane k mod 64 of a wavefront, so
    rows 64 and above sit in a second register slot.  At m_max = 64 on a
    24^3 column with h = 1.35 lattice spacings, top-layer particles keep 64
    rows plus ghost rows; with every stencil sent through the refit, the
    step matches the oracle's run with the same cap."""
    import dataclasses

    import torch
    wl = lpgen.column_bench(nx=24, ny=24, nz=24)
    h = wl.params[0].h * 1.35
    wl.params = [dataclasses.replace(p, h=h, R=2.5 * h) for p in wl.params]
    print("case column 24^3, h x1.35, m_max 64, QR refit, n", wl.n, flush=True)
    chk = lp.make_context(wl, m_max=64)
    s2 = lp.DeviceState.from_host(wl.state)
    chk.lp_build_cells(s2, want_perm=False)
    nb = chk.lp_neighbors(s2, candidates=False)
    rows = nb["sten_cnt"].to(torch.int64) + torch.stack(
        [(nb["ghost_mask"].to(torch.int64) >> o) & 1 for o in range(8)]).sum(0)
    n_big = int((rows > 64).sum())
    _log("rows max %d, %d stencils above 64 rows" % (int(rows.max()), n_big))
    assert n_big > 0
    del chk, s2
    ctx = lp.make_context(wl, m_max=64, debug_flags=lp.LP_DEBUG_QR_FIT)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ctx.lp_step(st, wl.dt, perm)
    ctx.sync_status()
    assert ctx.stats()["qr_refits"] == wl.n
    ost, operm, _ = oracle.step(wl.state, wl.offsets, wl.params, wl.dt,
                                cfg=dict(m_max=64))
    assert np.array_equal(perm.cpu().numpy(), operm)
    old = wl.state.take(operm)
    for k, (a, b, c) in enumerate(zip(st.to_host().arrays(), ost.arrays(), old.arrays())):
        ok, e = _incr_ok(a, b, c)
        assert ok, (lp.DeviceState.NAMES[k], e)


def test_neighbour_list_overflow_is_reported(lp):
    """A cluster denser than the neighbour list holds (more than 256
    entries within the list radius) latches LP_E_CAPACITY; every kernel
    stays within its buffers and the call returns normally."""
    h = 1.0 / 16.0
    p = lpgen.default_params(h)
    st0 = lpgen.lattice_column(8, 8, 8, h / 4, seed=9, params=p)   # spacing h/4
    wl = lpgen.Workload("cluster", st0, np.array([0, st0.n]), [p], 1e-5, 1)
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(st0)
    ctx.lp_step(st, wl.dt)
    with pytest.raises(lp.LPError) as e:
        ctx.sync_status()
    assert e.value.status == 2


def test_autotune_choice_and_step_parity(lp):
    """lp_autotune picks 1, 2 or 4 lanes per particle for each fit; steps
    afterwards still match the oracle."""
    import torch
    wl = CASES["sheared_20x20x12"]()
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    choice = ctx.lp_autotune(st)
    _log("autotune choice %s" % (choice,))
    assert choice[0] in (1, 2, 4) and choice[1] in (1, 2, 4)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ctx.lp_step(st, wl.dt, perm)
    ctx.sync_status()
    ost, operm, _ = oracle.step(wl.state, wl.offsets, wl.params, wl.dt)
    assert np.array_equal(perm.cpu().numpy(), operm)
    old = wl.state.take(operm)
    for k, (a, b, c) in enumerate(zip(st.to_host().arrays(), ost.arrays(), old.arrays())):
        ok, e = _incr_ok(a, b, c)
        assert ok, (lp.DeviceState.NAMES[k], e)


def test_cut_radius_pairs_classified_like_the_oracle(lp):
    """Regression: pairs whose r^2 straddles R^2 depending on fused
    multiply-add must be classified by the unfused definition, as the
    oracle does (the candidate test is compiled without contraction)."""
    from rounding_cases import straddle_workload
    wl, want = straddle_workload()
    _log("straddle pairs %d (inside-unfused %d)" % (len(want), sum(want)))
    _check_neighbours(lp, wl)


def _trajectory_oracle(wl, steps):
    """Oracle trajectory; returns the state indexed by original id."""
    st = wl.state
    ids = np.arange(wl.n)
    for _ in range(steps):
        st, perm, _ = oracle.step(st, wl.offsets, wl.params, wl.dt)
        ids = ids[perm]
    out = [np.empty(wl.n) for _ in range(7)]
    for a, src in zip(out, st.arrays()):
        a[ids] = src
    return lpgen.State(*out)


def _trajectory_gpu(lp, wl, steps, **cfg):
    import torch
    ctx = lp.make_context(wl, **cfg)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ids = np.arange(wl.n)
    for _ in range(steps):
        ctx.lp_step(st, wl.dt, perm)
        ids = ids[perm.cpu().numpy()]
    ctx.sync_status()
    stats = ctx.stats()
    host = st.to_host()
    out = [np.empty(wl.n) for _ in range(7)]
    for a, src in zip(out, host.arrays()):
        a[ids] = src
    return lpgen.State(*out), stats


@pytest.mark.parametrize("case", ["column16_flow_ragged", "sheared_20x20x12"])
def test_multi_step_trajectory_parity(lp, case):
    """Five steps: the neighbour list is built once and reused (particles
    move far less than the skin); the trajectory matches the oracle, which
    searches and re-sorts at every step, particle by particle."""
    wl = CASES[case]()
    steps = 5
    _log("case %s n=%d steps=%d" % (case, wl.n, steps))
    got, stats = _trajectory_gpu(lp, wl, steps)
    _log("stats %s" % stats)
    assert stats["rebuilds"] == 1
    want = _trajectory_oracle(wl, steps)
    for k, (a, b, c) in enumerate(zip(got.arrays(), want.arrays(), wl.state.arrays())):
        ok, e = _incr_ok(a, b, c, tol=1e-9, ulps=64)
        assert ok, (lp.DeviceState.NAMES[k], e)


def test_skin_zero_rebuilds_every_step_and_agrees(lp):
    """skin = 0 rebuilds the list and re-sorts at every step; the
    trajectory equals the default (skin 0.1) one particle by particle."""
    wl = CASES["column16_flow_ragged"]()
    a, sa = _trajectory_gpu(lp, wl, 4, skin=0.0)
    b, sb = _trajectory_gpu(lp, wl, 4)
    _log("skin 0: %s / skin 0.1: %s" % (sa, sb))
    assert sa["rebuilds"] == 4 and sb["rebuilds"] == 1
    for k, (x, y, c) in enumerate(zip(a.arrays(), b.arrays(), wl.state.arrays())):
        ok, e = _incr_ok(x, y, c, tol=1e-12, ulps=64)
        assert ok, (k, e)


def test_isolated_particle_free_fall(lp):
    """Edge case: a single gas-regime particle falls with a = g exactly."""
    import torch
    p = lpgen.default_params(0.05)
    st0 = lpgen.State(np.array([0.1]), np.array([0.2]), np.array([4.0]),
                      np.array([1.0]), np.array([-2.0]), np.array([0.5]),
                      np.array([1.0 / 0.3]))
    wl = lpgen.Workload("single", st0, np.array([0, 1]), [p], 1e-3, 1)
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(st0)
    ctx.lp_step(st, 1e-3)
    ctx.sync_status()
    ost, _, _ = oracle.step(st0, wl.offsets, wl.params, 1e-3)
    for a, b in zip(st.to_host().arrays(), ost.arrays()):
        assert np.array_equal(a, b)


def test_empty_system_and_neighbour_free_systems(lp):
    """Edge cases: an empty system between two others, and systems far
    apart in space that must not see each other."""
    a = lpgen.column_small()
    h = a.params[0].h
    b = lpgen.lattice_column(5, 5, 4, h, seed=3, params=a.params[0])
    st0 = lpgen.State.concat([a.state, b])   # b overlaps a in space
    offs = np.array([0, a.n, a.n, a.n + b.n])
    wl = lpgen.Workload("three", st0, offs, [a.params[0]] * 3, 1e-4, 1)
    _log("three systems n=%d" % wl.n)
    _check_neighbours(lp, wl)
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(st0)
    ctx.lp_step(st, 1e-4)
    ctx.sync_status()
    ost, _, _ = oracle.step(st0, offs, wl.params, 1e-4)
    old = st0.take(oracle.sort_perm(st0, offs, wl.params)[0])
    for k, (x, y, c) in enumerate(zip(st.to_host().arrays(), ost.arrays(), old.arrays())):
        ok, e = _incr_ok(x, y, c)
        assert ok, (k, e)


def test_full_size_column_step_parity(lp):
    """The 64 x 64 x 128 benchmark column (524,288 particles), one step in
    the benchmark's launch configuration, every particle against the
    oracle."""
    import torch
    wl = lpgen.column_bench()
    _log("column_bench n=%d" % wl.n)
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ctx.lp_step(st, wl.dt, perm)
    ctx.sync_status()
    _log("gpu stats %s" % ctx.stats())
    ost, operm, _ = oracle.step(wl.state, wl.offsets, wl.params, wl.dt, brute=False)
    assert np.array_equal(perm.cpu().numpy(), operm)
    old = wl.state.take(operm)
    for k, (a, b, c) in enumerate(zip(st.to_host().arrays(), ost.arrays(), old.arrays())):
        ok, e = _incr_ok(a, b, c)
        _log("  %s increment rel err %.3e; array rel err %.3e"
             % (lp.DeviceState.NAMES[k], e, _relerr(a, b)))
        assert ok and _relerr(a, b) <= TOL


def test_full_size_sheared_column_step_parity(lp):
    """The 128 x 128 x 64 sheared column (1,048,576 particles, stencils of
    8 to 60 rows, some particles with up to 193 list entries), one step,
    every particle against the oracle."""
    import torch
    wl = lpgen.column_sheared()
    _log("column_sheared n=%d" % wl.n)
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ctx.lp_step(st, wl.dt, perm)
    ctx.sync_status()
    _log("gpu stats %s" % ctx.stats())
    ost, operm, _ = oracle.step(wl.state, wl.offsets, wl.params, wl.dt, brute=False)
    assert np.array_equal(perm.cpu().numpy(), operm)
    old = wl.state.take(operm)
    for k, (a, b, c) in enumerate(zip(st.to_host().arrays(), ost.arrays(), old.arrays())):
        ok, e = _incr_ok(a, b, c)
        _log("  %s increment rel err %.3e" % (lp.DeviceState.NAMES[k], e))
        assert ok


def test_error_paths_report_cleanly(lp):
    """Host-side validation: bad dt, calls out of order, capacity."""
    wl = lpgen.column_small()
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    with pytest.raises(lp.LPError) as e:
        ctx.lp_step(st, -1.0)
    assert e.value.status == 1
    with pytest.raises(lp.LPError) as e:
        ctx.lp_neighbors(st)
    assert e.value.status == 5
    with pytest.raises(lp.LPError) as e:
        ctx.lp_step_adjoint(st, -1.0, st)
    assert e.value.status == 1
    gauss = lp.make_context(wl, weight=lp.LP_W_GAUSS)
    with pytest.raises(lp.LPError) as e:
        gauss.lp_step_adjoint(st, 1e-4, st)
    assert e.value.status == 1
    small = lp.Context()
    small.reserve(100)
    with pytest.raises(lp.LPError) as e:
        small.set_systems([0, wl.n], wl.params)
        small.lp_step(st, 1e-4)
    assert e.value.status == 2


@pytest.mark.parametrize("case", ["column16", "column16_flow_ragged", "sheared_20x20x12",
                                  "periodic_xy", "ensemble_3"])
def test_hydrostatic_wall_pressure_parity(lp, case):
    """wall_pressure = 1 (mirrors carry the hydrostatic weight between them
    and their source): a step against the oracle with the same option."""
    import torch
    wl = CASES[case]()
    ctx = lp.make_context(wl, wall_pressure=1)
    st = lp.DeviceState.from_host(wl.state)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ctx.lp_step(st, wl.dt, perm)
    ctx.sync_status()
    want, operm, _ = oracle.step(wl.state, wl.offsets, wl.params, wl.dt,
                                 cfg=dict(wall_pressure=1))
    assert np.array_equal(perm.cpu().numpy(), operm)
    old = wl.state.take(operm)
    for k, (a, b, c) in enumerate(zip(st.to_host().arrays(), want.arrays(), old.arrays())):
        ok, e = _incr_ok(a, b, c)
        assert ok, (lp.DeviceState.NAMES[k], e)


@pytest.mark.parametrize("kind", ["step", "step2"])
def test_reflecting_wall_parity(lp, kind):
    """wall_reflect = 1: the ragged flowing column lowered so that its
    bottom row sits 2-8 mm above the wall and pushed down at 10 m/s for
    1 ms, so that this row crosses the wall in one step; both step kinds
    against the oracle with the same option (skin 0.3 keeps the
    second-order predictor inside the list)."""
    import torch
    wl = CASES["column16_flow_ragged"]()
    st0 = wl.state.copy()
    st0.z = st0.z - 0.026
    st0.w = st0.w - 10.0
    dt, skin = 1e-3, 0.3
    ctx = lp.make_context(wl, wall_reflect=1, wall_pressure=1, skin=skin)
    st = lp.DeviceState.from_host(st0)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    (ctx.lp_step2 if kind == "step2" else ctx.lp_step)(st, dt, perm)
    ctx.sync_status()
    fn = oracle.step2 if kind == "step2" else oracle.step
    want, operm, _ = fn(st0, wl.offsets, wl.params, dt, skin=skin,
                        cfg=dict(wall_reflect=1, wall_pressure=1))
    free, _, _ = fn(st0, wl.offsets, wl.params, dt, skin=skin,
                    cfg=dict(wall_pressure=1))
    crossed = int(np.sum(free.z < 0.0))
    _log("%s: %d particles reflected" % (kind, crossed))
    assert crossed > 50 and np.all(want.z >= 0.0)
    assert np.array_equal(perm.cpu().numpy(), operm)
    old = st0.take(operm)
    got = st.to_host()
    for k, (a, b, c) in enumerate(zip(got.arrays(), want.arrays(), old.arrays())):
        ok, e = _incr_ok(a, b, c)
        assert ok, (lp.DeviceState.NAMES[k], e)
    assert ctx.stats()["below_wall"] == 0
