"""Neighbour lists built with a wavefront per cell against the per-particle
scan (LP_DEBUG_PARTICLE_LIST).

Both scans visit the same cells in the same order with the same test, so
the lists are identical entry for entry; everything computed from them
(candidates, stencils, fits, steps) must then be equal bit for bit.  The
per-particle scan is itself checked against the oracle through the
candidate sets of every case (test_gpu_parity.py runs with the default
scan; these tests tie the two scans together).
"""
import sys

import numpy as np
import pytest

import lpgen
from cases import CASES

pytestmark = pytest.mark.gpu


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


def _host(d):
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in d.items()}


def _run(lp, wl, flags, steps, **cfg):
    """Candidates after a sort, then `steps` steps (a rebuild at every step
    when skin is 0): neighbours, final state and permutation."""
    import torch
    ctx = lp.make_context(wl, debug_flags=flags, **cfg)
    st = lp.DeviceState.from_host(wl.state)
    ctx.lp_build_cells(st)
    nb = _host(ctx.lp_neighbors(st))
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    for _ in range(steps):
        ctx.lp_step(st, wl.dt, perm)
    ctx.sync_status()
    out = [a.copy() for a in st.to_host().arrays()]
    stats = ctx.stats()
    del ctx, st
    return nb, out, perm.cpu().numpy(), stats


def _same_runs(a, b):
    nb0, st0, p0, _ = a
    nb1, st1, p1, _ = b
    for k in nb0:
        assert np.array_equal(np.asarray(nb0[k]), np.asarray(nb1[k])), k
    for x, y in zip(st0, st1):
        assert np.array_equal(x, y)
    assert np.array_equal(p0, p1)


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("skin", [0.1, 0.0])
def test_cell_scan_equals_particle_scan(lp, case, skin):
    wl = CASES[case]()
    _log("case %s n=%d systems=%d skin %g" % (case, wl.n, wl.n_sys, skin))
    a = _run(lp, wl, 0, 3, skin=skin)
    b = _run(lp, wl, lp.LP_DEBUG_PARTICLE_LIST, 3, skin=skin)
    _log("stats %s" % a[3])
    _same_runs(a, b)


def test_cell_scan_on_the_full_column(lp):
    """524,288 particles (about 27,000 cells, mirrors along the wall): the
    same neighbours and two rebuilding steps bit for bit."""
    wl = lpgen.column_bench()
    _log("column n=%d" % wl.n)
    a = _run(lp, wl, 0, 2, skin=0.0)
    b = _run(lp, wl, lp.LP_DEBUG_PARTICLE_LIST, 2, skin=0.0)
    assert a[0]["n_mirror"] > 0
    _same_runs(a, b)


def test_cell_scan_in_captured_steps(lp):
    """Captured steps rebuild on the device (the cell count read there, the
    cells taken in grid-stride passes): the same trajectory as with the
    per-particle scan."""
    import torch
    wl = CASES["ensemble_3"]()
    got = []
    for flags in (0, lp.LP_DEBUG_PARTICLE_LIST):
        ctx = lp.make_context(wl, skin=0.002, debug_flags=flags)
        st = lp.DeviceState.from_host(wl.state)
        ids = torch.arange(wl.n, dtype=torch.int32, device="cuda")
        ctx.lp_step_graph(st, wl.dt, 6, ids)
        ctx.sync_status()
        stats = ctx.stats()
        _log("flags %d stats %s" % (flags, stats))
        assert stats["rebuilds"] >= 2
        got.append(([a.copy() for a in st.to_host().arrays()], ids.cpu().numpy()))
        del ctx, st
    for x, y in zip(got[0][0], got[1][0]):
        assert np.array_equal(x, y)
    assert np.array_equal(got[0][1], got[1][1])


@pytest.mark.parametrize("flags", [0, 128])
def test_list_overflow_with_either_scan(lp, flags):
    """A cluster denser than the list holds (spacing h/4: more than 256
    entries within the list radius) latches LP_E_CAPACITY with either scan;
    both store only the entries that fit."""
    assert lp.LP_DEBUG_PARTICLE_LIST == 128
    h = 1.0 / 16.0
    p = lpgen.default_params(h)
    st0 = lpgen.lattice_column(8, 8, 8, h / 4, seed=9, params=p)
    wl = lpgen.Workload("cluster", st0, np.array([0, st0.n]), [p], 1e-5, 1)
    ctx = lp.make_context(wl, debug_flags=flags)
    st = lp.DeviceState.from_host(st0)
    ctx.lp_step(st, wl.dt)
    with pytest.raises(lp.LPError) as e:
        ctx.sync_status()
    assert e.value.status == 2


def test_cell_scan_with_an_empty_system(lp):
    """Systems may be empty (equal offsets): an empty system keeps one empty
    cell in the tables, which the cell scan skips; the other systems' lists
    and steps equal the per-particle scan's bit for bit."""
    base = CASES["ensemble_3"]()
    off = [int(v) for v in base.offsets]
    offsets = np.array([off[0], off[1], off[1], off[2], off[3]], dtype=np.int64)
    params = [base.params[0], base.params[1], base.params[1], base.params[2]]
    wl = lpgen.Workload("ensemble_3_empty", base.state, offsets, params, base.dt, 1)
    _log("systems %d offsets %s" % (wl.n_sys, list(offsets)))
    a = _run(lp, wl, 0, 3, skin=0.0)
    b = _run(lp, wl, lp.LP_DEBUG_PARTICLE_LIST, 3, skin=0.0)
    _same_runs(a, b)


def _clumps(k=70, nclump=8, seed=21):
    """Dense clumps of k particles (more than a wavefront's 64 in one cell)
    within 0.3 list radii of their centres, centres three list radii apart
    on the wall plane (so their particles have mirror sources): every clump
    stays below the list capacity."""
    h = 1.0 / 16.0
    p = lpgen.default_params(h)
    rv = p.R * 1.1
    rng = np.random.default_rng(seed)
    pts = []
    for c in range(nclump):
        cx, cy = 3.0 * rv * (c % 4), 3.0 * rv * (c // 4)
        d = rng.normal(size=(k, 3))
        d *= (0.3 * rv * rng.random(k) ** (1.0 / 3.0) / np.linalg.norm(d, axis=1))[:, None]
        pts.append(d + np.array([cx, cy, 0.5 * rv]))
    xyz = np.concatenate(pts)
    n = xyz.shape[0]
    z0 = np.zeros(n)
    st = lpgen.State(xyz[:, 0].copy(), xyz[:, 1].copy(), xyz[:, 2].copy(),
                     z0.copy(), z0.copy(), z0.copy(), np.full(n, 1.0 / 0.55))
    return lpgen.Workload("clumps", st, np.array([0, n]), [p], 1e-5, 1)


def test_cell_scan_on_cells_of_more_than_64_particles(lp):
    """Cells holding 70 particles take two chunks of the wavefront, and
    their mirror scans replace and restore the cell's candidate sequence
    between chunks: the same neighbours as the per-particle scan, and both
    equal to the oracle's candidate sets."""
    import oracle
    wl = _clumps()
    got = []
    for flags in (0, lp.LP_DEBUG_PARTICLE_LIST):
        ctx = lp.make_context(wl, debug_flags=flags)
        st = lp.DeviceState.from_host(wl.state)
        ctx.lp_build_cells(st)
        got.append(_host(ctx.lp_neighbors(st)))
        ctx.sync_status()
        del ctx, st
    _log("clumps n=%d mirrors %d" % (wl.n, got[0]["n_mirror"]))
    assert got[0]["n_mirror"] > 0
    for k in got[0]:
        assert np.array_equal(np.asarray(got[0][k]), np.asarray(got[1][k])), k
    perm, _ = oracle.sort_perm(wl.state, wl.offsets, wl.params)
    ost = wl.state.take(perm)
    ost = lpgen.State(*[np.ascontiguousarray(a) for a in ost.arrays()])
    nb = oracle.Oracle(ost, wl.offsets, wl.params, brute=True).neighbours()
    g = got[0]
    assert g["n_mirror"] == nb.n_mirror
    assert np.array_equal(g["cand_off"], nb.cand_off)
    assert np.array_equal(g["cand_idx"], nb.cand_idx)
    assert np.array_equal(g["ghost_mask"], nb.ghost_mask)
    assert np.array_equal(g["sten_cnt"], nb.sten_cnt)
