"""Throughput of the LP granular-flow step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|fp32r]

A step is one lp_step over the whole 64 x 64 x 128 = 524,288-particle
granular column (h = 0.5/64 m, jitter 0.05 h, hydrostatic density, resting
on the wall z = 0, dt = 2e-5 s): Morton cell build, mirrors, neighbour
search and stencil selection with ghosts, least-squares fit of u, v, w,
mu(I) closure, fit of P and eta, right-hand side and explicit update.
The state is resident in HBM before the timed region; K consecutive steps
are timed between device synchronisations.

Printed (one JSON line): particle-updates/s in FP64 (and the refined-FP32
mode beside it), the dominant kernel's achieved rate against the FP64
vector roof (phase events on the library's stream), adjoint step-pairs/s
of a 50-step gradient on the 131,072-particle column, and the FP64 CPU
oracle timed on the host as a baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-updates/s per RHS eval (FP64 vs refined FP32) + adjoint steps/s"

# Peaks of one MI355X (published): FP64 vector 78.6 TFLOP/s, FP32 vector
# 157.3 TFLOP/s, HBM 8 TB/s.
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

# Algorithmic work of the pass-1 kernel per particle (fit of u, v, w on a
# 60-row, 9-column stencil plus closure), counted as for a Householder
# least-squares solve: 0.5k row build + 9.2k QR (2 m n^2 - 2 n^3 / 3) +
# 3 x 2.1k (Q^T b and back substitution) + 0.2k closure.
PASS1_FLOP_PER_PARTICLE = 16.2e3
# What the kernel actually executes per particle with 60 stencil rows:
# 60 x (45 Gram + 27 moment FMAs = 144 flop + 12 row flop) + ~1.4k for the
# Cholesky factor, 3 solves, 3 rows of G^-1 and the closure.
PASS1_FLOP_EXECUTED = 60 * 156 + 1.4e3
# The refined-FP32 pass-1 kernel per particle at 60 rows: a float32 sweep
# of Gram moments (as the FP64 kernel: 60 x 156 flop plus a float32
# Cholesky and solves, ~1.0k), and a float64 residual sweep (per row: 12
# row flop, 3 residuals of 9 FMAs, 3 x 9 FMAs into A^T r = 120 flop) with
# the correction solves (~0.4k).
PASS1_REF_FLOP_F32 = 60 * 156 + 1.0e3
PASS1_REF_FLOP_F64 = 60 * 120 + 0.4e3
# Average neighbour-list length of the benchmark column (reals within
# R (1 + skin) plus potential mirror sources; mean over 20,000 sampled
# particles of lpgen.column_bench()).
LIST_ENTRIES = 77.5
# Algorithmic HBM bytes per particle of the selection kernel: own position
# (24) and list count (4), the list (4 per entry), every neighbour position
# once (24), a bucket code per entry (1 per entry), the stencil record (12)
# and keep mask (32).
SELECT_BYTES_PER_PARTICLE = 24 + 4 + 4 * LIST_ENTRIES + 24 + LIST_ENTRIES + 12 + 32
# ... of the pass-2 kernel on a 60-row stencil: own state (56), P, eta and
# flags (17), record and mask (44), the slot words of the kept rows
# (2 x 60), the pass-1 hand-off (296), every neighbour's P, eta and
# position once (40), the new state written (56).
PASS2_BYTES_PER_PARTICLE = 56 + 17 + 44 + 2 * 60 + 296 + 40 + 56


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32r"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="time budget of the one-thread oracle runs")
    ap.add_argument("--adjoint-steps", type=int, default=50)
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-sheared", action="store_true")
    ap.add_argument("--ensemble-steps", type=int, default=20)
    ap.add_argument("--ensemble-adjoint-steps", type=int, default=20)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-step-only", action="store_true",
                    help="print only the timing of lp_step_adjoint calls (for counter runs)")
    ap.add_argument("--no-second-order", action="store_true")
    ap.add_argument("--no-layer", action="store_true")
    ap.add_argument("--no-cubic", action="store_true")
    ap.add_argument("--no-errors", action="store_true",
                    help="skip the per-output errors against the oracle")
    ap.add_argument("--collapse", action="store_true",
                    help="also run the a = 0.6 column collapse (Sec. 4.2.1) and "
                         "report its runout against the empirical fits")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with three 1 GiB device-to-device copies, the "
                         "reference for the HBM byte counters")
    return ap.parse_args()


# Sources that make up the pass-1 kernel; its committed byte counts hold only
# while they are unchanged.
PASS1_SOURCES = ("paper_2206_14061_amd/csrc/lp_fit.hip",
                 "paper_2206_14061_amd/csrc/lp_finish.h",
                 "paper_2206_14061_amd/csrc/lp_fitcore.h",
                 "paper_2206_14061_amd/csrc/lp_visit.h",
                 "paper_2206_14061_amd/csrc/lp_internal.h",
                 "paper_2206_14061_amd/build.py")
PASS1_PROFILE = "profiles/k_pass1_st_column_64x64x128.md"
SELECT_SOURCES = ("paper_2206_14061_amd/csrc/lp_stencil.hip",
                  "paper_2206_14061_amd/csrc/lp_visit.h",
                  "paper_2206_14061_amd/csrc/lp_internal.h",
                  "paper_2206_14061_amd/build.py")
SELECT_PROFILE = "profiles/k_select_column_64x64x128.md"
PASS2_SOURCES = PASS1_SOURCES
PASS2_PROFILE = "profiles/k_pass2_st_column_64x64x128.md"
# float64 flop one lp_step_adjoint call executes per particle, counted by
# SQ_INSTS_VALU_FLOPS_FP64 over every kernel of the call (committed record)
ADJOINT_SOURCES = ("paper_2206_14061_amd/csrc/lp_adjoint.hip",
                   "paper_2206_14061_amd/csrc/lp_fitcore.h",
                   "paper_2206_14061_amd/csrc/lp_visit.h",
                   "paper_2206_14061_amd/csrc/lp_internal.h",
                   "paper_2206_14061_amd/build.py")
ADJOINT_PROFILE = "profiles/adjoint_step_column_32x32x128.md"


def sources_digest(paths) -> str:
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def kernel_traffic(profile, sources):
    """HBM bytes per launch of a kernel from its committed FETCH_SIZE and
    WRITE_SIZE counts, each scaled by what the counter reads for a plain
    copy of known size; None when the kernel's sources have changed since
    the counters were taken."""
    path = os.path.join(ROOT, profile)
    if not os.path.exists(path):
        return None
    m = re.search(r"^traffic-record: (\{.*\})\s*$", open(path).read(), re.M)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("source_sha256") != sources_digest(sources):
        return None
    return 1024.0 * (rec["fetch_kib"] * rec["fetch_scale"]
                     + rec["write_kib"] * rec["write_scale"])


def adjoint_bench(torch, lp, lpgen, steps: int, warmup: int = 1, order: int = 1):
    """Gradient of the runout loss L = sum softplus((x - 0.3 m)/h) after
    `steps` steps (explicit, or second-order with order 2) of the 32 x 32 x
    128 column (131,072 particles, dt = 5e-5 s) with respect to the initial
    state and (mu_s, mu_2, I0), with a checkpoint every 10 steps: forward
    with checkpoints, then recompute and reverse.  Returns adjoint
    step-pairs/s and the split."""
    from paper_2206_14061_amd.autograd import simulate
    wl = lpgen.column_adjoint()
    h = wl.params[0].h
    ctx = lp.make_context(wl)
    theta0 = [[p.mu_s, p.mu_2, p.I0] for p in wl.params]

    def once():
        state = [torch.tensor(a, device="cuda", requires_grad=True)
                 for a in wl.state.arrays()]
        theta = torch.tensor(theta0, dtype=torch.float64, device="cuda",
                             requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = simulate(ctx, wl.offsets, wl.params, state, theta, wl.dt, steps,
                       checkpoint_every=10, order=order)
        loss = torch.nn.functional.softplus((out[0] - 0.3) / h).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ctx.sync_status()
        return t1 - t0, t2 - t1, loss.item(), theta.grad, state[3].grad

    for _ in range(warmup):
        once()
    tf, tb, loss, gth, gu = once()
    return {"workload": wl.name, "particles": wl.n, "steps": steps, "order": order,
            "checkpoint_every": 10, "dt": wl.dt,
            "step_pairs_per_s": steps / (tf + tb),
            "ms_forward": 1e3 * tf, "ms_backward": 1e3 * tb, "loss": loss,
            "dL_dtheta": gth.cpu().tolist(),
            "max_abs_dL_du0": float(gu.abs().max().item())}


def sheared_bench(torch, lp, lpgen, steps: int):
    """The 128 x 128 x 64 column after a seeded shear (1,048,576 particles,
    uneven stencils): stencil-size histogram, autotuned lanes per particle,
    FP64 and refined-FP32 step rates and the share of stencils refitted in
    float64."""
    wl = lpgen.column_sheared()
    out = {"workload": wl.name, "particles": wl.n, "steps": steps, "dt": wl.dt}
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    ctx.lp_build_cells(st, want_perm=False)
    nb = ctx.lp_neighbors(st, candidates=False)
    rows = nb["sten_cnt"].to(torch.int64) + \
        torch.stack([(nb["ghost_mask"].to(torch.int64) >> o) & 1 for o in range(8)]).sum(0)
    edges = list(range(0, 73, 8))
    hist = torch.histc(rows.to(torch.float64), bins=9, min=0, max=72).cpu().tolist()
    out["rows_histogram"] = {"bin_edges": edges, "counts": [int(c) for c in hist]}
    del ctx, st
    for name, prec in (("fp64", lp.LP_FP64), ("fp32r", lp.LP_FP32_REFINED)):
        ctx = lp.make_context(wl, precision=prec)
        st = lp.DeviceState.from_host(wl.state)
        lanes = ctx.lp_autotune(st)
        plan = ctx.lp_fit_plan()
        for _ in range(2):
            ctx.lp_step(st, wl.dt)
        ctx.sync_status()
        ctx.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.lp_step(st, wl.dt)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        ctx.sync_status()
        stt = ctx.stats()
        out[name] = {"value": wl.n * steps / t, "unit": "particle-updates/s",
                     "ms_per_step": 1e3 * t / steps, "lanes_per_particle": list(lanes),
                     "fit_plan": plan,
                     "fp64_refit_fraction": stt["qr_refits"] / (wl.n * steps),
                     "stats": stt}
        del ctx, st
    out["fp32r_speedup_vs_fp64"] = out["fp32r"]["value"] / out["fp64"]["value"]
    return out


def graded_bench(torch, lp, lpgen, steps: int):
    """Uneven stencils batched by size class: a 1,048,576-particle random
    cloud whose density falls tenfold with height (stencils from a few
    neighbours plus ghosts to the full 60 rows), FP64 steps with the fits
    as one launch per fit (LDS-staged, one lane per particle) and with the
    plan lp_autotune picks (size classes with their own lanes per particle
    when faster); the plan, the class histogram and the per-class times
    lp_autotune measured."""
    wl = lpgen.cloud_graded()
    out = {"workload": wl.name, "particles": wl.n, "steps": steps, "dt": wl.dt}

    def timed(ctx, st):
        for _ in range(2):
            ctx.lp_step(st, wl.dt)
        ctx.sync_status()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.lp_step(st, wl.dt)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        ctx.sync_status()
        return 1e3 * t / steps

    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    out["ms_per_step_one_launch"] = timed(ctx, st)
    del ctx, st
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    ctx.lp_autotune(st)
    out["fit_plan"] = ctx.lp_fit_plan()
    out["ms_per_step_autotuned"] = timed(ctx, st)
    del ctx, st
    ctx = lp.make_context(wl, debug_flags=lp.LP_DEBUG_CLASSES)
    st = lp.DeviceState.from_host(wl.state)
    out["ms_per_step_classes_fixed_lanes"] = timed(ctx, st)
    out["value"] = wl.n / (1e-3 * out["ms_per_step_autotuned"])
    out["unit"] = "particle-updates/s"
    return out


def second_order_bench(torch, lp, wl, steps: int, warmup: int, precision: int,
                       ms_first_order: float):
    """lp_step2 (Heun: two right-hand-side evaluations per step) on the
    benchmark column: steps per second and RHS evaluations per second."""
    ctx = lp.make_context(wl, precision=precision)
    st = lp.DeviceState.from_host(wl.state)
    for _ in range(warmup):
        ctx.lp_step2(st, wl.dt)
    ctx.sync_status()
    ctx.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.lp_step2(st, wl.dt)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ctx.sync_status()
    ms = 1e3 * t / steps
    return {"ms_per_step": ms, "value": wl.n / (ms * 1e-3), "unit": "particle-updates/s",
            "rhs_evals_per_step": 2, "particle_rhs_evals_per_s": 2 * wl.n / (ms * 1e-3),
            "cost_vs_first_order_step": ms / ms_first_order, "steps": steps,
            "stats": ctx.stats()}


def cubic_bench(torch, lp, wl, steps: int, warmup: int):
    """lp_step with cubic (19-unknown) fits on the benchmark column (m_max
    56 so that stencil and ghost rows fill one wavefront), with the phase
    split; against the quadratic fits at the same m_max."""
    out = {"m_max": 56}
    for name, order in (("cubic", 3), ("quadratic", 2)):
        ctx = lp.make_context(wl, fit_order=order, m_max=56)
        st = lp.DeviceState.from_host(wl.state)
        for _ in range(warmup):
            ctx.lp_step(st, wl.dt)
        ctx.sync_status()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.lp_step(st, wl.dt)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        ctx.profile(True)
        ctx.profile_read()
        for _ in range(steps):
            ctx.lp_step(st, wl.dt)
        torch.cuda.synchronize()
        ph = ctx.profile_read()
        ctx.profile(False)
        ctx.sync_status()
        nst = max(ph.pop("steps"), 1)
        out[name] = {"ms_per_step": 1e3 * t / steps, "value": wl.n * steps / t,
                     "unit": "particle-updates/s",
                     "phases_ms": {k: v / nst for k, v in ph.items()}}
    out["cost_vs_quadratic"] = out["cubic"]["ms_per_step"] / out["quadratic"]["ms_per_step"]
    # roofline of the two cubic fits against the FP64 vector peak: Householder
    # QR of the m x 19 row matrix (2 m n^2 - 2 n^3 / 3) in each pass, with 3
    # right-hand sides in pass 1 and 2 in pass 2 (4 m n - n^2 each), m the
    # mean rows (kept stencil rows plus ghost rows at m_max 56)
    ctx = lp.make_context(wl, fit_order=3, m_max=56)
    st = lp.DeviceState.from_host(wl.state)
    ctx.lp_build_cells(st, want_perm=False)
    nb = ctx.lp_neighbors(st, candidates=False, ghosts=True)
    ghosts = torch.zeros_like(nb["ghost_mask"], dtype=torch.int64)
    gm = nb["ghost_mask"].to(torch.int64)
    for o in range(8):
        ghosts += (gm >> o) & 1
    m = float((nb["sten_cnt"].to(torch.float64) + ghosts.to(torch.float64)).mean().item())
    del ctx, st, nb
    ncol = 19
    flop = (2 * (2 * m * ncol * ncol - 2.0 * ncol ** 3 / 3)
            + 5 * (4 * m * ncol - ncol * ncol))
    ph = out["cubic"]["phases_ms"]
    t = (ph["pass1"] + ph["pass2"]) * 1e-3
    achieved = flop * wl.n / t / 1e12
    out["roofline"] = {"kernel": "k_pass1_cubic + k_pass2_cubic (16 lanes per particle)",
                       "bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                       "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                       "traffic": None, "mean_rows": m, "per_particle": flop}
    return out


def layer_bench(torch, lp, lpgen, t_end: float = 0.05, every: float = 0.005):
    """Granular-layer compression (the paper's Sec. 4.1): a 0.03 m layer
    periodic in x and y (12 x 12 x 40 particles) at rest with mean solid
    fraction 0.5 settles on the wall under gravity; captured steps of
    5e-6 s.  Reports twice the mass centroid over time, the quasi-static
    rest height H0 phi_mean / phi_max of the closure, the paper's figures,
    and the step rate of this small system."""
    wl = lpgen.layer_periodic()
    p = wl.params[0]
    per = int(round(every / wl.dt))
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    ids = torch.arange(wl.n, dtype=torch.int32, device="cuda")
    mass = torch.tensor(1.0 / wl.state.V, device="cuda")
    heights = []
    ctx.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nchunks = int(round(t_end / every))
    for c in range(nchunks + 1):
        if c:
            ctx.lp_step_graph(st, wl.dt, per, ids)
        m = mass[ids.long()]
        heights.append(2.0 * float((st.t[2] * m).sum() / m.sum()))
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ctx.sync_status()
    stt = ctx.stats()
    phi_mean = float(np.mean(1.0 / wl.state.V))
    return {"workload": wl.name, "particles": wl.n, "dt": wl.dt, "t_end": t_end,
            "two_centroid_height_m": heights, "settled_height_m": float(np.mean(heights[-3:])),
            "quasi_static_height_m": 0.03 * phi_mean / p.phi_max,
            "paper_expected_m": 0.025, "paper_reported_m": 0.020,
            "below_wall_particle_steps": stt["below_wall"], "rebuilds": stt["rebuilds"],
            "steps_per_s": nchunks * per / t}


def collapse_run(torch, lp, lpgen, t_end: float = 0.17, every: float = 0.01,
                 dv_max: float = 0.02, dt_floor: float = 1.0 / 1024):
    """Axisymmetric column collapse, a = 0.6 (r_i = 0.05 m, h_i = 0.03 m,
    120,631 particles, h = 1.25 mm) to t_end: second-order steps with the
    reflecting wall, the hydrostatic mirror pressure, a linear-fallback
    tolerance of 5e-2, the linear fit for stencils of fewer than 9 real rows
    and a list skin of 0.3, under a step-size control on the relative
    volume change: a step that changes some particle's V by more than
    dv_max (relative), or whose predictor leaves the neighbour list, is
    undone and retried at half the step (re-sorting first); the step grows
    back by 1.25x, up to the workload's dt, after steps that change V by
    less than dv_max / 4.  Reports the runout radius (99th percentile of the
    particle radius), the centre height and the largest speed every `every`
    s, and the empirical fits r_inf = r_i (1 + 1.24 a), h_inf = a r_i, t_inf
    = 3 sqrt(h_i / g)."""
    wl = lpgen.column_cylinder()
    p = wl.params[0]
    # skin 0.3: fast front particles leave the predictor inside the list;
    # a large cell reservation: ejected particles widen the bounding box
    ctx = lp.Context(wall_reflect=1, wall_pressure=1, fallback_tol=5e-2, min_real_rows=9,
                     skin=0.3)
    ctx.reserve(wl.n, 1 << 24)
    ctx.set_systems(list(wl.offsets), wl.params)
    st = lp.DeviceState.from_host(wl.state)
    q = torch.tensor([0.99], dtype=torch.float64, device="cuda")
    dt0 = wl.dt
    dt, t, steps, rejected, dt_min = dt0, 0.0, 0, 0, dt0
    resort = lp.StepRecord(wl.n, force_sort=True)
    perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    rows, stop = [], "t_end"

    def sample():
        r = torch.sqrt(st.t[0] ** 2 + st.t[1] ** 2)
        u = torch.sqrt(st.t[3] ** 2 + st.t[4] ** 2 + st.t[5] ** 2)
        core = r < 0.2 * 0.05
        rows.append({"t": t, "r99_m": float(torch.quantile(r, q)),
                     "h_center_m": float(st.t[2][core].max()) if bool(core.any()) else None,
                     "u_max": float(u.max()), "phi_max": float((1.0 / st.t[6]).max()),
                     "dt": dt, "steps": steps})
        _progress("collapse t = %.3f s: r99 %.4f m, u_max %.2f m/s, %d steps, %d undone"
                  % (t, rows[-1]["r99_m"], rows[-1]["u_max"], steps, rejected))

    sample()
    t0 = time.perf_counter()
    retry = False
    next_sample = every
    while t < t_end - 1e-12:
        h_dt = min(dt, t_end - t)
        prev = st.clone()
        ok = True
        try:
            if retry:
                ctx.lp_step2(st, h_dt, rec=resort)
                order = resort.perm[:wl.n].long()
            else:
                ctx.lp_step2(st, h_dt, perm)
                order = perm.long()
            ctx.sync_status()
            # the step may re-sort: perm[new] = old
            dv = float((st.t[6] / prev.t[6][order] - 1.0).abs().max())
            ok = dv <= dv_max
        except lp.LPError as e:
            if e.status != lp._lib.LP_E_STATE:
                stop = "error: %s" % e
                break
            ok, dv = False, float("inf")
        if not ok:
            # undo: the previous state, a fresh sort, half the step
            st = prev
            rejected += 1
            dt *= 0.5
            dt_min = min(dt_min, dt)
            retry = True
            if dt < dt_floor * dt0:
                stop = ("some particle's volume collapses faster than any step "
                        "resolves (the step fell below %g of dt)" % dt_floor)
                break
            continue
        retry = False
        t += h_dt
        steps += 1
        if dv < 0.25 * dv_max:
            dt = min(dt0, 1.25 * dt)
        if t >= next_sample - 1e-12:
            sample()
            next_sample += every
    if rows[-1]["t"] < t:
        sample()
    a, r_i, h_i = 0.6, 0.05, 0.03
    return {"workload": wl.name, "particles": wl.n, "dt": dt0, "series": rows,
            "stopped": stop, "seconds": time.perf_counter() - t0, "steps": steps,
            "rejected_steps": rejected, "dt_min": dt_min, "dv_max": dv_max,
            "lube_r_inf_m": r_i * (1.0 + 1.24 * a), "lube_h_inf_m": a * r_i,
            "lube_t_inf_s": 3.0 * (h_i / abs(p.g[2])) ** 0.5,
            "paper_r_m": 0.085, "paper_h_m": 0.027}


def ensemble_bench(torch, lp, lpgen, steps: int, adjoint_steps: int):
    """64 independent columns (8k-200k particles each, their own mu(I)
    parameters; 6.7M particles) advanced in the same launches: `steps`
    steps captured in one HIP graph, FP64 and refined FP32, then the
    gradient of a runout loss through `adjoint_steps` steps."""
    from paper_2206_14061_amd.autograd import simulate
    wl = lpgen.ensemble()
    out = {"workload": "ensemble_64_columns", "systems": len(wl.params),
           "particles": wl.n, "graph_steps": steps, "dt": wl.dt}
    for name, prec in (("fp64", lp.LP_FP64), ("fp32r", lp.LP_FP32_REFINED)):
        ctx = lp.make_context(wl, precision=prec)
        st = lp.DeviceState.from_host(wl.state)
        ids = torch.arange(wl.n, dtype=torch.int32, device="cuda")
        ctx.lp_step_graph(st, wl.dt, steps, ids)     # capture + first replay
        ctx.sync_status()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.lp_step_graph(st, wl.dt, steps, ids)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        ctx.sync_status()
        out[name] = {"value": wl.n * steps / t, "unit": "particle-updates/s",
                     "ms_per_step": 1e3 * t / steps, "stats": ctx.stats()}
        del ctx, st, ids
    out["fp32r_speedup_vs_fp64"] = out["fp32r"]["value"] / out["fp64"]["value"]
    # forward + adjoint (checkpointed, eager steps), from a seeded smooth
    # flow (0.5 m/s, wavelength 8h) so that particles leave the
    # quasi-static branch and mu(I) acts.  Runout target of each column:
    # 5 cm beyond its initial right face; particles stay in their system's
    # index range through re-sorts, so targets are set by index.
    wl = lpgen.with_shear_velocity(wl)
    ctx = lp.make_context(wl)
    h = wl.params[0].h
    off = wl.offsets
    xt = np.empty(wl.n)
    for c in range(len(wl.params)):
        xt[off[c]:off[c + 1]] = wl.state.x[off[c]:off[c + 1]].max() + 0.05
    xt = torch.tensor(xt, device="cuda")
    state = [torch.tensor(a, device="cuda", requires_grad=True) for a in wl.state.arrays()]
    theta = torch.tensor([[p.mu_s, p.mu_2, p.I0] for p in wl.params],
                         dtype=torch.float64, device="cuda", requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fin = simulate(ctx, wl.offsets, wl.params, state, theta, wl.dt, adjoint_steps,
                   checkpoint_every=10)
    loss = torch.nn.functional.softplus((fin[0] - xt) / h).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ctx.sync_status()
    out["adjoint"] = {"steps": adjoint_steps, "checkpoint_every": 10,
                      "step_pairs_per_s": adjoint_steps / (t2 - t0),
                      "ms_forward": 1e3 * (t1 - t0), "ms_backward": 1e3 * (t2 - t1),
                      "initial_velocity": "seeded smooth field, 0.5 m/s, wavelength 8h",
                      "max_abs_dL_dtheta": float(theta.grad.abs().max().item()),
                      "systems_with_nonzero_dL_dtheta":
                          int((theta.grad.abs().amax(dim=1) > 0).sum().item())}
    return out


def copy_calibration(torch):
    """Three device-to-device copies of 1 GiB: far beyond the L2 and the
    last-level cache, so each reads and writes exactly 2^30 bytes of HBM."""
    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return 8 * n


def cpu_baseline(wl, seconds: float):
    """The FP64 oracle as it stands on the host: one full step of the same
    column (Morton order, cell-list neighbours, stencils, fits, closure,
    update), timed three times on all host cores (OpenMP over particles)
    and on one thread; the median of the runs.  The one-thread runs stop
    early once they have used `seconds` (at least one run)."""
    import oracle

    def runs(threads, budget):
        oracle.set_threads(threads)
        used = oracle.num_threads()
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            oracle.step(wl.state, wl.offsets, wl.params, wl.dt, brute=False)
            times.append(time.perf_counter() - t0)
            if sum(times) >= budget:
                break
        return used, float(np.median(times)), len(times)

    try:
        cores, t_all, n_all = runs(0, float("inf"))
        _, t_one, n_one = runs(1, seconds)
    finally:
        oracle.set_threads(0)
    return {"value": wl.n / t_all, "unit": "particle-updates/s", "cores": cores,
            "kind": "oracle",
            "sample": "one full oracle step of the %d-particle column, median of "
                      "%d runs on %d threads (%.2f s per step)" % (wl.n, n_all, cores, t_all),
            "one_thread": {"value": wl.n / t_one, "cores": 1, "runs": n_one,
                           "s_per_step": t_one}}


def _errors(got, want, scale=None):
    """max |got - want| / max |want| (or / scale), and the element-wise
    relative error with a floor of 1e-3 max |want|."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    sc = float(np.max(np.abs(want))) if scale is None else float(scale)
    if want.size == 0 or sc == 0.0:
        return {"max_rel": 0.0, "elem_rel": 0.0}
    d = np.abs(got - want)
    return {"max_rel": float(np.max(d) / sc),
            "elem_rel": float(np.max(d / np.maximum(np.abs(want), 1e-3 * sc)))}


def errors_vs_oracle(torch, lp, wl):
    """Every output of one step of `wl` against the FP64
    oracle on the same input (outside any timed region).  FP64: the
    velocity derivatives (lp_fit_derivs), P, eta and the closure
    diagnostics, grad P, grad eta, the acceleration and dV/dt
    (lp_rheology_rhs on the GPU's velocity derivatives), and the step's new
    x, u, V (lp_step, as increments new - old).  Refined FP32: the step's
    new x, u, V (its fits run inside lp_step only); u' - u = dt a and
    V' - V = dt dV/dt carry the acceleration and volume rate."""
    import oracle
    onew, operm, r = oracle.step(wl.state, wl.offsets, wl.params, wl.dt, brute=False)
    old = wl.state.take(operm)
    out = {}
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    perm = ctx.lp_build_cells(st)
    same_order = bool(np.array_equal(perm.cpu().numpy(), operm))
    ctx.lp_neighbors(st, candidates=False, stencils=False, ghosts=False)
    U = torch.stack([st.t[3], st.t[4], st.t[5]]).contiguous()
    coef, _ = ctx.lp_fit_derivs(st, U, [1, 1, -1], [0, 0, 0])
    g = ctx.lp_rheology_rhs(st, coef.reshape(27, -1))
    ctx.sync_status()
    c = coef.cpu().numpy()
    fp64 = {"grad_u": _errors(c[:, :3], r["coef_u"][:, :3]),
            "hess_u": _errors(c[:, 3:], r["coef_u"][:, 3:])}
    diag, grad = g["diag"].cpu().numpy(), g["grad"].cpu().numpy()
    for k, name in enumerate(("P", "eta", "I", "mu", "shear_rate")):
        fp64[name] = _errors(diag[k], r["diag"][k])
    fp64["grad_P"] = _errors(grad[:3], r["grad"][:3])
    fp64["grad_eta"] = _errors(grad[3:], r["grad"][3:])
    fp64["acc"] = _errors(g["acc"].cpu().numpy(), r["acc"])
    fp64["dVdt"] = _errors(g["dVdt"].cpu().numpy(), r["dVdt"])
    del ctx, st
    for name, prec in (("fp64", lp.LP_FP64), ("fp32r", lp.LP_FP32_REFINED)):
        ctx = lp.make_context(wl, precision=prec)
        st = lp.DeviceState.from_host(wl.state)
        perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
        ctx.lp_step(st, wl.dt, perm)
        ctx.sync_status()
        same_order = same_order and bool(np.array_equal(perm.cpu().numpy(), operm))
        new = st.to_host()
        res = fp64 if name == "fp64" else {}
        for lab, idx in (("x_increment", (0, 1, 2)), ("u_increment", (3, 4, 5)),
                         ("V_increment", (6,))):
            a = np.stack([new.arrays()[q] - old.arrays()[q] for q in idx])
            b = np.stack([onew.arrays()[q] - old.arrays()[q] for q in idx])
            res[lab] = _errors(a, b)
            # the new value is stored rounded: the largest difference in
            # units of the spacing of the largest new value (the GPU rounds
            # x + dt (u + u')/2 once, the oracle twice)
            big = max(float(np.max(np.abs(onew.arrays()[q]))) for q in idx)
            res[lab]["max_abs_in_ulps_of_value"] = float(np.max(np.abs(a - b))
                                                         / np.spacing(big)) if big else 0.0
        out[name] = res
        del ctx, st
    out["particle_order_equal"] = same_order
    out["note"] = ("max_rel = max|gpu - oracle| / max|oracle| per output; elem_rel = "
                   "max_i |gpu_i - oracle_i| / max(|oracle_i|, 1e-3 max|oracle|); "
                   "step outputs as increments new - old")
    return out


def flop_record(profile, sources):
    """Float64 flop per particle of a committed counter record; None when
    the sources have changed since the counters were taken."""
    path = os.path.join(ROOT, profile)
    if not os.path.exists(path):
        return None
    m = re.search(r"^flop-record: (\{.*\})\s*$", open(path).read(), re.M)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("source_sha256") != sources_digest(sources):
        return None
    return rec["flop_per_particle"]


def adjoint_step_bench(torch, lp, lpgen, calls: int = 10):
    """One lp_step_adjoint call on the 32 x 32 x 128 column (131,072
    particles) after 10 steps from a seeded flow (0.5 m/s, wavelength 8h),
    reversing a recorded step with a seeded cotangent: mean time per call
    from HIP events on the library's stream over `calls` calls, and its
    float64 rate against the vector peak (flop per particle from the
    committed counter record)."""
    wl = lpgen.with_shear_velocity(lpgen.column_adjoint())
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    for _ in range(10):
        ctx.lp_step(st, wl.dt)
    rec = lp.StepRecord(wl.n, force_sort=True)
    inp = st.clone()
    ctx.lp_step(st, wl.dt, rec=rec)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(220614061)
    lam = lp.DeviceState([torch.randn(wl.n, dtype=torch.float64, device="cuda",
                                      generator=gen) for _ in range(7)])
    dth = torch.zeros(len(wl.params), 3, dtype=torch.float64, device="cuda")
    ctx.lp_step_adjoint(inp, wl.dt, lam, dth, rec=rec)
    ctx.sync_status()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(calls):
        ctx.lp_step_adjoint(inp, wl.dt, lam, dth, rec=rec)
    ev1.record()
    torch.cuda.synchronize()
    ctx.sync_status()
    ms = ev0.elapsed_time(ev1) / calls
    out = {"workload": wl.name, "particles": wl.n, "calls": calls, "ms_per_call": ms}
    fpp = flop_record(ADJOINT_PROFILE, ADJOINT_SOURCES)
    if fpp is not None:
        tf = fpp * wl.n / (ms * 1e-3) / 1e12
        out["roofline"] = {"kernel": "lp_step_adjoint (every kernel of one call)",
                           "bound": "alu", "achieved": tf, "peak": PEAK_FP64_TFLOPS,
                           "unit": "TFLOP/s", "frac": tf / PEAK_FP64_TFLOPS,
                           "per_particle": fpp, "avg_call_ms": ms}
    else:
        out["roofline"] = None
    return out


def adjoint_fd_check(torch, lp, lpgen, grad, steps: int):
    """Central differences of the runout loss of the adjoint benchmark (the
    131,072-particle column, `steps` steps, L = sum softplus((x - 0.3)/h))
    in mu_s, mu_2 and I0 against the adjoint gradient `grad`: at eps = 1e-6,
    and Richardson-extrapolated from eps = 1e-4 and 2e-4
    ((4 D(eps) - D(2 eps)) / 3), each a full re-run of the steps.  (Steps of
    1e-3 and more move a particle across the quasi-static threshold in the
    run, a kink of L that the adjoint, with branches held fixed, does not
    see.)"""
    import dataclasses
    wl = lpgen.column_adjoint()
    h = wl.params[0].h
    ctx = lp.make_context(wl)
    p0 = wl.params[0]
    th0 = [p0.mu_s, p0.mu_2, p0.I0]

    def loss(q, e):
        th = list(th0)
        th[q] += e
        ctx.set_systems(wl.offsets, [dataclasses.replace(p0, mu_s=th[0], mu_2=th[1],
                                                        I0=th[2])])
        st = lp.DeviceState.from_host(wl.state)
        for _ in range(steps):
            ctx.lp_step(st, wl.dt)
        ctx.sync_status()
        return float(torch.nn.functional.softplus((st.t[0] - 0.3) / h).sum())

    def central(q, e):
        return (loss(q, e) - loss(q, -e)) / (2.0 * e)

    out = {"steps": steps, "params": ["mu_s", "mu_2", "I0"], "adjoint": list(grad)}
    fd6, rich = [], []
    for q in range(3):
        fd6.append(central(q, 1e-6))
        rich.append((4.0 * central(q, 1e-4) - central(q, 2e-4)) / 3.0)
    scale = max(abs(v) for v in grad) or 1.0
    out["fd_eps_1e-6"] = fd6
    out["fd_richardson_1e-4_2e-4"] = rich
    out["rel_err_eps_1e-6"] = max(abs(a - b) for a, b in zip(fd6, grad)) / scale
    out["rel_err_richardson"] = max(abs(a - b) for a, b in zip(rich, grad)) / scale
    return out


def _progress(msg):
    """One line on stderr as each block of the benchmark finishes."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def main():
    args = _parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the LP step is measured on a "
              "single MI355X (--gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    import lpgen
    import paper_2206_14061_amd as lp

    torch.cuda.set_device(0)
    if args.adjoint_step_only:
        print(json.dumps({"adjoint_step": adjoint_step_bench(torch, lp, lpgen)}), flush=True)
        return
    wl = lpgen.column_bench()

    def run(steps, warmup, **cfg):
        """Times `steps` lp_step calls after `warmup`, then the same number
        again with phase events; returns (ms/step, phases, stats)."""
        ctx = lp.make_context(wl, **cfg)
        st = lp.DeviceState.from_host(wl.state)
        torch.cuda.synchronize()
        for _ in range(warmup):
            ctx.lp_step(st, wl.dt)
        ctx.sync_status()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.lp_step(st, wl.dt)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        ctx.sync_status()
        ctx.profile(True)
        ctx.profile_read()
        for _ in range(steps):
            ctx.lp_step(st, wl.dt)
        torch.cuda.synchronize()
        ph = ctx.profile_read()
        ctx.profile(False)
        ctx.sync_status()
        nst = max(ph.pop("steps"), 1)
        return 1e3 * elapsed / steps, {k: v / nst for k, v in ph.items()}, ctx.stats()

    def run_graph(steps, warmup, **cfg):
        """The same steps captured as one HIP graph (lp_step_graph: device-side
        re-sort decisions, no host synchronisation between steps): one
        warm-up call captures and runs `steps` steps, the timed call replays
        them.  Returns ms/step."""
        ctx = lp.make_context(wl, **cfg)
        st = lp.DeviceState.from_host(wl.state)
        ids = torch.arange(wl.n, dtype=torch.int32, device="cuda")
        for _ in range(max(warmup, 1)):
            ctx.lp_step_graph(st, wl.dt, steps, ids)
        ctx.sync_status()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.lp_step_graph(st, wl.dt, steps, ids)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        ctx.sync_status()
        return 1e3 * elapsed / steps

    main_prec = lp.LP_FP64 if args.precision == "fp64" else lp.LP_FP32_REFINED
    ms_eager, phases, stats = run(args.steps, args.warmup, precision=main_prec)
    ms_graph = run_graph(args.steps, args.warmup, precision=main_prec)
    ms_per_step = ms_eager
    value = wl.n / (ms_per_step * 1e-3)
    dominant = max(("select", "pass1", "pass2"), key=lambda k: phases[k])
    # the other precision on the same column
    other = "fp32r" if args.precision == "fp64" else "fp64"
    ms_o, ph_o, st_o = run(args.steps, args.warmup,
                           precision=lp.LP_FP32_REFINED if other == "fp32r" else lp.LP_FP64)
    ms64 = ms_eager if args.precision == "fp64" else ms_o
    ms32 = ms_o if args.precision == "fp64" else ms_eager
    compare = {"precision": other, "value": wl.n / (ms_o * 1e-3),
               "ms_per_step": ms_o, "phases_ms": ph_o, "stats": st_o,
               "fp32r_speedup_vs_fp64": ms64 / ms32}
    # the same steps with the neighbour list rebuilt (and the column
    # re-sorted) at every step
    k0 = max(2, args.steps // 2)
    ms_rebuild, _, _ = run(k0, args.warmup, precision=main_prec, skin=0.0)
    _progress("column steps done (%.4f ms/step)" % ms_eager)
    fp64 = args.precision == "fp64"
    t_pass1 = phases["pass1"] * 1e-3
    if fp64:
        # the work the kernel executes (normal equations), against the FP64
        # vector peak; the Householder count of the same fit beside it
        executed = PASS1_FLOP_EXECUTED * wl.n / t_pass1 / 1e12
        house = PASS1_FLOP_PER_PARTICLE * wl.n / t_pass1 / 1e12
        roof1 = {"kernel": "k_pass1_st (fit of u, v, w + mu(I) closure)",
                 "bound": "alu", "achieved": executed, "peak": PEAK_FP64_TFLOPS,
                 "unit": "TFLOP/s", "frac": executed / PEAK_FP64_TFLOPS,
                 "per_particle": PASS1_FLOP_EXECUTED,
                 "householder_equivalent": {"per_particle": PASS1_FLOP_PER_PARTICLE,
                                            "tflops": house,
                                            "frac": house / PEAK_FP64_TFLOPS}}
    else:
        # float32 moment sweep and float64 residual sweep: the time both
        # would take at their peaks, over the launch time
        t_roof = wl.n * (PASS1_REF_FLOP_F32 / (PEAK_FP32_TFLOPS * 1e12)
                         + PASS1_REF_FLOP_F64 / (PEAK_FP64_TFLOPS * 1e12))
        roof1 = {"kernel": "k_pass1_ref (float32 fit + float64 residual correction "
                           "of u, v, w; mu(I) closure)",
                 "bound": "alu", "achieved": t_roof / t_pass1, "peak": 1.0,
                 "unit": "fraction of the mixed FP32/FP64 roof",
                 "frac": t_roof / t_pass1,
                 "per_particle": {"f32": PASS1_REF_FLOP_F32, "f64": PASS1_REF_FLOP_F64},
                 "tflops_f32": PASS1_REF_FLOP_F32 * wl.n / t_pass1 / 1e12,
                 "tflops_f64": PASS1_REF_FLOP_F64 * wl.n / t_pass1 / 1e12}
    roof1["traffic"] = kernel_traffic(PASS1_PROFILE, PASS1_SOURCES) if fp64 else None
    roof1["avg_launch_ms"] = phases["pass1"]
    roofs = {"pass1": roof1}
    for ph, name, per, prof, src in (
            ("select", "k_select (exact candidate test, octant firsts, ghosts, keep mask)",
             SELECT_BYTES_PER_PARTICLE, SELECT_PROFILE, SELECT_SOURCES),
            ("pass2", ("k_pass2_st" if fp64 else "k_pass2_ref")
             + " (fit of P, eta; right-hand side; update)",
             PASS2_BYTES_PER_PARTICLE, PASS2_PROFILE, PASS2_SOURCES)):
        gbs = per * wl.n / (phases[ph] * 1e-3) / 1e9
        roofs[ph] = {"kernel": name, "bound": "hbm", "achieved": gbs,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
                     "traffic": kernel_traffic(prof, src) if (fp64 or ph == "select")
                     else None,
                     "avg_launch_ms": phases[ph], "per_particle": per}
    roof = dict(roofs[dominant])
    roof["dominant_phase"] = dominant
    # neighbour data the rows of the two fits consume (48 B per row in
    # pass 1: position and velocity; 40 B in pass 2: position, P and eta;
    # read from LDS in staged tiles), over the mean kept rows of the
    # column's stencils (ghost rows read nothing); and the least-squares
    # work of both fits at the Householder count (2 m n^2 - 2 n^3 / 3 for
    # the factor, 4 m n - n^2 per right-hand side)
    ctx_n = lp.make_context(wl)
    st_n = lp.DeviceState.from_host(wl.state)
    ctx_n.lp_build_cells(st_n, want_perm=False)
    nb = ctx_n.lp_neighbors(st_n, candidates=False, ghosts=False)
    rows = float(nb["sten_cnt"].to(torch.float64).mean().item())
    del ctx_n, st_n, nb
    t_fit = (phases["pass1"] + phases["pass2"]) * 1e-3
    ncol = 9
    qr_flop = sum(2 * rows * ncol * ncol - 2.0 * ncol ** 3 / 3 + k * (4 * rows * ncol - ncol * ncol)
                  for k in (3, 2))
    fit_rates = {"mean_stencil_rows": rows,
                 "row_data_gbs": wl.n * rows * (48 + 40) / t_fit / 1e9,
                 "qr_tflops": wl.n * qr_flop / t_fit / 1e12}
    out = {"metric": METRIC, "value": value, "unit": "particle-updates/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms_per_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if args.precision == "fp64" else "f32+f64",
           "data": "synthetic",
           "config": {"workload": wl.name, "particles": wl.n, "dt": wl.dt,
                      "precision": args.precision, "m_max": 60,
                      "R_over_h": 2.5, "skin": 0.1, "parallelism": "none"},
           "phases_ms": phases, "stats": stats, "other_precision": compare,
           "ms_per_step_graph": ms_graph,
           "ms_per_step_rebuild_every_step": ms_rebuild,
           "roofline": roof, "roofline_by_kernel": roofs, "fit_rates": fit_rates}
    if not args.no_second_order:
        out["second_order"] = second_order_bench(torch, lp, wl, args.steps, args.warmup,
                                                 main_prec, ms_eager)
        _progress("second-order steps done")
    if not args.no_cubic:
        out["cubic_fits"] = cubic_bench(torch, lp, wl, args.steps, args.warmup)
        _progress("cubic fits done")
    if not args.no_errors:
        # the benchmark column starts at rest (u = 0: every velocity
        # derivative, eta and I are exactly 0), so the errors are taken on
        # the same column with a seeded flow (0.5 m/s, wavelength 8h)
        wl_flow = lpgen.with_shear_velocity(wl)
        out["errors_vs_oracle"] = {"workload": wl_flow.name,
                                   **errors_vs_oracle(torch, lp, wl_flow)}
        _progress("errors against the oracle done")
    if not args.no_adjoint:
        out["adjoint"] = adjoint_bench(torch, lp, lpgen, args.adjoint_steps)
        out["adjoint"]["adjoint_step"] = adjoint_step_bench(torch, lp, lpgen)
        out["adjoint"]["fd_check"] = adjoint_fd_check(
            torch, lp, lpgen, out["adjoint"]["dL_dtheta"][0], args.adjoint_steps)
        _progress("adjoint and its central differences done")
        if not args.no_second_order:
            out["adjoint_second_order"] = adjoint_bench(torch, lp, lpgen,
                                                        args.adjoint_steps, order=2)
            _progress("second-order adjoint done")
    if not args.no_sheared:
        out["sheared"] = sheared_bench(torch, lp, lpgen, 20)
        out["graded_cloud"] = graded_bench(torch, lp, lpgen, 10)
        _progress("sheared column and graded cloud done")
    if not args.no_layer:
        out["layer_compression"] = layer_bench(torch, lp, lpgen)
        _progress("layer compression done")
    if args.collapse:
        out["collapse"] = collapse_run(torch, lp, lpgen)
        _progress("column collapse done")
    if not args.no_ensemble:
        out["ensemble"] = ensemble_bench(torch, lp, lpgen, args.ensemble_steps,
                                         args.ensemble_adjoint_steps)
        _progress("ensemble done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
        _progress("cpu baseline done")
    if args.copy_calibration:
        out["copy_calibration_bytes"] = copy_calibration(torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
