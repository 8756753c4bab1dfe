"""MI355X-native Lagrangian-particle granular-flow step (arXiv:2206.14061).

The method's work runs in the HIP library ``liblp_gfx950.so`` behind the C
ABI of ``include/lp.h``; this module only marshals torch CUDA tensors
(device memory and the current stream) into those calls.  Function names
follow the C ABI: ``lp_build_cells``, ``lp_neighbors``, ``lp_fit_derivs``,
``lp_rheology_rhs``, ``lp_step``, ``lp_step2``, ``lp_step_adjoint``,
``lp_step2_adjoint``.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, List, Optional, Sequence

from . import _lib
from ._lib import (LP_DEBUG_CLASSES, LP_DEBUG_GLOBAL_GATHER, LP_DEBUG_LANES2,
                   LP_DEBUG_LANES4, LP_DEBUG_MIRROR_SCAN, LP_DEBUG_PARTICLE_LIST,
                   LP_DEBUG_QR_FIT, LP_DEBUG_SORTED_STENCIL, LP_FP32_REFINED,
                   LP_FP64, LP_W_GAUSS, LP_W_UNIT, LPConfig, LPError,
                   LPParams, LPState, LPStepRecord)

FLAG_LINEAR = 1
FLAG_QR = 8


def _torch():
    import torch
    return torch


def params_struct(p) -> LPParams:
    """LPParams from an object with the lp_params fields (e.g. lpgen.Params)."""
    s = LPParams()
    for k in ("rho_s", "d", "mu_s", "mu_2", "I0", "phi_c", "phi_min",
              "phi_max", "alpha", "beta", "h", "R", "wall_z"):
        setattr(s, k, float(getattr(p, k)))
    for a in range(3):
        s.g[a] = float(p.g[a])
    lo = getattr(p, "box_lo", (0.0, 0.0))
    ln = getattr(p, "box_len", (0.0, 0.0))
    for a in range(2):
        s.box_lo[a] = float(lo[a])
        s.box_len[a] = float(ln[a])
    return s


class DeviceState:
    """Seven float64 CUDA tensors x y z u v w V (structure of arrays)."""

    NAMES = ("x", "y", "z", "u", "v", "w", "V")

    def __init__(self, arrays: Sequence):
        torch = _torch()
        self.t = [a if isinstance(a, torch.Tensor) else
                  torch.as_tensor(a, dtype=torch.float64, device="cuda")
                  for a in arrays]
        for a in self.t:
            if a.dtype != torch.float64 or not a.is_cuda or not a.is_contiguous():
                raise ValueError("state arrays must be contiguous float64 CUDA tensors")

    @staticmethod
    def from_host(st) -> "DeviceState":
        torch = _torch()
        return DeviceState([torch.tensor(a, dtype=torch.float64, device="cuda")
                            for a in st.arrays()])

    def to_host(self):
        import lpgen
        return lpgen.State(*[a.detach().cpu().numpy() for a in self.t])

    def clone(self) -> "DeviceState":
        return DeviceState([a.clone() for a in self.t])

    def struct(self) -> LPState:
        s = LPState()
        for k, a in zip(self.NAMES, self.t):
            setattr(s, k, a.data_ptr())
        return s

    @property
    def n(self) -> int:
        return int(self.t[0].numel())


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class StepRecord:
    """lp_step_record of one step plus its device permutation array:
    ``force_sort`` (set before the step), ``resorted`` and ``list_gen``
    (filled by the step), ``perm`` (int32 device tensor, written when the
    step re-sorted)."""

    def __init__(self, n: int, force_sort: bool = False):
        torch = _torch()
        self.perm = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        self.s = LPStepRecord()
        self.s.force_sort = 1 if force_sort else 0
        self.s.resorted = 0
        self.s.list_gen = -1
        self.s.perm = self.perm.data_ptr()

    @property
    def resorted(self) -> bool:
        return bool(self.s.resorted)

    @property
    def list_gen(self) -> int:
        return int(self.s.list_gen)


def _rec(rec: Optional[StepRecord]):
    return None if rec is None else C.byref(rec.s)


class Context:
    """An lp_ctx bound to the current CUDA device and stream."""

    def __init__(self, m_max: int = 60, precision: int = LP_FP64,
                 cond_max: float = 20.0, weight: int = LP_W_UNIT,
                 ghost_margin: float = 0.5, fallback_tol: float = 1e-12,
                 debug_flags: int = 0, skin: float = 0.1, wall_reflect: int = 0,
                 wall_pressure: int = 0, fit_order: int = 2, min_real_rows: int = 0,
                 stream=None):
        torch = _torch()
        self.lib = _lib.load()
        cfg = LPConfig()
        self.lib.lp_config_default(C.byref(cfg))
        cfg.m_max, cfg.precision, cfg.cond_max = m_max, precision, cond_max
        cfg.weight, cfg.ghost_margin = weight, ghost_margin
        cfg.fallback_tol, cfg.debug_flags = fallback_tol, debug_flags
        cfg.skin = skin
        cfg.wall_reflect = int(wall_reflect)
        cfg.wall_pressure = int(wall_pressure)
        cfg.fit_order = int(fit_order)
        cfg.min_real_rows = int(min_real_rows)
        self.cfg = cfg
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        rc = self.lib.lp_create(C.byref(h), C.c_void_p(stream.cuda_stream),
                                C.byref(cfg))
        if rc != 0:
            raise LPError(rc, "lp_create failed")
        self.h = h
        self.n = 0
        self.n_sys = 0

    def close(self):
        if getattr(self, "h", None):
            self.lib.lp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != 0:
            raise LPError(rc, self.lib.lp_last_error(self.h).decode())

    def reserve(self, n_max: int, cells_max: Optional[int] = None):
        if cells_max is None:
            cells_max = max(1 << 20, 4 * int(n_max))
        self._check(self.lib.lp_reserve(self.h, int(n_max), int(cells_max)))

    def set_systems(self, offsets: Sequence[int], params: Sequence):
        ns = len(params)
        off = (C.c_int64 * (ns + 1))(*[int(v) for v in offsets])
        prm = (LPParams * ns)(*[params_struct(p) for p in params])
        self._check(self.lib.lp_set_systems(self.h, ns, off, prm))
        self.n = int(offsets[-1])
        self.n_sys = ns
        self.offsets = [int(v) for v in offsets]
        self.params = list(params)

    # ---- entry points (names of the C ABI) --------------------------------
    def lp_build_cells(self, st: DeviceState, want_perm: bool = True):
        torch = _torch()
        perm = torch.empty(st.n, dtype=torch.int32, device="cuda") if want_perm else None
        s = st.struct()
        self._check(self.lib.lp_build_cells(self.h, C.byref(s), _ptr(perm)))
        return perm

    def lp_neighbors(self, st: DeviceState, candidates: bool = True,
                     stencils: bool = True, ghosts: bool = True) -> Dict:
        torch = _torch()
        n = st.n
        s = st.struct()
        out: Dict = {}
        needed = C.c_int64(0)
        nm = C.c_int64(0)
        coff = torch.empty(n + 1, dtype=torch.int64, device="cuda") if candidates else None
        scnt = torch.empty(n, dtype=torch.int32, device="cuda") if stencils else None
        sidx = (torch.empty(n * self.cfg.m_max, dtype=torch.int32, device="cuda")
                if stencils else None)
        gm = torch.empty(n, dtype=torch.uint8, device="cuda") if ghosts else None
        # first call: build stencils, counts and the candidate offsets
        self._check(self.lib.lp_neighbors(
            self.h, C.byref(s), _ptr(coff), None, 0,
            C.byref(needed) if candidates else None, _ptr(scnt), _ptr(sidx),
            _ptr(gm), C.byref(nm)))
        out["n_mirror"] = int(nm.value)
        if candidates:
            cidx = torch.empty(max(int(needed.value), 1), dtype=torch.int32, device="cuda")
            self._check(self.lib.lp_neighbors(
                self.h, C.byref(s), _ptr(coff), _ptr(cidx), int(cidx.numel()),
                C.byref(needed), None, None, None, None))
            out["cand_off"] = coff
            out["cand_idx"] = cidx[:int(needed.value)]
        if stencils:
            out["sten_cnt"] = scnt
            out["sten_idx"] = sidx.view(n, self.cfg.m_max)
        if ghosts:
            out["ghost_mask"] = gm
        return out

    def lp_fit_derivs(self, st: DeviceState, f, mirror_sign: Sequence[int],
                      ghost_zero: Sequence[int]):
        torch = _torch()
        f = f.contiguous()
        k = f.shape[0] if f.dim() == 2 else 1
        n = st.n
        coef = torch.empty((k, 9, n), dtype=torch.float64, device="cuda")
        flags = torch.empty(n, dtype=torch.uint8, device="cuda")
        ms = (C.c_int32 * k)(*[int(v) for v in mirror_sign])
        gz = (C.c_int32 * k)(*[int(v) for v in ghost_zero])
        s = st.struct()
        self._check(self.lib.lp_fit_derivs(self.h, C.byref(s), f.data_ptr(), k,
                                           ms, gz, coef.data_ptr(), flags.data_ptr()))
        return coef, flags

    def lp_rheology_rhs(self, st: DeviceState, coef_u) -> Dict:
        torch = _torch()
        n = st.n
        coef_u = coef_u.contiguous()
        out = dict(dVdt=torch.empty(n, dtype=torch.float64, device="cuda"),
                   acc=torch.empty((3, n), dtype=torch.float64, device="cuda"),
                   diag=torch.empty((5, n), dtype=torch.float64, device="cuda"),
                   grad=torch.empty((6, n), dtype=torch.float64, device="cuda"),
                   flags=torch.empty(n, dtype=torch.uint8, device="cuda"))
        s = st.struct()
        self._check(self.lib.lp_rheology_rhs(
            self.h, C.byref(s), coef_u.data_ptr(), out["dVdt"].data_ptr(),
            out["acc"].data_ptr(), out["diag"].data_ptr(), out["grad"].data_ptr(),
            out["flags"].data_ptr()))
        return out

    def lp_step(self, st: DeviceState, dt: float, perm=None,
                rec: Optional[StepRecord] = None):
        """One step in place; rec (optional) records it for lp_step_adjoint."""
        s = st.struct()
        self._check(self.lib.lp_step(self.h, C.byref(s), float(dt), _ptr(perm),
                                     _rec(rec)))

    def lp_step2(self, st: DeviceState, dt: float, perm=None,
                 rec: Optional[StepRecord] = None):
        """Second-order (Heun) step; same state order, perm and record as
        lp_step."""
        s = st.struct()
        self._check(self.lib.lp_step2(self.h, C.byref(s), float(dt), _ptr(perm),
                                      _rec(rec)))

    def lp_autotune(self, st: DeviceState):
        """Times 1, 2 and 4 lanes per particle in both fits on st's stencils
        and keeps the fastest; returns (lanes pass 1, lanes pass 2)."""
        ch = (C.c_int32 * 2)()
        s = st.struct()
        self._check(self.lib.lp_autotune(self.h, C.byref(s), ch))
        return int(ch[0]), int(ch[1])

    def lp_fit_plan(self) -> Dict:
        """The fit plan (lanes per particle, size classes) and the times the
        last lp_autotune measured."""
        plan = (C.c_int32 * 12)()
        ms = (C.c_double * 8)()
        self._check(self.lib.lp_fit_plan(self.h, plan, ms))
        return {"lanes": [plan[0], plan[1]], "size_classes": bool(plan[2]),
                "class_rows": ["<=16", "<=32", ">32"],
                "class_lanes_pass1": [plan[3], plan[4], plan[5]],
                "class_lanes_pass2": [plan[6], plan[7], plan[8]],
                "class_particles": [plan[9], plan[10], plan[11]],
                "ms_one_launch": [ms[0], ms[1]],
                "ms_class_pass1": [ms[2], ms[3], ms[4]],
                "ms_class_pass2": [ms[5], ms[6], ms[7]]}

    def lp_step_graph(self, st: DeviceState, dt: float, nsteps: int, ids=None):
        """nsteps steps replayed as one HIP graph (captured on first use);
        ids (int32 device tensor, optional) follow the particles."""
        s = st.struct()
        self._check(self.lib.lp_step_graph(self.h, C.byref(s), _ptr(ids), float(dt),
                                           int(nsteps)))

    def lp_step_adjoint(self, st: DeviceState, dt: float, adj_out: DeviceState,
                        adj_params=None, want_perm: bool = False,
                        rec: Optional[StepRecord] = None):
        """Reverse of lp_build_cells + lp_step at st (rec None), or of the
        lp_step that filled rec: returns dL/d(st) for dL/d(output) = adj_out
        (and the step's permutation, if asked); adds dL/d(mu_s, mu_2, I0)
        into adj_params (n_sys x 3, float64, device)."""
        return self._adjoint(self.lib.lp_step_adjoint, st, dt, adj_out, adj_params,
                             want_perm, rec)

    def lp_step2_adjoint(self, st: DeviceState, dt: float, adj_out: DeviceState,
                         adj_params=None, want_perm: bool = False,
                         rec: Optional[StepRecord] = None):
        """Reverse of lp_build_cells + lp_step2 at st, or of the lp_step2
        that filled rec (arguments as for lp_step_adjoint)."""
        return self._adjoint(self.lib.lp_step2_adjoint, st, dt, adj_out, adj_params,
                             want_perm, rec)

    def _adjoint(self, fn, st, dt, adj_out, adj_params, want_perm, rec=None):
        torch = _torch()
        adj_in = DeviceState([torch.empty_like(a) for a in st.t])
        if adj_params is None:
            adj_params = torch.zeros(self.n_sys, 3, dtype=torch.float64, device="cuda")
        perm = torch.empty(st.n, dtype=torch.int32, device="cuda") if want_perm else None
        s, ao, ai = st.struct(), adj_out.struct(), adj_in.struct()
        self._check(fn(self.h, C.byref(s), float(dt), C.byref(ao), C.byref(ai),
                       _ptr(adj_params), _ptr(perm), _rec(rec)))
        return (adj_in, perm) if want_perm else adj_in

    def sync_status(self):
        idx = C.c_int64(-1)
        rc = self.lib.lp_sync_status(self.h, C.byref(idx))
        self._check(rc)

    PHASES = ("rebuild_or_copy", "select", "select_sorted", "pass1", "pass1_qr",
              "pass2", "pass2_qr")

    def profile(self, enable: bool = True):
        self._check(self.lib.lp_profile(self.h, 1 if enable else 0))

    def profile_read(self) -> Dict[str, float]:
        """Summed milliseconds per phase since the last read, and steps."""
        ms = (C.c_double * 8)()
        steps = C.c_int64(0)
        self._check(self.lib.lp_profile_read(self.h, ms, C.byref(steps)))
        out = {k: ms[q] for q, k in enumerate(self.PHASES)}
        out["steps"] = int(steps.value)
        return out

    def stats(self) -> Dict[str, int]:
        out = (C.c_int64 * 8)()
        self._check(self.lib.lp_stats(self.h, out))
        return dict(particles=out[0], mirrors=out[1], qr_refits=out[2],
                    sorted_stencils=out[3], below_wall=out[4], rebuilds=out[5],
                    unstaged_tiles=out[6], tiles=out[7])


def lp_step_noalloc(offsets: Sequence[int], params: Sequence, st: DeviceState,
                    dt: float, perm=None, stream=None, **cfg) -> None:
    """One step of st in place through the allocation-free entry point (no
    context; a static device workspace of at most 16384 particles); cfg
    fields as for Context.  Raises LPError on failure."""
    torch = _torch()
    lib = _lib.load()
    c = LPConfig()
    lib.lp_config_default(C.byref(c))
    for k, v in cfg.items():
        setattr(c, k, v)
    ns = len(params)
    off = (C.c_int64 * (ns + 1))(*[int(v) for v in offsets])
    prm = (LPParams * ns)(*[params_struct(p) for p in params])
    if stream is None:
        stream = torch.cuda.current_stream()
    s = st.struct()
    rc = lib.lp_step_noalloc(C.c_void_p(stream.cuda_stream), C.byref(c), ns, off, prm,
                             C.byref(s), float(dt), _ptr(perm))
    if rc != 0:
        raise LPError(rc, "lp_step_noalloc failed")


def make_context(workload, **cfg) -> Context:
    """Context reserved and configured for an lpgen.Workload."""
    ctx = Context(**cfg)
    ctx.reserve(workload.n)
    ctx.set_systems(list(workload.offsets), workload.params)
    return ctx
