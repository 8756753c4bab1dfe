"""Python access to the FP64 CPU oracle (``oracle/lp_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke``
and the CPU-baseline leg of ``bench.py``.  The HIP library and its binding
never import it.

The shared object is compiled with gcc (``-O2 -ffp-contract=off -fopenmp``)
into ``oracle/liblporacle.so`` the first time it is needed, or again when
the C source is newer than the library.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess
import threading
from typing import List, Optional, Sequence

import numpy as np

from lpgen import Params, State

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lp_oracle.c")
_LIB = os.path.join(_HERE, "liblporacle.so")
_lock = threading.Lock()
_lib = None

CFG_DEFAULT = dict(m_max=60, ghost_margin=0.5, phi_ghost_frac=0.99,
                   fallback_tol=1e-12, weight=0, wall_reflect=0, wall_pressure=0,
                   fit_order=2, min_real_rows=0)

FLAG_LINEAR = 1
FLAG_QUAD = 16
BR_GAS, BR_INERTIAL, BR_QUASI = 0, 1, 2


def build(force: bool = False) -> str:
    """Compiles the oracle library; returns its path."""
    with _lock:
        if (not force and os.path.exists(_LIB)
                and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
            return _LIB
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
               "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
        return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = build()
    lib = C.CDLL(path)
    P = C.c_void_p
    i64, i32 = C.c_int64, C.c_int32
    lib.orc_sort.argtypes = [i64, i32, P, P, C.c_double, P, P, P, P, P]
    lib.orc_sort.restype = C.c_int
    lib.orc_nbr_build.argtypes = [i64, i32, P, P, P] + [P] * 7 + [C.c_int]
    lib.orc_nbr_build.restype = C.c_void_p
    lib.orc_nbr_sizes.argtypes = [P, P]
    lib.orc_nbr_export.argtypes = [P] * 8
    lib.orc_nbr_free.argtypes = [P]
    lib.orc_fit.argtypes = [P, P, C.c_int, P, P, P, P]
    lib.orc_fit.restype = C.c_int
    lib.orc_eval.argtypes = [P] * 8
    lib.orc_eval.restype = C.c_int
    lib.orc_update.argtypes = [i64, i32, P, P, C.c_double] + [P] * 9 + [C.c_int]
    lib.orc_update.restype = i64
    lib.orc_boundary.argtypes = [i64, i32, P, P, P, P, P, P, C.c_int]
    lib.orc_num_threads.restype = C.c_int
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_set_threads.restype = None
    lib.orc_lsq.argtypes = [C.c_int, C.c_int, P, P, C.c_int, P]
    lib.orc_lsq.restype = C.c_double
    lib.orc_closure_point.argtypes = [P, C.c_double, P, P, P]
    lib.orc_closure_point.restype = C.c_int
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(t: int) -> None:
    """OpenMP threads of later oracle calls (0: back to the initial count)."""
    _load().orc_set_threads(int(t))


def cfg_vector(cfg: Optional[dict] = None) -> np.ndarray:
    c = dict(CFG_DEFAULT)
    if cfg:
        c.update(cfg)
    return np.array([c["m_max"], c["ghost_margin"], c["phi_ghost_frac"],
                     c["fallback_tol"], c["weight"], c["wall_pressure"],
                     c["fit_order"], c["min_real_rows"]], dtype=np.float64)


def prm_matrix(params: Sequence[Params]) -> np.ndarray:
    return np.ascontiguousarray(np.stack([p.as_vector() for p in params]))


def lsq(A: np.ndarray, B: np.ndarray):
    """Raw Householder least squares of the oracle: returns (C, ratio)."""
    lib = _load()
    A = _f64(A)
    B = _f64(B.reshape(B.shape[0], -1))
    m, nc = A.shape
    nb = B.shape[1]
    Cm = np.empty((nc, nb))
    r = lib.orc_lsq(m, nc, _ptr(A), _ptr(B), nb, _ptr(Cm))
    if r < 0:
        raise ValueError("bad lsq shape")
    return Cm, float(r)


def closure_point(p: Params, V: float, G: np.ndarray):
    """Closure at one point: returns (branch, P, eta, I, mu, |gd|, gd)."""
    lib = _load()
    prm = p.as_vector()
    G = _f64(np.asarray(G).reshape(9))
    out = np.empty(5)
    gd = np.empty(9)
    br = lib.orc_closure_point(_ptr(prm), float(V), _ptr(G), _ptr(out),
                               _ptr(gd))
    return (int(br), out[0], out[1], out[2], out[3], out[4], gd.reshape(3, 3))


SKIN_DEFAULT = 0.1


def sort_perm(state: State, offsets: np.ndarray, params: Sequence[Params],
              skin: float = SKIN_DEFAULT):
    """Morton order inside each system over cells of edge R (1 + skin)
    (1 + 2^-20): returns (perm new->old, keys)."""
    lib = _load()
    n = state.n
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    prm = prm_matrix(params)
    perm = np.empty(n, dtype=np.int32)
    keys = np.empty(n, dtype=np.uint64)
    x, y, z = _f64(state.x), _f64(state.y), _f64(state.z)
    rc = lib.orc_sort(n, len(params), _ptr(off), _ptr(prm), float(skin),
                      _ptr(x), _ptr(y), _ptr(z), _ptr(perm), _ptr(keys))
    if rc != 0:
        raise ValueError("cell coordinate exceeds 21 bits")
    return perm, keys


@dataclasses.dataclass
class Neighbours:
    n: int
    n_mirror: int
    cand_off: np.ndarray      # int64 n+1
    cand_idx: np.ndarray      # int32, ascending ids per particle
    sten_cnt: np.ndarray      # int32 n (without ghosts)
    sten_idx: np.ndarray      # int32 n x m_max (canonical order, padded 0)
    ghost_mask: np.ndarray    # uint8 n
    mirror_src: np.ndarray    # int32 n_mirror
    mirror_state: np.ndarray  # float64 7 x n_mirror (x y z u v w V)


class Oracle:
    """Oracle evaluation of one state (particles in the order given)."""

    def __init__(self, state: State, offsets, params: Sequence[Params],
                 cfg: Optional[dict] = None, brute: Optional[bool] = None):
        self.lib = _load()
        self.state = State(*[_f64(a) for a in state.arrays()])
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self.params = list(params)
        self.prm = prm_matrix(self.params)
        self.cfg = cfg_vector(cfg)
        self.n = state.n
        if brute is None:
            brute = self.n <= 16384
        s = self.state
        self.h = self.lib.orc_nbr_build(
            self.n, len(self.params), _ptr(self.offsets), _ptr(self.prm),
            _ptr(self.cfg), _ptr(s.x), _ptr(s.y), _ptr(s.z), _ptr(s.u),
            _ptr(s.v), _ptr(s.w), _ptr(s.V), int(bool(brute)))
        sz = np.zeros(3, dtype=np.int64)
        self.lib.orc_nbr_sizes(self.h, _ptr(sz))
        self.n_mirror, self.n_cand, self.m_max = (int(v) for v in sz)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_nbr_free(h)
            self.h = None

    def neighbours(self) -> Neighbours:
        n, nm = self.n, self.n_mirror
        coff = np.empty(n + 1, dtype=np.int64)
        cidx = np.empty(max(self.n_cand, 1), dtype=np.int32)
        scnt = np.empty(n, dtype=np.int32)
        sidx = np.empty((n, self.m_max), dtype=np.int32)
        gm = np.empty(n, dtype=np.uint8)
        msrc = np.empty(max(nm, 1), dtype=np.int32)
        m7 = np.empty((7, max(nm, 1)), dtype=np.float64)
        self.lib.orc_nbr_export(self.h, _ptr(coff), _ptr(cidx), _ptr(scnt),
                                _ptr(sidx), _ptr(gm), _ptr(msrc), _ptr(m7))
        return Neighbours(n, nm, coff, cidx[:self.n_cand], scnt, sidx, gm,
                          msrc[:nm], m7[:, :nm])

    def fit(self, fields: np.ndarray, mirror_sign: Sequence[int],
            ghost_zero: Sequence[int]):
        """Fits k fields (k x n at the reals).  Returns (coef k x 9 x n,
        flags n)."""
        f = _f64(np.atleast_2d(fields))
        k = f.shape[0]
        ms = np.ascontiguousarray(mirror_sign, dtype=np.int32)
        gz = np.ascontiguousarray(ghost_zero, dtype=np.int32)
        coef = np.empty((k, 9, self.n), dtype=np.float64)
        flags = np.empty(self.n, dtype=np.uint8)
        rc = self.lib.orc_fit(self.h, _ptr(f), k, _ptr(ms), _ptr(gz),
                              _ptr(coef), _ptr(flags))
        if rc != 0:
            raise ValueError("orc_fit failed")
        return coef, flags

    def evaluate(self, form_m: bool = False) -> dict:
        """Full right-hand side (Form E).  Returns a dict of arrays:
        coef_u (3 x 9 x n), diag (5 x n: P eta I mu |gd|), grad (6 x n:
        grad P, grad eta), acc (3 x n), dVdt (n), flags (n) and, with
        ``form_m``, accM (3 x n, NaN off the inertial branch)."""
        n = self.n
        out = dict(coef_u=np.empty((3, 9, n)), diag=np.empty((5, n)),
                   grad=np.empty((6, n)), acc=np.empty((3, n)),
                   dVdt=np.empty(n), flags=np.empty(n, dtype=np.uint8))
        accM = np.empty((3, n)) if form_m else None
        rc = self.lib.orc_eval(self.h, _ptr(out["coef_u"]), _ptr(out["diag"]),
                               _ptr(out["grad"]), _ptr(out["acc"]),
                               _ptr(out["dVdt"]), _ptr(out["flags"]),
                               _ptr(accM))
        if rc != 0:
            raise ValueError("orc_eval failed")
        if form_m:
            out["accM"] = accM
        return out


def _reflect(cfg: Optional[dict]) -> int:
    return int(bool((cfg or {}).get("wall_reflect", 0)))


def update(state: State, offsets, params: Sequence[Params], dt: float,
           acc: np.ndarray, dVdt: np.ndarray, reflect: int = 0):
    """Explicit update in place (with `reflect`, particles ending below the
    wall are reflected across it); returns the count of particles below
    the wall afterwards."""
    lib = _load()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    prm = prm_matrix(params)
    acc = _f64(acc)
    dVdt = _f64(dVdt)
    arrs = state.arrays()
    for a in arrs:
        assert a.dtype == np.float64 and a.flags.c_contiguous
    return int(lib.orc_update(state.n, len(params), _ptr(off), _ptr(prm),
                              float(dt), *[_ptr(a) for a in arrs], _ptr(acc),
                              _ptr(dVdt), int(reflect)))


def step(state: State, offsets, params: Sequence[Params], dt: float,
         cfg: Optional[dict] = None, brute: Optional[bool] = None,
         skin: float = SKIN_DEFAULT, sort: bool = True):
    """One oracle step: Morton order (unless ``sort`` is false), RHS,
    explicit update.  Returns (new state, perm new->old, RHS dict)."""
    if sort:
        perm, _ = sort_perm(state, offsets, params, skin)
    else:
        perm = np.arange(state.n, dtype=np.int32)
    st = state.take(perm)
    st = State(*[np.ascontiguousarray(a) for a in st.arrays()])
    o = Oracle(st, offsets, params, cfg, brute)
    r = o.evaluate()
    update(st, offsets, params, dt, r["acc"], r["dVdt"], _reflect(cfg))
    return st, perm, r


def step2(state: State, offsets, params: Sequence[Params], dt: float,
          cfg: Optional[dict] = None, brute: Optional[bool] = None,
          skin: float = SKIN_DEFAULT, sort: bool = True):
    """One second-order step by Heun's method (the explicit trapezoidal
    rule), the higher-order time integration the paper's conclusions leave
    for later, applied to the right-hand side f of Sec. 2.1 as evaluated in
    Sec. 3.1 step 7:  s* = s + dt f(s),  s' = s + dt (f(s) + f(s*)) / 2,
    with f = (u, acc, dVdt) for (x, V u, V) read as (x, u, V).  The predictor
    is evaluated in the order of s (neighbours and stencils selected afresh
    at s*).  Returns (new state, perm new->old, (RHS at s, RHS at s*))."""
    if sort:
        perm, _ = sort_perm(state, offsets, params, skin)
    else:
        perm = np.arange(state.n, dtype=np.int32)
    st = state.take(perm)
    st = State(*[np.ascontiguousarray(a, dtype=np.float64) for a in st.arrays()])
    r1 = Oracle(st, offsets, params, cfg, brute).evaluate()
    a1, d1 = r1["acc"], r1["dVdt"]
    vel = (st.u, st.v, st.w)
    pred = State(st.x + dt * st.u, st.y + dt * st.v, st.z + dt * st.w,
                 st.u + dt * a1[0], st.v + dt * a1[1], st.w + dt * a1[2],
                 st.V + dt * d1)
    r2 = Oracle(pred, offsets, params, cfg, brute).evaluate()
    a2, d2 = r2["acc"], r2["dVdt"]
    pvel = (pred.u, pred.v, pred.w)
    half = 0.5 * dt
    pos = [p + half * (q + qs) for p, q, qs in zip((st.x, st.y, st.z), vel, pvel)]
    new_vel = [q + half * (a1[k] + a2[k]) for k, q in enumerate(vel)]
    out = State(*pos, *new_vel, st.V + half * (d1 + d2))
    wrap(out, offsets, params, _reflect(cfg))
    return out, perm, (r1, r2)


def wrap(state: State, offsets, params: Sequence[Params], reflect: int = 0):
    """Maps x and y along periodic axes into their box, in place; with
    `reflect`, particles below the wall are reflected across it."""
    lib = _load()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    prm = prm_matrix(params)
    for a in (state.x, state.y, state.z, state.w):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib.orc_boundary(state.n, len(params), _ptr(off), _ptr(prm), _ptr(state.x),
                     _ptr(state.y), _ptr(state.z), _ptr(state.w), int(reflect))
