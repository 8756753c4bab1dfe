"""ctypes binding of the C ABI in ``include/lp.h`` (argument marshalling
only: every step of the method runs in the HIP library).

Device arrays are torch CUDA tensors; their ``data_ptr()`` is passed
through.  The library must have been built (``python -m
paper_2206_14061_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblp_gfx950.so")

LP_OK, LP_E_ARG, LP_E_CAPACITY, LP_E_NUMERIC, LP_E_HIP, LP_E_STATE = range(6)
LP_FP64, LP_FP32_REFINED = 0, 1
LP_W_UNIT, LP_W_GAUSS = 0, 1
LP_DEBUG_SORTED_STENCIL, LP_DEBUG_QR_FIT = 1, 2
LP_DEBUG_LANES2, LP_DEBUG_LANES4, LP_DEBUG_GLOBAL_GATHER = 4, 8, 16
LP_DEBUG_CLASSES = 32
LP_DEBUG_MIRROR_SCAN = 64
LP_DEBUG_PARTICLE_LIST = 128

STATUS_NAMES = {0: "LP_OK", 1: "LP_E_ARG", 2: "LP_E_CAPACITY",
                3: "LP_E_NUMERIC", 4: "LP_E_HIP", 5: "LP_E_STATE"}

# every symbol include/lp.h declares
EXPORTS = ["lp_config_default", "lp_create", "lp_destroy", "lp_last_error",
           "lp_reserve", "lp_set_systems", "lp_build_cells", "lp_neighbors",
           "lp_fit_derivs", "lp_rheology_rhs", "lp_step", "lp_step2", "lp_autotune",
           "lp_step_graph", "lp_step_adjoint", "lp_step2_adjoint",
           "lp_sync_status", "lp_stats", "lp_profile", "lp_profile_read",
           "lp_step_noalloc", "lp_fit_plan"]


class LPParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("rho_s", "d", "mu_s", "mu_2", "I0", "phi_c", "phi_min",
                 "phi_max", "alpha", "beta")] + \
               [("g", C.c_double * 3)] + \
               [(k, C.c_double) for k in ("h", "R", "wall_z")] + \
               [("box_lo", C.c_double * 2), ("box_len", C.c_double * 2)]


class LPConfig(C.Structure):
    _fields_ = [("m_max", C.c_int32), ("precision", C.c_int32),
                ("cond_max", C.c_double), ("weight", C.c_int32),
                ("ghost_margin", C.c_double), ("fallback_tol", C.c_double),
                ("debug_flags", C.c_int32), ("skin", C.c_double),
                ("wall_reflect", C.c_int32), ("wall_pressure", C.c_int32),
                ("fit_order", C.c_int32), ("min_real_rows", C.c_int32)]


class LPState(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("x", "y", "z", "u", "v", "w", "V")]


class LPStepRecord(C.Structure):
    _fields_ = [("force_sort", C.c_int32), ("resorted", C.c_int32),
                ("list_gen", C.c_int64), ("perm", C.c_void_p)]


class LPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_lib = None


def load():
    """Loads the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("HIP library %s is missing; build it with "
                          "`python -m paper_2206_14061_amd.build`" % LIB_PATH)
    lib = C.CDLL(LIB_PATH)
    P, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    pp = C.POINTER
    lib.lp_config_default.argtypes = [pp(LPConfig)]
    lib.lp_config_default.restype = None
    lib.lp_create.argtypes = [pp(C.c_void_p), P, pp(LPConfig)]
    lib.lp_create.restype = C.c_int
    lib.lp_destroy.argtypes = [P]
    lib.lp_destroy.restype = None
    lib.lp_last_error.argtypes = [P]
    lib.lp_last_error.restype = C.c_char_p
    lib.lp_reserve.argtypes = [P, i64, i64]
    lib.lp_reserve.restype = C.c_int
    lib.lp_set_systems.argtypes = [P, i32, pp(C.c_int64), pp(LPParams)]
    lib.lp_set_systems.restype = C.c_int
    lib.lp_build_cells.argtypes = [P, pp(LPState), P]
    lib.lp_build_cells.restype = C.c_int
    lib.lp_neighbors.argtypes = [P, pp(LPState), P, P, i64, pp(C.c_int64), P, P,
                                 P, pp(C.c_int64)]
    lib.lp_neighbors.restype = C.c_int
    lib.lp_fit_derivs.argtypes = [P, pp(LPState), P, i32, pp(C.c_int32),
                                  pp(C.c_int32), P, P]
    lib.lp_fit_derivs.restype = C.c_int
    lib.lp_rheology_rhs.argtypes = [P, pp(LPState), P, P, P, P, P, P]
    lib.lp_rheology_rhs.restype = C.c_int
    lib.lp_step.argtypes = [P, pp(LPState), C.c_double, P, pp(LPStepRecord)]
    lib.lp_step.restype = C.c_int
    lib.lp_step2.argtypes = [P, pp(LPState), C.c_double, P, pp(LPStepRecord)]
    lib.lp_step2.restype = C.c_int
    lib.lp_autotune.argtypes = [P, pp(LPState), pp(C.c_int32)]
    lib.lp_autotune.restype = C.c_int
    lib.lp_fit_plan.argtypes = [P, pp(C.c_int32), pp(C.c_double)]
    lib.lp_fit_plan.restype = C.c_int
    lib.lp_step_graph.argtypes = [P, pp(LPState), P, C.c_double, i32]
    lib.lp_step_graph.restype = C.c_int
    lib.lp_step_adjoint.argtypes = [P, pp(LPState), C.c_double, pp(LPState),
                                    pp(LPState), P, P, pp(LPStepRecord)]
    lib.lp_step_adjoint.restype = C.c_int
    lib.lp_step2_adjoint.argtypes = lib.lp_step_adjoint.argtypes
    lib.lp_step2_adjoint.restype = C.c_int
    lib.lp_step_noalloc.argtypes = [P, pp(LPConfig), i32, pp(C.c_int64),
                                    pp(LPParams), pp(LPState), C.c_double, P]
    lib.lp_step_noalloc.restype = C.c_int
    lib.lp_sync_status.argtypes = [P, pp(C.c_int64)]
    lib.lp_sync_status.restype = C.c_int
    lib.lp_stats.argtypes = [P, pp(C.c_int64)]
    lib.lp_stats.restype = C.c_int
    lib.lp_profile.argtypes = [P, i32]
    lib.lp_profile.restype = C.c_int
    lib.lp_profile_read.argtypes = [P, pp(C.c_double), pp(C.c_int64)]
    lib.lp_profile_read.restype = C.c_int
    _lib = lib
    return lib
