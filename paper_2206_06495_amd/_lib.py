"""ctypes declarations of the C ABI in include/rbffd.h.

Loads ``librbffd.so`` from this package directory.  torch is imported first
so that the library binds to the HIP runtime torch already loaded (one HIP
runtime per process).  A missing library is an error: there is no fallback.
"""
import ctypes
import os

import torch  # noqa: F401  (must precede the HIP library load)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librbffd.so")

RBF_OK = 0
RBF_E_ARG = -1
RBF_E_SINGULAR = -2
RBF_E_NOCONV = -3
RBF_E_DEVICE = -4
RBF_E_NOMEM = -5
RBF_E_NAN = -6

OP_ID, OP_DX, OP_DY, OP_LAP = 1, 2, 4, 8
FORCE_SMALL_STENCIL = 0x80000000

EXPORTED = [
    "rbf_last_error", "rbf_abi_version", "rbf_build_nodes", "rbf_knn", "rbf_knn_noalloc",
    "rbf_assemble_weights", "rbf_ell_apply", "rbf_ell_autotune", "rbf_cast_f32", "rbf_ell_transpose",
    "rbf_ell_transpose_weights", "rbf_ell_apply_transpose", "rbf_solver_create",
    "rbf_step", "rbf_step_batch", "rbf_solve_pressure", "rbf_solver_apply_precond", "rbf_solver_profile", "rbf_solver_query",
    "rbf_solver_diagnostics", "rbf_solver_forces", "rbf_adjoint_step",
    "rbf_solver_destroy",
]

c_double_p = ctypes.POINTER(ctypes.c_double)
c_int64_p = ctypes.POINTER(ctypes.c_int64)
c_int8_p = ctypes.POINTER(ctypes.c_int8)
c_void_p = ctypes.c_void_p


class Grid(ctypes.Structure):
    _fields_ = [("n_v", ctypes.c_int64), ("n_p", ctypes.c_int64),
                ("xv", c_void_p), ("xp", c_void_p), ("v_tag", c_void_p),
                ("p_tag", c_void_p), ("p_normal", c_void_p)]


class Ops(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32),
                ("idx_vv", c_void_p), ("vv_dx", c_void_p), ("vv_dy", c_void_p), ("vv_lap", c_void_p),
                ("idx_pv", c_void_p), ("pv_dx", c_void_p), ("pv_dy", c_void_p),
                ("idx_pp", c_void_p), ("pp_dx", c_void_p), ("pp_dy", c_void_p), ("pp_lap", c_void_p),
                ("idx_vp", c_void_p), ("vp_dx", c_void_p), ("vp_dy", c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("dt", ctypes.c_double),
                ("rtol_h", ctypes.c_double), ("rtol_p", ctypes.c_double),
                ("maxit_h", ctypes.c_int32), ("maxit_p", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("u_conv", ctypes.c_double)]


class State(ctypes.Structure):
    _fields_ = [("u", c_void_p), ("v", c_void_p), ("p_tilde", c_void_p), ("p", c_void_p),
                ("cu_prev", c_void_p), ("cv_prev", c_void_p), ("step", ctypes.c_int64)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("restarts", ctypes.c_int32),
                ("final_flag", ctypes.c_int32)]


class Diagnostics(ctypes.Structure):
    _fields_ = [("div_max", ctypes.c_double), ("div_rms", ctypes.c_double),
                ("kinetic_energy", ctypes.c_double), ("speed_max", ctypes.c_double),
                ("cfl", ctypes.c_double)]


class SolverInfo(ctypes.Structure):
    _fields_ = [("viscous_jacobi", ctypes.c_int32), ("lattice_precond", ctypes.c_int32),
                ("jacobi_bound", ctypes.c_double), ("aux_precond", ctypes.c_int32),
                ("aux_cells", ctypes.c_int32), ("viscous_mixed", ctypes.c_int32),
                ("aux_smooth_weight", ctypes.c_double)]


class StepStats(ctypes.Structure):
    _fields_ = [("steps_done", ctypes.c_int32), ("status", ctypes.c_int32),
                ("helmholtz_iters", ctypes.c_int64), ("poisson_iters", ctypes.c_int64),
                ("last_helmholtz_u", SolveStats), ("last_helmholtz_v", SolveStats),
                ("last_poisson", SolveStats)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python paper_2206_06495_amd/build.py` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    S = ctypes.c_int32
    lib.rbf_last_error.restype = ctypes.c_char_p
    lib.rbf_last_error.argtypes = []
    lib.rbf_abi_version.restype = ctypes.c_int32
    lib.rbf_abi_version.argtypes = []
    lib.rbf_build_nodes.restype = S
    lib.rbf_build_nodes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64,
                                    c_int64_p, c_void_p, c_void_p, c_int64_p, c_void_p, c_void_p,
                                    c_void_p]
    lib.rbf_knn.restype = S
    lib.rbf_knn.argtypes = [c_void_p, ctypes.c_int64, c_void_p, ctypes.c_int64, ctypes.c_int32,
                            c_void_p, c_void_p]
    lib.rbf_knn_noalloc.restype = S
    lib.rbf_knn_noalloc.argtypes = [c_void_p, ctypes.c_int64, c_void_p, ctypes.c_int64,
                                    ctypes.c_int32, c_void_p, c_void_p]
    lib.rbf_assemble_weights.restype = S
    lib.rbf_assemble_weights.argtypes = [c_void_p, ctypes.c_int64, c_void_p, ctypes.c_int64,
                                         c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_uint32, c_void_p, c_void_p, c_int64_p, c_void_p]
    lib.rbf_ell_apply.restype = S
    lib.rbf_ell_apply.argtypes = [ctypes.c_int64, ctypes.c_int32, c_void_p, c_void_p, c_void_p,
                                  c_void_p, ctypes.c_int32, c_void_p]
    lib.rbf_ell_autotune.restype = S
    lib.rbf_ell_autotune.argtypes = [ctypes.c_int64, ctypes.c_int32, c_void_p, c_void_p, c_void_p,
                                     c_void_p, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float),
                                     c_void_p]
    lib.rbf_cast_f32.restype = S
    lib.rbf_cast_f32.argtypes = [c_void_p, c_void_p, ctypes.c_int64, c_void_p]
    lib.rbf_ell_transpose.restype = S
    lib.rbf_ell_transpose.argtypes = [ctypes.c_int64, ctypes.c_int32, c_void_p, ctypes.c_int64,
                                      c_void_p, c_void_p, c_void_p, c_int64_p, c_void_p]
    lib.rbf_ell_transpose_weights.restype = S
    lib.rbf_ell_transpose_weights.argtypes = [ctypes.c_int64, ctypes.c_int32, c_void_p, c_void_p,
                                              c_void_p, c_void_p, ctypes.c_int32, c_void_p]
    lib.rbf_ell_apply_transpose.restype = S
    lib.rbf_ell_apply_transpose.argtypes = [ctypes.c_int64, c_void_p, c_void_p, c_void_p,
                                            c_void_p, c_void_p, ctypes.c_int32, c_void_p]
    lib.rbf_solver_create.restype = S
    lib.rbf_solver_create.argtypes = [ctypes.POINTER(c_void_p), ctypes.POINTER(Grid),
                                      ctypes.POINTER(Ops), c_void_p, c_void_p,
                                      ctypes.POINTER(Params), c_void_p]
    lib.rbf_step.restype = S
    lib.rbf_step.argtypes = [c_void_p, ctypes.c_int32, ctypes.POINTER(State),
                             ctypes.POINTER(StepStats)]
    lib.rbf_step_batch.restype = S
    lib.rbf_step_batch.argtypes = [ctypes.POINTER(c_void_p), ctypes.c_int32, ctypes.c_int32,
                                   ctypes.POINTER(State), ctypes.POINTER(StepStats),
                                   ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
    lib.rbf_solve_pressure.restype = S
    lib.rbf_solve_pressure.argtypes = [c_void_p, c_void_p, c_void_p, ctypes.POINTER(SolveStats)]
    lib.rbf_solver_apply_precond.restype = S
    lib.rbf_solver_apply_precond.argtypes = [c_void_p, c_void_p, c_void_p]
    lib.rbf_solver_profile.restype = S
    lib.rbf_solver_profile.argtypes = [c_void_p, ctypes.c_int32, c_double_p, c_int64_p]
    lib.rbf_solver_query.restype = S
    lib.rbf_solver_query.argtypes = [c_void_p, ctypes.POINTER(SolverInfo)]
    lib.rbf_solver_diagnostics.restype = S
    lib.rbf_solver_diagnostics.argtypes = [c_void_p, ctypes.POINTER(State),
                                           ctypes.POINTER(Diagnostics)]
    lib.rbf_solver_forces.restype = S
    lib.rbf_solver_forces.argtypes = [c_void_p, ctypes.POINTER(Grid), ctypes.POINTER(State),
                                      ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
    lib.rbf_adjoint_step.restype = S
    lib.rbf_adjoint_step.argtypes = [c_void_p, ctypes.POINTER(State), ctypes.POINTER(State),
                                     c_void_p, c_double_p]
    lib.rbf_solver_destroy.restype = None
    lib.rbf_solver_destroy.argtypes = [c_void_p]
    return lib


lib = _load()


class RbfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


def check(status):
    if status != RBF_OK:
        raise RbfError(status, lib.rbf_last_error().decode(errors="replace"))
    return status
