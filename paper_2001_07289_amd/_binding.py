"""ctypes declarations of the C ABI in ``include/bddcso.h``.

Argument marshalling only.  Loading fails loudly when the library has not
been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libbddcso.so")

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "ESINGULAR", -4: "EBREAKDOWN", -5: "ENOCONV",
          -6: "EHIP"}
MAX_RHS = 64

# every function declared in include/bddcso.h
EXPORTED = [
    "bddcso_default_options", "bddcso_problem_create", "bddcso_problem_info", "bddcso_setup",
    "bddcso_refactor", "bddcso_check_pivots", "bddcso_operator_apply", "bddcso_apply", "bddcso_solve",
    "bddcso_element_grad", "bddcso_box_filter", "bddcso_precond_info", "bddcso_local_coarse",
    "bddcso_precond_destroy", "bddcso_problem_destroy", "bddcso_last_error",
    "bddcso_plan_info", "bddcso_profile", "bddcso_profile_read", "bddcso_copy_probe",
    "bddcso_setup_workspace_size", "bddcso_precond_generation", "bddcso_coef_from_log",
    "bddcso_solve_noalloc", "bddcso_profile_reference", "bddcso_autotune",
]


class Options(C.Structure):
    _fields_ = [("primal_mask", C.c_int), ("weighting", C.c_int), ("precision", C.c_int),
                ("coarse_solver", C.c_int), ("max_nrhs", C.c_int), ("maxit", C.c_int),
                ("rtol", C.c_double), ("fixed_iters", C.c_int), ("flexible", C.c_int),
                ("block_target", C.c_int), ("graph", C.c_int), ("sweep_reg_rows", C.c_int),
                ("slab_lookahead", C.c_int), ("mr_min_rhs", C.c_int), ("update_tile", C.c_int),
                ("slab_width", C.c_int)]


TUNE_MAX = 32


class TuneReport(C.Structure):
    _fields_ = [("n_trials", C.c_int), ("best", C.c_int), ("tried", Options * TUNE_MAX),
                ("step_ms", C.c_double * TUNE_MAX), ("status", C.c_int * TUNE_MAX)]


class Stats(C.Structure):
    _fields_ = [("nrhs", C.c_int), ("iters", C.c_int * MAX_RHS), ("converged", C.c_int * MAX_RHS),
                ("relres", C.c_double * MAX_RHS), ("lambda_min", C.c_double * MAX_RHS),
                ("lambda_max", C.c_double * MAX_RHS), ("kappa", C.c_double * MAX_RHS),
                ("n_coarse", C.c_int64), ("t_solve_ms", C.c_double)]


class PlanStats(C.Structure):
    _fields_ = [("n_coarse", C.c_int64), ("n_fronts", C.c_int64), ("levels", C.c_int64),
                ("max_front", C.c_int64), ("max_front_pivots", C.c_int64), ("n_blocks", C.c_int64),
                ("max_block", C.c_int64), ("coarse_factor_entries", C.c_double),
                ("coarse_sweep_flops", C.c_double), ("local_sweep_flops", C.c_double),
                ("device_bytes", C.c_double)]


class BDDCSOError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


_lib = None


def load() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2001_07289_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i64p = C.c_void_p, C.POINTER(C.c_int64)
    dp = C.POINTER(C.c_double)
    i32p = C.POINTER(C.c_int32)
    sig = {
        "bddcso_default_options": (None, [C.POINTER(Options)]),
        "bddcso_problem_create": (C.c_int, [C.c_int, i64p, dp, i32p, i32p, C.POINTER(vp)]),
        "bddcso_problem_info": (C.c_int, [vp, C.c_int, i64p, i64p, i64p, C.POINTER(C.c_int), i64p]),
        "bddcso_setup_workspace_size": (C.c_int, [vp, C.POINTER(Options), C.POINTER(C.c_size_t)]),
        "bddcso_setup": (C.c_int, [vp, vp, C.POINTER(Options), vp, C.c_size_t, vp, C.POINTER(vp)]),
        "bddcso_precond_generation": (C.c_int, [vp, i64p]),
        "bddcso_coef_from_log": (C.c_int, [vp, vp, vp, vp]),
        "bddcso_refactor": (C.c_int, [vp, vp, vp]),
        "bddcso_check_pivots": (C.c_int, [vp, vp]),
        "bddcso_operator_apply": (C.c_int, [vp, vp, vp, C.c_int, vp]),
        "bddcso_apply": (C.c_int, [vp, vp, vp, C.c_int, vp]),
        "bddcso_solve": (C.c_int, [vp, vp, vp, C.c_int, C.POINTER(Stats), vp]),
        "bddcso_solve_noalloc": (C.c_int, [vp, vp, vp, C.c_int, C.POINTER(Stats), vp]),
        "bddcso_element_grad": (C.c_int, [vp, vp, vp, vp, C.c_int, vp]),
        "bddcso_box_filter": (C.c_int, [vp, vp, vp, C.c_int, vp]),
        "bddcso_precond_info": (C.c_int, [vp, i64p, i64p, i64p, i64p]),
        "bddcso_local_coarse": (C.c_int, [vp, C.c_int, dp, i64p, C.c_int64, i64p, vp]),
        "bddcso_precond_destroy": (None, [vp]),
        "bddcso_problem_destroy": (None, [vp]),
        "bddcso_last_error": (C.c_char_p, []),
        "bddcso_plan_info": (C.c_int, [vp, C.POINTER(Options), C.POINTER(PlanStats)]),
        "bddcso_profile": (C.c_int, [vp, C.c_int]),
        "bddcso_copy_probe": (C.c_int, [vp, vp, C.c_int64, vp]),
        "bddcso_profile_read": (C.c_int, [vp, C.c_int, i64p, dp, dp, dp]),
        "bddcso_profile_reference": (C.c_int, [vp, C.c_int, dp, dp]),
        "bddcso_autotune": (C.c_int, [vp, vp, C.POINTER(Options), vp, C.c_int, vp, C.POINTER(Options),
                                      C.POINTER(TuneReport)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != 0:
        msg = load().bddcso_last_error().decode(errors="replace")
        raise BDDCSOError(status, msg)
