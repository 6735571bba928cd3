"""ctypes declarations of the C ABI in include/cpm.h (argument marshalling only).

Loading fails loudly when the in-tree library is missing: there is no CPU or
Python fallback for any entry point.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpm.so")

CPM_OK = 0
STATUS = {0: "CPM_OK", 1: "CPM_ERR_ARG", 2: "CPM_ERR_BAND", 3: "CPM_ERR_PIVOT", 4: "CPM_ERR_DEVICE",
          5: "CPM_ERR_OOM", 6: "CPM_NOT_CONVERGED", 7: "CPM_ERR_STATE"}


class CpmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class Surface(C.Structure):
    _fields_ = [("kind", C.c_int32), ("params", C.c_double * 3), ("center", C.c_double * 3)]


class BandInfo(C.Structure):
    _fields_ = [("n_active", C.c_int64), ("n_ghost", C.c_int64), ("n_band", C.c_int64),
                ("d", C.c_int32), ("p", C.c_int32), ("h", C.c_double), ("gamma", C.c_double),
                ("lo", C.c_double * 3), ("shape", C.c_int32 * 3), ("n_bricks", C.c_int64),
                ("closure_iterations", C.c_int32), ("reach", C.c_int32)]


class PrecondOpts(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_parts", C.c_int32), ("overlap", C.c_double),
                ("alpha", C.c_double), ("alpha_cross", C.c_double), ("subsolver", C.c_int32),
                ("precision", C.c_int32), ("transpose", C.c_int32), ("ordering", C.c_int32),
                ("coarse", C.c_int32)]


class PrecondInfo(C.Structure):
    _fields_ = [("n_parts", C.c_int32), ("total_rows", C.c_int64), ("total_nnz", C.c_int64),
                ("max_rows", C.c_int32), ("max_levels", C.c_int32), ("precision", C.c_int32),
                ("kind", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("rtol", C.c_double), ("atol", C.c_double),
                ("max_it", C.c_int32), ("mode", C.c_int32), ("transpose", C.c_int32),
                ("use_graph", C.c_int32), ("inner_rtol", C.c_double), ("stagnation_cycles", C.c_int32),
                ("profile", C.c_int32), ("poly_n", C.c_int32), ("poly_coef", C.c_double * 5),
                ("pc_power", C.c_int32), ("pc_inner_rtol", C.c_double), ("pc_inner_max_it", C.c_int32)]


class OperatorOpts(C.Structure):
    _fields_ = [("order", C.c_int32), ("apply_lds_bytes", C.c_int32)]


class OperatorInfo(C.Structure):
    _fields_ = [("order", C.c_int32), ("two_kernel", C.c_int32), ("two_pass", C.c_int32),
                ("apply_lds_bytes", C.c_int32), ("n_tiles", C.c_int32), ("n_fallback_tiles", C.c_int32),
                ("apply_variant", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("status", C.c_int32), ("relres", C.c_double), ("ms_total", C.c_double),
                ("ms_precond", C.c_double), ("ms_apply", C.c_double), ("n_precond", C.c_int32),
                ("n_apply", C.c_int32)]


class ImexOpts(C.Structure):
    _fields_ = [("scheme", C.c_int32), ("kind", C.c_int32), ("nspecies", C.c_int32), ("dt", C.c_double),
                ("mu", C.c_double * 2), ("F", C.c_double), ("k", C.c_double), ("tune", C.c_int32),
                ("rd", C.c_double * 3)]


class TuneResult(C.Structure):
    _fields_ = [("apply_variant", C.c_int32), ("schwarz_variant", C.c_int32), ("schwarz_threads", C.c_int32),
                ("schwarz_sleep", C.c_int32), ("apply_ms", C.c_double), ("precond_ms", C.c_double),
                ("from_cache", C.c_int32)]


P = C.c_void_p
I32 = C.c_int32
# int32 cb(int64 n, const double* x, double* cp, int32* flag, void* ctx)
CP_CALLBACK = C.CFUNCTYPE(C.c_int32, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double),
                          C.POINTER(C.c_int32), C.c_void_p)
I64 = C.c_int64
D = C.c_double

# (name, restype, argtypes) for every function declared in include/cpm.h
SIGNATURES = [
    ("cpm_band_build", I32, [C.POINTER(Surface), I32, D, I32, C.POINTER(D), C.POINTER(D), D, C.POINTER(P)]),
    ("cpm_band_build_user", I32, [CP_CALLBACK, P, I32, D, I32, C.POINTER(D), C.POINTER(D), D, C.POINTER(P)]),
    ("cpm_band_build_reach", I32, [C.POINTER(Surface), CP_CALLBACK, P, I32, D, I32, C.POINTER(D), C.POINTER(D), D,
                                   I32, C.POINTER(P)]),
    ("cpm_band_get_info", I32, [P, C.POINTER(BandInfo)]),
    ("cpm_band_export", I32, [P, P, P, P]),
    ("cpm_band_export_interp", I32, [P, P, P]),
    ("cpm_band_destroy", None, [P]),
    ("cpm_operator_create", I32, [P, D, P, C.POINTER(P)]),
    ("cpm_operator_opts_default", I32, [C.POINTER(OperatorOpts)]),
    ("cpm_operator_create_ex", I32, [P, D, C.POINTER(OperatorOpts), P, C.POINTER(P)]),
    ("cpm_operator_get_info", I32, [P, C.POINTER(OperatorInfo)]),
    ("cpm_operator_set_shift", I32, [P, D]),
    ("cpm_operator_get_shift", D, [P]),
    ("cpm_operator_n_active", I64, [P]),
    ("cpm_operator_destroy", None, [P]),
    ("cpm_extend_apply", I32, [P, P, P, P]),
    ("cpm_apply", I32, [P, P, P, I32, P]),
    ("cpm_apply_T", I32, [P, P, P, I32, P]),
    ("cpm_apply_T_noalloc", I32, [P, P, P, I32, P]),
    ("cpm_shift_gradient", I32, [P, P, P, I32, P, P]),
    ("cpm_poly_apply", I32, [P, I32, C.POINTER(D), P, P, I32, P]),
    ("cpm_precond_create", I32, [P, C.POINTER(PrecondOpts), C.POINTER(P)]),
    ("cpm_precond_get_info", I32, [P, C.POINTER(PrecondInfo)]),
    ("cpm_precond_export_partition", I32, [P, P, P, P]),
    ("cpm_precond_apply", I32, [P, P, P, I32, P]),
    ("cpm_precond_destroy", None, [P]),
    ("cpm_solve_opts_default", I32, [C.POINTER(SolveOpts)]),
    ("cpm_precond_opts_default", I32, [C.POINTER(PrecondOpts)]),
    ("cpm_solve", I32, [P, P, P, P, I32, C.POINTER(SolveOpts), C.POINTER(SolveStats), P]),
    ("cpm_batch_create", I32, [I32, C.POINTER(P), C.POINTER(P), C.POINTER(I32), C.POINTER(P)]),
    ("cpm_batch_solve", I32, [P, C.POINTER(P), C.POINTER(P), C.POINTER(SolveOpts), C.POINTER(SolveStats), P]),
    ("cpm_batch_apply", I32, [P, C.POINTER(P), C.POINTER(P), P]),
    ("cpm_batch_destroy", None, [P]),
    ("cpm_autotune", I32, [P, P, I32, C.c_char_p, I32, P, C.POINTER(TuneResult)]),
    ("cpm_batch_autotune", I32, [P, C.c_char_p, I32, P, C.POINTER(TuneResult)]),
    ("cpm_gray_scott_rhs", I32, [I64, P, P, D, D, D, D, D, P, P, P]),
    ("cpm_imex_opts_default", I32, [C.POINTER(ImexOpts)]),
    ("cpm_imex_shift", D, [C.POINTER(ImexOpts), I32]),
    ("cpm_imex_create", I32, [C.POINTER(P), C.POINTER(P), C.POINTER(ImexOpts), C.POINTER(P), C.POINTER(P)]),
    ("cpm_imex_step", I32, [P, D, C.POINTER(P), I32, C.POINTER(SolveOpts), C.POINTER(SolveStats), P]),
    ("cpm_imex_destroy", None, [P]),
    ("cpm_last_error", C.c_char_p, []),
    ("cpm_version", I32, []),
    ("cpm_device_count", I32, []),
    ("cpm_abi_sizeof", I64, [I32]),
]

# ctypes mirrors of the public structs, in the order cpm_abi_sizeof numbers them
ABI_STRUCTS = [SolveOpts, SolveStats, PrecondOpts, TuneResult, ImexOpts, BandInfo, OperatorOpts, OperatorInfo]

_lib = None


def lib():
    """The loaded library; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code: int):
    if code != CPM_OK:
        raise CpmError(code, lib().cpm_last_error().decode(errors="replace"))
    return code
