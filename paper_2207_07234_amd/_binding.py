"""ctypes binding of libpdhg.so (the C ABI declared in include/pdhg.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch supplies device memory and the current stream.  Importing this module
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdhg.so")

PDHG_OK, PDHG_NOT_CONVERGED, PDHG_DIVERGED, PDHG_STALLED = 0, 1, 2, 3
PDHG_EINVAL, PDHG_EHIP, PDHG_EUNSUPPORTED, PDHG_EWORKSPACE = -1, -2, -3, -4
PDHG_F32, PDHG_F64 = 0, 1
PDHG_BE, PDHG_BDF2 = 0, 1
PDHG_FD_UPWIND, PDHG_FD_LF, PDHG_DG_P2_LLF, PDHG_DG_P1_UPWIND = 0, 1, 2, 3
PDHG_PRECOND_GRAM, PDHG_PRECOND_FULL, PDHG_PRECOND_GRAM_F32 = 0, 1, 2
PDHG_ADJ_APPLY, PDHG_ADJ_SOLVE = 0, 1


class pdhg_problem(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("nt", C.c_int32),
        ("length", C.c_double), ("t_final", C.c_double),
        ("alpha", C.c_double), ("beta", C.c_double), ("gamma", C.c_double),
        ("time", C.c_int32), ("space", C.c_int32), ("dtype", C.c_int32), ("precond_kind", C.c_int32),
        ("lf_speed", C.c_double), ("precond_c", C.c_double), ("precond_gamma_hat", C.c_double),
    ]


class pdhg_params(C.Structure):
    _fields_ = [
        ("tau_u", C.c_double), ("tau_phi", C.c_double), ("eps", C.c_double),
        ("max_iter", C.c_int64), ("check_every", C.c_int32), ("warm_start", C.c_int32),
        ("diverge_factor", C.c_double), ("variant", C.c_int32), ("backoff", C.c_int32),
        ("history", C.c_void_p), ("eps_rel", C.c_double), ("stall_iters", C.c_int32),
        ("init_multiplier", C.c_int32), ("tau_u0", C.c_double), ("tau_lam", C.c_double),
    ]


class pdhg_stats(C.Structure):
    _fields_ = [
        ("iters", C.c_int64), ("res_primal", C.c_double), ("res_dual", C.c_double),
        ("tau_u", C.c_double), ("tau_phi", C.c_double), ("nu_max", C.c_double),
        ("lf_speed", C.c_double), ("precond_c", C.c_double), ("seconds", C.c_double),
        ("mass_drift", C.c_double), ("status", C.c_int32), ("variant", C.c_int32),
    ]


class pdhg_refine_params(C.Structure):
    _fields_ = [
        ("nt_start", C.c_int32), ("reserved", C.c_int32), ("coarse_max_iter", C.c_int64), ("coarse_eps", C.c_double),
    ]


class pdhg_batch_params(C.Structure):
    _fields_ = [
        ("tau_u", C.c_void_p), ("tau_phi", C.c_void_p), ("eps", C.c_double),
        ("max_iter", C.c_int64), ("check_every", C.c_int32), ("warm_start", C.c_int32),
        ("diverge_factor", C.c_double),
    ]


EXPORTED = (
    "pdhg_setup", "pdhg_workspace_bytes", "pdhg_solve", "pdhg_solve_refined", "pdhg_solve_onestep", "pdhg_residual", "pdhg_residual_static", "pdhg_precond",
    "pdhg_adjoint", "pdhg_time_kernel", "pdhg_destroy", "pdhg_status_string", "pdhg_last_error",
    "pdhg_batch_setup", "pdhg_batch_sizes", "pdhg_batch_offsets", "pdhg_batch_solve", "pdhg_batch_solve_onestep", "pdhg_batch_tune",
    "pdhg_batch_time_kernel", "pdhg_batch_destroy", "pdhg_batch_last_error",
)


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(
            f"HIP library {path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "or `make -C paper_2207_07234_amd/csrc`")
    lib = C.CDLL(path)
    H = C.c_void_p
    vp = C.c_void_p
    lib.pdhg_setup.argtypes = [C.POINTER(pdhg_problem), C.POINTER(H)]
    lib.pdhg_setup.restype = C.c_int
    lib.pdhg_workspace_bytes.argtypes = [H]
    lib.pdhg_workspace_bytes.restype = C.c_size_t
    lib.pdhg_solve.argtypes = [H, vp, vp, vp, vp, C.POINTER(pdhg_params), C.POINTER(pdhg_stats), vp]
    lib.pdhg_solve.restype = C.c_int
    lib.pdhg_solve_refined.argtypes = [H, vp, vp, vp, vp, C.POINTER(pdhg_params), C.POINTER(pdhg_refine_params),
                                       C.POINTER(pdhg_stats), C.POINTER(C.c_int64), vp]
    lib.pdhg_solve_refined.restype = C.c_int
    lib.pdhg_solve_onestep.argtypes = [H, vp, vp, vp, C.POINTER(pdhg_params), C.POINTER(pdhg_stats),
                                       C.POINTER(C.c_int64), C.POINTER(C.c_double), vp]
    lib.pdhg_solve_onestep.restype = C.c_int
    lib.pdhg_residual.argtypes = [H, vp, vp, vp, vp, C.POINTER(C.c_double), vp]
    lib.pdhg_residual.restype = C.c_int
    lib.pdhg_residual_static.argtypes = [H, vp, vp, vp, vp, C.POINTER(C.c_double), vp]
    lib.pdhg_residual_static.restype = C.c_int
    lib.pdhg_precond.argtypes = [H, vp, vp, vp]
    lib.pdhg_precond.restype = C.c_int
    lib.pdhg_adjoint.argtypes = [H, C.c_int32, vp, vp, vp, vp, vp, vp]
    lib.pdhg_adjoint.restype = C.c_int
    lib.pdhg_time_kernel.argtypes = [H, C.c_int32, C.c_int32, C.POINTER(C.c_double), vp]
    lib.pdhg_time_kernel.restype = C.c_int
    lib.pdhg_destroy.argtypes = [H]
    lib.pdhg_destroy.restype = None
    lib.pdhg_status_string.argtypes = [C.c_int]
    lib.pdhg_status_string.restype = C.c_char_p
    lib.pdhg_last_error.argtypes = [H]
    lib.pdhg_last_error.restype = C.c_char_p
    i64p = C.POINTER(C.c_int64)
    lib.pdhg_batch_setup.argtypes = [C.POINTER(pdhg_problem), C.c_int32, C.POINTER(H)]
    lib.pdhg_batch_setup.restype = C.c_int
    lib.pdhg_batch_sizes.argtypes = [H, i64p, i64p, i64p, C.POINTER(C.c_size_t)]
    lib.pdhg_batch_sizes.restype = C.c_int
    lib.pdhg_batch_offsets.argtypes = [H, C.c_int32, i64p, i64p, i64p]
    lib.pdhg_batch_offsets.restype = C.c_int
    lib.pdhg_batch_solve.argtypes = [H, vp, vp, vp, vp, C.POINTER(pdhg_batch_params), C.POINTER(pdhg_stats), vp]
    lib.pdhg_batch_solve.restype = C.c_int
    lib.pdhg_batch_solve_onestep.argtypes = [H, vp, vp, vp, C.POINTER(pdhg_batch_params), C.POINTER(pdhg_stats),
                                             C.POINTER(C.c_int64), vp]
    lib.pdhg_batch_solve_onestep.restype = C.c_int
    lib.pdhg_batch_tune.argtypes = [H, vp, vp, vp, vp, C.POINTER(pdhg_batch_params), C.POINTER(C.c_int32), vp]
    lib.pdhg_batch_tune.restype = C.c_int
    lib.pdhg_batch_time_kernel.argtypes = [H, C.c_int32, C.c_int32, C.POINTER(C.c_double), vp]
    lib.pdhg_batch_time_kernel.restype = C.c_int
    lib.pdhg_batch_destroy.argtypes = [H]
    lib.pdhg_batch_destroy.restype = None
    lib.pdhg_batch_last_error.argtypes = [H]
    lib.pdhg_batch_last_error.restype = C.c_char_p
    return lib


_LIB = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB
