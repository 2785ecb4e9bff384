"""ctypes binding of librr.so (argument marshalling only; no arithmetic here)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librr.so")

RR_OK = 0
STATUS_NAMES = {0: "RR_OK", 1: "RR_ERR_INVALID", 2: "RR_ERR_SINGULAR", 3: "RR_ERR_NOT_CONVERGED",
                4: "RR_ERR_BREAKDOWN", 5: "RR_ERR_NONFINITE", 6: "RR_ERR_NOMEM", 7: "RR_ERR_HIP",
                8: "RR_ERR_TIMEOUT"}
RR_FP64, RR_MIXED = 0, 1
RR_RESP_AV, RR_RESP_QU, RR_RESP_NONE = 0, 1, 2
TEST_MATRICES = {"gaussian": 0, "rademacher": 1, "sparse": 2, "orthonormal": 3}
REFINE_METHODS = {"plain": 0, "gmres": 1}
SOLVERS = {"lu": 0, "bicgstab": 1, "gmres": 2}
PRECONDS = {"jacobi": 0, "ilu0": 1}

# every symbol include/rr.h declares (the last three are test hooks)
EXPORTS = ("rr_burgers_coeffs", "rr_apply", "rr_factor", "rr_refactor", "rr_sketch_solve",
           "rr_adjoint_solve", "rr_solve", "rr_gains", "rr_resvd", "rr_grad", "rr_check", "rr_refine_count",
           "rr_bytes", "rr_factors_free", "rr_set_allocator", "rr_factor_bytes", "rr_graph_capture",
           "rr_graph_launch", "rr_graph_free", "rr_autotune", "rr_last_error", "rr_philox_raw",
           "rr_sketch", "rr_factor_schedule", "rr_set_test_matrix", "rr_set_jacobi_sweeps",
           "rr_grad_noalloc", "rr_set_timing_events", "rr_precond_apply")


class RRError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("coef", ctypes.c_void_p), ("phi", ctypes.c_void_p), ("U", ctypes.c_void_p),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double),
                ("y1", ctypes.c_double), ("nu", ctypes.c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Tuning(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("refine_iters", ctypes.c_int32), ("refine_tol", ctypes.c_double),
                ("refine_tol_sketch", ctypes.c_double), ("refine_method", ctypes.c_int32),
                ("gmres_restart", ctypes.c_int32), ("superblock", ctypes.c_int32),
                ("solver", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("krylov_maxit", ctypes.c_int32), ("krylov_tol", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load librr.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1902_01458_amd.build` (there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                              ctypes.c_double)
    pp = ctypes.POINTER(Problem)
    sig = {
        "rr_burgers_coeffs": [i32, i32, vp, dbl, dbl, dbl, dbl, dbl, vp, vp, vp],
        "rr_apply": [pp, vp, vp, i32, i32, i32, vp, vp, vp],
        "rr_factor": [pp, vp, vp, i32, i32, ctypes.c_int, ctypes.POINTER(Tuning), vp,
                      ctypes.POINTER(vp)],
        "rr_refactor": [vp, vp],
        "rr_sketch_solve": [vp, i32, u64, i32, vp, vp],
        "rr_adjoint_solve": [vp, i32, vp, vp, vp],
        "rr_solve": [vp, i32, vp, vp, vp],
        "rr_gains": [vp, i32, vp, vp, ctypes.c_int, vp, vp, vp, vp, vp],
        "rr_resvd": [vp, i32, vp, vp, vp, vp, vp, vp, vp],
        "rr_grad": [vp, vp, vp, vp, i64, vp, vp, vp, vp],
        "rr_grad_noalloc": [pp, i32, vp, vp, vp, i64, vp, vp, vp, vp],
        "rr_check": [vp, vp],
        "rr_refine_count": [vp],
        "rr_bytes": [vp],
        "rr_factors_free": [vp],
        "rr_last_error": [],
        "rr_philox_raw": [vp, i64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                          ctypes.c_uint32, vp],
        "rr_sketch": [pp, i32, u64, ctypes.c_int, i32, vp, vp],
        "rr_set_test_matrix": [vp, ctypes.c_int, i32],
        "rr_set_jacobi_sweeps": [vp, i32],
        "rr_set_timing_events": [vp, vp, vp, vp, vp],
        "rr_precond_apply": [vp, i32, i32, vp, vp, vp],
        "rr_factor_bytes": [i32, i32, i32, i32, ctypes.c_int, i32],
        "rr_factor_schedule": [i32, i32, vp, i64],
        "rr_set_allocator": [ALLOC_FN, FREE_FN, vp],
        "rr_graph_capture": [vp, i32, i32, u64, i32, ctypes.c_int, vp, vp, vp, vp, vp, vp,
                             ctypes.POINTER(vp)],
        "rr_graph_launch": [vp, vp],
        "rr_graph_free": [vp],
        "rr_autotune": [pp, vp, vp, i32, i32, ctypes.c_int, i32, vp, ctypes.POINTER(Tuning),
                        ctypes.POINTER(dbl)],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.rr_last_error.restype = ctypes.c_char_p
    L.rr_bytes.restype = ctypes.c_size_t
    L.rr_factors_free.restype = None
    L.rr_factor_bytes.restype = ctypes.c_size_t
    L.rr_graph_free.restype = None
    L.rr_refine_count.restype = ctypes.c_int32
    L.rr_factor_schedule.restype = ctypes.c_int64
    _lib = L
    return L


def check(status: int):
    if status != RR_OK:
        raise RRError(status, lib().rr_last_error().decode())
