"""ctypes declarations of the C ABI in include/se.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libse.so")

SE_OK = 0
SE_NOT_CONVERGED = 1
SE_ERR_INVALID_ARG = -1
SE_ERR_OOM = -2
SE_ERR_HIP = -3
SE_ERR_BREAKDOWN = -4
SE_ERR_REJECTED = -5
SE_ERR_UNSUPPORTED = -6

SE_LOBPCG, SE_SI, SE_SD, SE_TRACEMIN = 0, 1, 2, 3
SOLVERS = {"lobpcg": SE_LOBPCG, "si": SE_SI, "sd": SE_SD, "tracemin": SE_TRACEMIN}
STRATEGIES = {"none": 0, "fix": 1, "slope": 2, "slopek": 3}
EXPAND_VECTORS = {"xdrop": 0, "random": 1, "powered": 2}
PRECONDS = {"none": 0, "jacobi": 1}
SE_FP64 = 0
SE_FP32_MIXED = 1
SE_BF16_MIXED = 2
SE_PTR_HOST, SE_PTR_DEVICE = 0, 1
SE_MATRIX_HOST, SE_MATRIX_DEVICE = 0, 1
SE_HISTORY_FIELDS = 8
KERNEL_CLASSES = ["spmm", "gram", "update", "resid", "eig", "small", "copy", "other"]


class SeParams(C.Structure):
    _fields_ = [
        ("solver", C.c_int32), ("strategy", C.c_int32), ("precision", C.c_int32),
        ("ptr_mode", C.c_int32), ("n_ev", C.c_int32), ("n_extra", C.c_int32),
        ("n_es", C.c_int32), ("soft_lock", C.c_int32), ("j_e", C.c_int32),
        ("j_s", C.c_int32), ("j_p", C.c_int32), ("j_warm", C.c_int32),
        ("max_iter", C.c_int32), ("profile", C.c_int32), ("mu", C.c_double),
        ("r_warm", C.c_double), ("tol", C.c_double), ("sigma", C.c_double),
        ("time_limit_s", C.c_double), ("r_switch", C.c_double), ("implicit_pivot", C.c_double),
        ("seed", C.c_uint64),
        ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int32),
        ("expand_vectors", C.c_int32), ("filter_degree", C.c_int32), ("cg_steps", C.c_int32),
        ("precond", C.c_int32), ("reserved", C.c_int32),
    ]


class SeInfo(C.Structure):
    _fields_ = [
        ("iterations", C.c_int32), ("converged", C.c_int32), ("n_shrinks", C.c_int32),
        ("n_expands", C.c_int32), ("max_stop_ratio", C.c_double),
        ("max_paper_ratio", C.c_double), ("time_ms", C.c_double),
        ("kern_ms", C.c_double * 8), ("kern_bytes", C.c_double * 8),
        ("kern_flops", C.c_double * 8), ("kern_calls", C.c_int32 * 8),
        ("workspace_bytes", C.c_uint64),
        ("hip_error", C.c_int32), ("history_len", C.c_int32),
        ("lp_iterations", C.c_int32), ("n_reprojections", C.c_int32),
    ]


_lib = None

# name -> (restype, argtypes)
PROTOTYPES = {
    "se_params_default": (None, [C.POINTER(SeParams)]),
    "se_ctx_create": (C.c_int, [C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    "se_ctx_destroy": (None, [C.c_void_p]),
    "se_matrix_create_csr": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_uint32, C.c_double,
                                        C.POINTER(C.c_void_p)]),
    "se_matrix_destroy": (None, [C.c_void_p]),
    "se_matrix_n": (C.c_int64, [C.c_void_p]),
    "se_matrix_anorm": (C.c_double, [C.c_void_p]),
    "se_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(SeParams), C.c_void_p, C.c_void_p,
                           C.c_void_p, C.POINTER(SeInfo)]),
    "se_op_spmm": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                             C.c_int64, C.c_int32]),
    "se_op_gram": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int32,
                             C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]),
    "se_op_gram_noalloc": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int32,
                                     C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]),
    "se_op_update": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int32,
                               C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_double]),
    "se_op_syev": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "se_op_spmm_lp": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                C.c_int64, C.c_int32]),
    "se_op_gram_lp": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_int64, C.c_int32,
                                C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]),
    "se_op_update_lp": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_int64, C.c_int32,
                                  C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_double]),
    "se_op_syev_lowest": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                    C.c_void_p]),
    "se_op_cholqr": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int32,
                               C.POINTER(C.c_int32)]),
    "se_solve_footprint": (C.c_uint64, [C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                        C.c_int32]),
    "se_server_create": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int32, C.POINTER(C.c_void_p)]),
    "se_ctx_last_hip_error": (C.c_int32, [C.c_void_p]),
    "se_hip_error_name": (C.c_char_p, [C.c_int32]),
    "se_server_create_batched": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int32, C.POINTER(C.c_void_p)]),
    "se_batched_footprint": (C.c_uint64, [C.c_int64, C.c_int32, C.c_int32]),
    "se_server_batch_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "se_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(SeParams), C.c_void_p, C.c_void_p,
                            C.c_void_p, C.POINTER(C.c_uint64)]),
    "se_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32)]),
    "se_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(SeInfo), C.POINTER(C.c_double),
                          C.POINTER(C.c_double)]),
    "se_server_destroy": (None, [C.c_void_p]),
    "se_strategy_replay": (C.c_int, [C.POINTER(SeParams), C.c_int32, C.POINTER(C.c_double),
                                     C.POINTER(C.c_int32)]),
    "se_status_string": (C.c_char_p, [C.c_int]),
    "se_matrix_create_csr_z": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_uint32, C.c_double,
                                          C.POINTER(C.c_void_p)]),
    "se_solve_z": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(SeParams), C.c_void_p, C.c_void_p,
                             C.c_void_p, C.POINTER(SeInfo)]),
    "se_op_spmm_z": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                               C.c_int64, C.c_int32]),
    "se_op_gram_z": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int32,
                               C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]),
    "se_op_update_z": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int32,
                                 C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_double]),
    "se_op_heev_lowest_z": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                      C.c_void_p]),
}


def lib():
    """Load libse.so (after torch, so both share one HIP runtime); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2409_05572_amd.build` "
            "(or __graft_entry__.build()); there is no CPU fallback"
        )
    try:
        import torch  # noqa: F401  (loads torch's HIP runtime first)
    except ImportError:
        pass
    h = C.CDLL(LIB_PATH, mode=C.RTLD_GLOBAL)
    for name, (res, args) in PROTOTYPES.items():
        f = getattr(h, name)
        f.restype = res
        f.argtypes = args
    _lib = h
    return h


class SeError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        msg = lib().se_status_string(status).decode()
        super().__init__(f"{what}: status {status} ({msg})" if what else f"status {status} ({msg})")
        self.status = status


def check(status: int, what: str = "") -> int:
    if status < 0:
        raise SeError(status, what)
    return status
