"""ctypes declarations mirroring include/clr.h (no logic beyond marshalling)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libclr_mi355x.so")

CLR_OK = 0
CLR_ERR_INVALID_ARG = 1
CLR_ERR_SHAPE = 2
CLR_ERR_CAPACITY = 3
CLR_ERR_NONFINITE = 4
CLR_ERR_NOT_CONVERGED = 5
CLR_ERR_HIP = 6
CLR_ERR_NORM_MISMATCH = 7
CLR_ERR_DIVERGED = 8
CLR_ERR_INTERNAL = 9

CLR_FP64 = 0
CLR_COMPRESS_SVD, CLR_COMPRESS_RRQR = 0, 1
CLR_KERNEL_GAUSSIAN, CLR_KERNEL_COULOMB = 0, 1
CLR_MIXED = 1
CLR_OZAKI = 2
CLR_SCREEN_ABS = 0
CLR_SCREEN_AREA = 1

# Every function declared in include/clr.h.
EXPORTS = [
    "clr_context_create", "clr_context_destroy", "clr_set_allocator", "clr_last_error",
    "clr_status_string",
    "clr_create", "clr_compress", "clr_destroy", "clr_matrix_info", "clr_matrix_arena",
    "clr_compact", "clr_get_meta",
    "clr_get_block", "clr_to_dense", "clr_gemm", "clr_axpby", "clr_sqrt_inv",
    "clr_identity_residual", "clr_identity_residual_noalloc", "clr_gemm_backward", "clr_sqrt_inv_backward",
    "clr_plan_create", "clr_plan_execute", "clr_plan_destroy", "clr_gemm_batch",
    "clr_set_tile_edges", "clr_set_tile_classes", "clr_get_tile_classes", "clr_autotune",
    "clr_set_dense_certificate", "clr_set_compression",
    "clr_kernel_matrix", "clr_measure_peaks",
]


class GemmOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("eps_sp", C.c_double), ("screen", C.c_int),
                ("precision", C.c_int), ("split", C.c_int), ("alpha", C.c_double)]


class SqrtInvOpts(C.Structure):
    _fields_ = [("g", GemmOpts), ("alpha", C.c_double), ("conv_tol", C.c_double),
                ("max_iter", C.c_int), ("fixed_iters", C.c_int), ("reduced_below", C.c_double),
                ("correction", C.c_int), ("graph", C.c_int), ("graph_margin", C.c_double)]


# clr_set_allocator callbacks: alloc(bytes, stream, user) -> ptr, release(ptr, bytes, stream, user)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class GemmStats(C.Structure):
    _fields_ = [("candidates", C.c_int64), ("computed", C.c_int64), ("dropped", C.c_int64),
                ("triples", C.c_int64), ("n_dd", C.c_int64), ("n_ld", C.c_int64),
                ("n_dl", C.c_int64), ("n_ll", C.c_int64), ("out_dense", C.c_int64),
                ("out_lowrank", C.c_int64), ("densified", C.c_int64),
                ("flops_dd", C.c_double), ("flops_ld", C.c_double), ("flops_dl", C.c_double),
                ("flops_ll", C.c_double), ("flops_densify", C.c_double),
                ("flops_products", C.c_double), ("bytes_compulsory", C.c_double),
                ("ms_symbolic", C.c_double), ("ms_products", C.c_double),
                ("ms_recompress", C.c_double), ("ms_total", C.c_double),
                ("ms_thin", C.c_double), ("ms_dense", C.c_double),
                ("flops_rec_engine", C.c_double), ("ms_rec_engine", C.c_double),
                ("certified_dense", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SqrtInvStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("alpha", C.c_double),
                ("internal_residual", C.c_double), ("explicit_residual", C.c_double),
                ("n_gemms", C.c_int), ("flops_products", C.c_double), ("ms_total", C.c_double),
                ("graph_replays", C.c_int), ("graph_captures", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ClrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"clr status {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library with "
            "`python -m paper_1509_00309_amd.build` (there is no CPU fallback)")
    h = C.CDLL(LIB_PATH)
    P = C.c_void_p
    I64 = C.c_int64
    D = C.c_double
    IP = C.POINTER(C.c_int)
    DP = C.POINTER(C.c_double)
    sig = {
        "clr_context_create": [C.POINTER(P), P],
        "clr_context_destroy": [P],
        "clr_create": [P, C.c_int, IP, C.c_int, IP, C.POINTER(C.c_int8), IP, DP, C.POINTER(P),
                       C.POINTER(P), C.POINTER(P)],
        "clr_compress": [P, P, I64, C.c_int, IP, C.c_int, IP, D, D, C.POINTER(P)],
        "clr_destroy": [P],
        "clr_matrix_info": [P, IP, IP, C.POINTER(I64), C.POINTER(I64), C.POINTER(I64)],
        "clr_matrix_arena": [P, C.POINTER(I64), C.POINTER(C.c_size_t)],
        "clr_compact": [P, P],
        "clr_get_meta": [P, P, C.POINTER(C.c_int8), IP, DP],
        "clr_get_block": [P, P, C.c_int, C.c_int, P, P],
        "clr_to_dense": [P, P, P, I64],
        "clr_gemm": [P, P, P, C.POINTER(GemmOpts), C.POINTER(P), C.POINTER(GemmStats)],
        "clr_axpby": [P, D, P, D, P, D, C.POINTER(GemmOpts), C.POINTER(P)],
        "clr_sqrt_inv": [P, P, C.POINTER(SqrtInvOpts), C.POINTER(P), C.POINTER(SqrtInvStats)],
        "clr_identity_residual": [P, P, DP],
        "clr_identity_residual_noalloc": [P, P, P],
        "clr_measure_peaks": [P, DP, DP],
        "clr_gemm_backward": [P, P, P, D, P, I64, P, I64, P, I64],
        "clr_sqrt_inv_backward": [P, P, C.POINTER(SqrtInvOpts), C.c_int, C.c_int, P, P, I64,
                                  C.POINTER(P)],
        "clr_plan_create": [P, C.c_int, C.POINTER(P), C.POINTER(P), C.POINTER(GemmOpts), C.c_int,
                            C.POINTER(P), C.POINTER(P)],
        "clr_plan_execute": [P, P, C.POINTER(GemmStats)],
        "clr_plan_destroy": [P],
        "clr_set_tile_edges": [P, C.c_int, C.c_int, C.c_int],
        "clr_set_allocator": [P, ALLOC_FN, RELEASE_FN, P],
        "clr_set_tile_classes": [P, C.c_int, IP, IP],
        "clr_get_tile_classes": [P, C.c_int, IP, IP],
        "clr_set_dense_certificate": [P, C.c_int],
        "clr_set_compression": [P, C.c_int],
        "clr_kernel_matrix": [P, P, C.c_int64, P, C.c_int64, C.c_int, C.c_int, C.c_double,
                              C.c_double, P, C.c_int64],
        "clr_autotune": [P, P, P, C.POINTER(GemmOpts), IP, IP, DP, DP],
        "clr_gemm_batch": [P, C.c_int, C.POINTER(P), C.POINTER(P), C.POINTER(GemmOpts),
                           C.POINTER(P), C.POINTER(GemmStats)],
    }
    for name, args in sig.items():
        f = getattr(h, name)
        f.argtypes = args
        f.restype = C.c_int
    h.clr_last_error.argtypes = [P]
    h.clr_last_error.restype = C.c_char_p
    h.clr_status_string.argtypes = [C.c_int]
    h.clr_status_string.restype = C.c_char_p
    return h


lib = _load()


def check(rc, ctx_handle):
    if rc == CLR_OK:
        return
    msg = lib.clr_last_error(ctx_handle).decode() if ctx_handle else ""
    raise ClrError(rc, f"{lib.clr_status_string(rc).decode()}: {msg}")
