"""Python binding of the MI355X CLR block-product library (libclr_mi355x.so).

Argument marshalling only: every step of the product, the recompression and
the square-root inverse runs in the library's HIP kernels.  PyTorch supplies
device memory (input/output tensors) and the stream.  Importing this package
loads the shared library and fails loudly if it has not been built
(``python -m paper_1509_00309_amd.build``).
"""
from __future__ import annotations

import atexit
import sys
import ctypes as C
import os
from dataclasses import dataclass
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

from . import _abi
from ._abi import (CLR_FP64, CLR_MIXED, CLR_OZAKI, CLR_SCREEN_ABS, CLR_SCREEN_AREA, ClrError,
                   GemmOpts, GemmStats, SqrtInvOpts, SqrtInvStats, lib, LIB_PATH)

__all__ = [
    "Context", "CLRMatrix", "ClrError", "GemmStats", "SqrtInvStats", "lib", "LIB_PATH",
    "CLR_FP64", "CLR_MIXED", "CLR_OZAKI", "gemm_dense", "sqrt_inv_dense", "Plan",
]


def _torch():
    import torch
    return torch


def _col_major(t):
    """A column-major copy of a 2-D float64 CUDA tensor: returns (buffer, ld)."""
    torch = _torch()
    if t.dtype != torch.float64:
        raise TypeError("float64 tensors are required")
    if not t.is_cuda:
        raise TypeError("device (cuda) tensors are required")
    buf = t.t().contiguous()            # (cols, rows) row-major == (rows, cols) column-major
    return buf, t.shape[0]


def _gemm_opts(tol, eps_sp, screen, precision, split, alpha) -> GemmOpts:
    o = GemmOpts()
    o.tol = float(tol)
    o.eps_sp = float(eps_sp)
    o.screen = {"abs": CLR_SCREEN_ABS, "area": CLR_SCREEN_AREA}[screen] if isinstance(screen, str) else int(screen)
    o.precision = ({"fp64": CLR_FP64, "mixed": CLR_MIXED, "ozaki": CLR_OZAKI}[precision]
                   if isinstance(precision, str) else int(precision))
    o.split = int(split)
    o.alpha = float(alpha)
    return o


# Set at interpreter exit, before objects are collected: callbacks into torch's allocator
# stop then (see Context.use_torch_allocator).
_FINALIZING = [False]
atexit.register(lambda: _FINALIZING.__setitem__(0, True))


class Context:
    """A library context bound to the current device and a torch stream."""

    def __init__(self, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("the CLR library needs a ROCm GPU")
        self.device = torch.cuda.current_device()
        s = stream if stream is not None else torch.cuda.current_stream()
        self._stream = s
        h = C.c_void_p()
        _abi.check(lib.clr_context_create(C.byref(h), C.c_void_p(s.cuda_stream)), None)
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib.clr_context_destroy(self._h)
            self._h = None

    def use_torch_allocator(self, enable: bool = True):
        """Back this context's matrices and work lists with torch's caching allocator
        (clr_set_allocator) on the context's stream; enable=False returns to hipMalloc.
        The callbacks allocate and release through torch.cuda.caching_allocator_alloc /
        caching_allocator_delete; they are kept alive by the context object."""
        torch = _torch()
        if not enable:
            self._check(lib.clr_set_allocator(self._h, None, None, None))
            self._alloc_cbs = None
            return
        device = self.device

        def _alloc(nbytes, stream, user):
            if _FINALIZING[0] or sys.is_finalizing():
                return None
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream or 0)
            except RuntimeError:
                return None

        def _release(ptr, nbytes, stream, user):
            # once the interpreter is shutting down torch's allocator may already be gone:
            # the process is ending, so the memory is left to the driver
            if _FINALIZING[0] or sys.is_finalizing():
                return
            torch.cuda.caching_allocator_delete(ptr)

        cbs = (_abi.ALLOC_FN(_alloc), _abi.RELEASE_FN(_release))
        self._check(lib.clr_set_allocator(self._h, cbs[0], cbs[1], None))
        self._alloc_cbs = cbs

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        _abi.check(rc, self._h)

    # -- matrices ------------------------------------------------------------
    def create(self, row_sizes: Sequence[int], col_sizes: Sequence[int], kind, rank,
               f0: Dict[Tuple[int, int], object], f1: Dict[Tuple[int, int], object],
               norms=None) -> "CLRMatrix":
        """CLR matrix from per-block factors (torch float64 cuda tensors, any 2-D layout).

        kind/rank: (nrb, ncb) arrays; f0[(I,J)] dense m x n or U m x r; f1[(I,J)] V n x r.
        """
        nrb, ncb = len(row_sizes), len(col_sizes)
        kind = np.ascontiguousarray(np.asarray(kind, dtype=np.int8).reshape(nrb, ncb))
        rank = np.ascontiguousarray(np.asarray(rank, dtype=np.int32).reshape(nrb, ncb))
        keep = []
        p0 = (C.c_void_p * (nrb * ncb))()
        p1 = (C.c_void_p * (nrb * ncb))()
        for i in range(nrb):
            for j in range(ncb):
                if kind[i, j] == 0:
                    continue
                b0, _ = _col_major(f0[(i, j)])
                keep.append(b0)
                p0[i * ncb + j] = b0.data_ptr()
                if kind[i, j] == 2:
                    b1, _ = _col_major(f1[(i, j)])
                    keep.append(b1)
                    p1[i * ncb + j] = b1.data_ptr()
        rs = (C.c_int * nrb)(*map(int, row_sizes))
        cs = (C.c_int * ncb)(*map(int, col_sizes))
        nptr = None
        if norms is not None:
            nrm = np.ascontiguousarray(np.asarray(norms, dtype=np.float64).reshape(nrb, ncb))
            keep.append(nrm)
            nptr = nrm.ctypes.data_as(C.POINTER(C.c_double))
        h = C.c_void_p()
        self._check(lib.clr_create(self._h, nrb, rs, ncb, cs,
                                   kind.ctypes.data_as(C.POINTER(C.c_int8)),
                                   rank.ctypes.data_as(C.POINTER(C.c_int)), nptr, p0, p1,
                                   C.byref(h)))
        return CLRMatrix(self, h)

    def compress(self, dense, row_sizes, col_sizes, tol: float, drop: float,
                 method: str = "svd") -> "CLRMatrix":
        """CLR form of a dense float64 cuda matrix, each block truncated by its SVD or, with
        method="rrqr", by the paper's column-pivoted QR (see clr.h)."""
        buf, ld = _col_major(dense)
        nrb, ncb = len(row_sizes), len(col_sizes)
        rs = (C.c_int * nrb)(*map(int, row_sizes))
        cs = (C.c_int * ncb)(*map(int, col_sizes))
        h = C.c_void_p()
        code = {"svd": _abi.CLR_COMPRESS_SVD, "rrqr": _abi.CLR_COMPRESS_RRQR}[method]
        self._check(lib.clr_set_compression(self._h, code))
        try:
            self._check(lib.clr_compress(self._h, C.c_void_p(buf.data_ptr()), C.c_int64(ld), nrb,
                                         rs, ncb, cs, C.c_double(tol), C.c_double(drop),
                                         C.byref(h)))
        finally:
            lib.clr_set_compression(self._h, _abi.CLR_COMPRESS_SVD)
        return CLRMatrix(self, h)

    def kernel_matrix(self, points, kernel: str = "gaussian", a: float = 0.3, diag: float = 0.0,
                      col_points=None):
        """Dense kernel matrix generated on the device (see clr.h): exp(-a r^2) ("gaussian") or
        1 / sqrt(r^2 + a^2) ("coulomb"), plus diag where i == j.  points: (n, dim) float64
        cuda tensor; col_points (default: points) gives the columns.  Returns an
        (n, n_cols) float64 cuda tensor (a transposed view of column-major storage)."""
        torch = _torch()
        x = points.contiguous()
        y = x if col_points is None else col_points.contiguous()
        for t in (x, y):
            if t.dtype != torch.float64 or not t.is_cuda or t.dim() != 2:
                raise TypeError("points must be 2-D float64 cuda tensors")
        if x.shape[1] != y.shape[1]:
            raise ValueError("row and column points differ in dimension")
        nr, nc = x.shape[0], y.shape[0]
        out = torch.empty((nc, nr), dtype=torch.float64, device=x.device)
        code = {"gaussian": _abi.CLR_KERNEL_GAUSSIAN, "coulomb": _abi.CLR_KERNEL_COULOMB}[kernel]
        self._check(lib.clr_kernel_matrix(self._h, C.c_void_p(x.data_ptr()), C.c_int64(nr),
                                          C.c_void_p(y.data_ptr()), C.c_int64(nc),
                                          int(x.shape[1]), code, C.c_double(a), C.c_double(diag),
                                          C.c_void_p(out.data_ptr()), C.c_int64(nr)))
        return out.t()

    # -- the method ----------------------------------------------------------
    def gemm(self, A: "CLRMatrix", B: "CLRMatrix", tol: float, eps_sp: float, screen="abs",
             precision="fp64", split: int = 0, alpha: float = 1.0, stats: bool = False):
        o = _gemm_opts(tol, eps_sp, screen, precision, split, alpha)
        h = C.c_void_p()
        st = GemmStats()
        self._check(lib.clr_gemm(self._h, A._h, B._h, C.byref(o), C.byref(h), C.byref(st) if stats else None))
        M = CLRMatrix(self, h)
        return (M, st) if stats else M

    def axpby(self, a: float, X: "CLRMatrix", b: float, Y: Optional["CLRMatrix"], c: float,
              tol: float, eps_sp: float, screen="abs", precision="fp64") -> "CLRMatrix":
        o = _gemm_opts(tol, eps_sp, screen, precision, 0, 1.0)
        h = C.c_void_p()
        self._check(lib.clr_axpby(self._h, C.c_double(a), X._h, C.c_double(b),
                                  Y._h if Y is not None else None, C.c_double(c), C.byref(o),
                                  C.byref(h)))
        return CLRMatrix(self, h)

    def sqrt_inv(self, S: "CLRMatrix", tol: float, eps_sp: float, conv_tol: float = 1e-10,
                 max_iter: int = 50, fixed_iters: int = 0, alpha: float = 0.0, screen="abs",
                 precision="fp64", split: int = 0, allow_not_converged: bool = False,
                 reduced_below: float = 0.0, correction: bool = False, graph: bool = False,
                 graph_margin: float = 0.0):
        """W = S^-1/2 (Newton-Schulz, Eqs. (8)-(11)); returns (W, SqrtInvStats).

        An iteration that stops without meeting conv_tol raises ClrError
        (CLR_ERR_NOT_CONVERGED) unless allow_not_converged is set; then W is
        returned and SqrtInvStats.converged is 0.  reduced_below / correction:
        the precision schedule of the reduced-precision forms; graph /
        graph_margin: iterations replayed from a recorded HIP graph (see clr.h)."""
        o = SqrtInvOpts()
        o.g = _gemm_opts(tol, eps_sp, screen, precision, split, 1.0)
        o.alpha = float(alpha)
        o.conv_tol = float(conv_tol)
        o.max_iter = int(max_iter)
        o.fixed_iters = int(fixed_iters)
        o.reduced_below = float(reduced_below)
        o.correction = 1 if correction else 0
        o.graph = 1 if graph else 0
        o.graph_margin = float(graph_margin)
        h = C.c_void_p()
        st = SqrtInvStats()
        rc = lib.clr_sqrt_inv(self._h, S._h, C.byref(o), C.byref(h), C.byref(st))
        if rc == _abi.CLR_ERR_NOT_CONVERGED and allow_not_converged and h.value:
            return CLRMatrix(self, h), st
        self._check(rc)
        return CLRMatrix(self, h), st

    # -- launch shapes -----------------------------------------------------------
    def set_tile_edges(self, precision="fp64", dense_edge: int = 0, thin_edge: int = 0):
        prec = {"fp64": CLR_FP64, "mixed": CLR_MIXED}[precision]
        self._check(lib.clr_set_tile_edges(self._h, prec, int(dense_edge), int(thin_edge)))

    def set_dense_certificate(self, enable: bool = True):
        """Prove dense-accumulated blocks dense from their Gram matrix before the SVD."""
        self._check(lib.clr_set_dense_certificate(self._h, 1 if enable else 0))

    def autotune(self, A: "CLRMatrix", B: "CLRMatrix", tol: float, eps_sp: float, screen="abs",
                 precision="fp64", split: int = 0) -> dict:
        """Pick the grouped-GEMM item edges for this context by timing A B."""
        o = _gemm_opts(tol, eps_sp, screen, precision, split, 1.0)
        de, te = C.c_int(), C.c_int()
        md, mt = C.c_double(), C.c_double()
        self._check(lib.clr_autotune(self._h, A._h, B._h, C.byref(o), C.byref(de), C.byref(te),
                                     C.byref(md), C.byref(mt)))
        dense, thin = self.get_tile_classes(precision)
        return {"dense_edge": de.value, "thin_edge": te.value, "ms_dense": md.value,
                "ms_thin": mt.value, "dense_classes": dense, "thin_classes": thin}

    # Shape classes of the item edges (clr.h): dense items by their block's longer edge
    # (<=32, <=64, <=96, <=128, <=160, >160), factor-product items by their rank
    # (<=8, <=16, <=32, <=64, >64).
    DENSE_CLASSES = 6
    THIN_CLASSES = 5

    def set_tile_classes(self, precision, dense_edges, thin_edges):
        prec = {"fp64": CLR_FP64, "mixed": CLR_MIXED}[precision]
        d = (C.c_int * self.DENSE_CLASSES)(*[int(v) for v in dense_edges])
        t = (C.c_int * self.THIN_CLASSES)(*[int(v) for v in thin_edges])
        self._check(lib.clr_set_tile_classes(self._h, prec, d, t))

    def get_tile_classes(self, precision="fp64"):
        prec = {"fp64": CLR_FP64, "mixed": CLR_MIXED}[precision]
        d = (C.c_int * self.DENSE_CLASSES)()
        t = (C.c_int * self.THIN_CLASSES)()
        self._check(lib.clr_get_tile_classes(self._h, prec, d, t))
        return list(d), list(t)

    # -- batches of products ----------------------------------------------------
    def plan(self, As: Sequence["CLRMatrix"], Bs: Sequence["CLRMatrix"], tol: float,
             eps_sp: float, screen="abs", precision="fp64", split: int = 0,
             alpha: float = 1.0, graph: bool = False) -> "Plan":
        """Plan C_p = A_p B_p for all p; execute() computes every product of the batch."""
        if len(As) != len(Bs) or not As:
            raise ValueError("need equally many (and at least one) A and B operands")
        n = len(As)
        o = _gemm_opts(tol, eps_sp, screen, precision, split, alpha)
        pa = (C.c_void_p * n)(*[a._h.value for a in As])
        pb = (C.c_void_p * n)(*[b._h.value for b in Bs])
        pc = (C.c_void_p * n)()
        h = C.c_void_p()
        self._check(lib.clr_plan_create(self._h, n, pa, pb, C.byref(o), int(bool(graph)),
                                        C.byref(h), pc))
        outs = [CLRMatrix(self, C.c_void_p(pc[i])) for i in range(n)]
        return Plan(self, h, outs, list(As), list(Bs))

    def gemm_batch(self, As, Bs, tol: float, eps_sp: float, screen="abs", precision="fp64",
                   split: int = 0, alpha: float = 1.0, stats: bool = False):
        """C_p = A_p B_p for all p, one launch per phase for the whole batch."""
        n = len(As)
        o = _gemm_opts(tol, eps_sp, screen, precision, split, alpha)
        pa = (C.c_void_p * n)(*[a._h.value for a in As])
        pb = (C.c_void_p * n)(*[b._h.value for b in Bs])
        pc = (C.c_void_p * n)()
        st = GemmStats()
        self._check(lib.clr_gemm_batch(self._h, n, pa, pb, C.byref(o), pc,
                                       C.byref(st) if stats else None))
        outs = [CLRMatrix(self, C.c_void_p(pc[i])) for i in range(n)]
        return (outs, st) if stats else outs

    # -- adjoints -------------------------------------------------------------
    def gemm_backward(self, A: "CLRMatrix", B: "CLRMatrix", dC, alpha: float = 1.0,
                      want_a: bool = True, want_b: bool = True):
        """(alpha dC B^T, alpha A^T dC) restricted to the stored blocks of A and B."""
        torch = _torch()
        dcb, ldc = _col_major(dC)
        dA = torch.empty((A.cols, A.rows), dtype=torch.float64, device="cuda") if want_a else None
        dB = torch.empty((B.cols, B.rows), dtype=torch.float64, device="cuda") if want_b else None
        self._check(lib.clr_gemm_backward(
            self._h, A._h, B._h, C.c_double(alpha), C.c_void_p(dcb.data_ptr()), C.c_int64(ldc),
            C.c_void_p(dA.data_ptr()) if dA is not None else None, C.c_int64(A.rows),
            C.c_void_p(dB.data_ptr()) if dB is not None else None, C.c_int64(B.rows)))
        return (dA.t() if dA is not None else None, dB.t() if dB is not None else None)

    def sqrt_inv_backward(self, S: "CLRMatrix", Wbar, iters: int, checkpoint_every: int,
                          tol: float, eps_sp: float, alpha: float = 0.0, screen="abs",
                          precision="fp64", split: int = 0):
        """dS of sum(Wbar * W), W from `iters` unrolled iterations; returns (dS, W)."""
        torch = _torch()
        o = SqrtInvOpts()
        o.g = _gemm_opts(tol, eps_sp, screen, precision, split, 1.0)
        o.alpha = float(alpha)
        o.conv_tol = 0.0
        o.max_iter = int(iters)
        o.fixed_iters = int(iters)
        wb, ld = _col_major(Wbar)
        dS = torch.empty((S.cols, S.rows), dtype=torch.float64, device="cuda")
        h = C.c_void_p()
        self._check(lib.clr_sqrt_inv_backward(self._h, S._h, C.byref(o), int(iters),
                                              int(checkpoint_every), C.c_void_p(wb.data_ptr()),
                                              C.c_void_p(dS.data_ptr()), C.c_int64(ld), C.byref(h)))
        return dS.t(), CLRMatrix(self, h)

    def identity_residual(self, X: "CLRMatrix") -> float:
        out = C.c_double()
        self._check(lib.clr_identity_residual(self._h, X._h, C.byref(out)))
        return out.value

    def measure_peaks(self) -> dict:
        """Measured FP64 MFMA loop rate (TFLOP/s) and device copy bandwidth (GB/s)."""
        t, b = C.c_double(), C.c_double()
        self._check(lib.clr_measure_peaks(self._h, C.byref(t), C.byref(b)))
        return {"mfma_f64_tflops": t.value, "copy_gbps": b.value}

    def identity_residual_noalloc(self, X: "CLRMatrix", out):
        """||X - I||_F / sqrt(N) written to out[0] (a caller-owned float64 cuda tensor) on the
        context stream, with no allocation inside the library (see clr.h)."""
        torch = _torch()
        if out.dtype != torch.float64 or not out.is_cuda or out.numel() < 1:
            raise TypeError("out must be a float64 cuda tensor with at least one element")
        self._check(lib.clr_identity_residual_noalloc(self._h, X._h, C.c_void_p(out.data_ptr())))
        return out


class Plan:
    """A planned batch of products (optionally recorded as a HIP graph)."""

    def __init__(self, ctx: Context, handle: C.c_void_p, outputs, As, Bs):
        self.ctx = ctx
        self._h = handle
        self.outputs = outputs
        self._keep = (As, Bs)   # operands must outlive the plan

    def execute(self, stats: bool = False):
        st = GemmStats()
        self.ctx._check(lib.clr_plan_execute(self.ctx._h, self._h, C.byref(st) if stats else None))
        return st if stats else None

    def close(self):
        if getattr(self, "_h", None):
            if getattr(self.ctx, "_h", None):
                lib.clr_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CLRMatrix:
    """Handle of a library-owned CLR matrix."""

    def __init__(self, ctx: Context, handle: C.c_void_p):
        self.ctx = ctx
        self._h = handle
        nrb, ncb = C.c_int(), C.c_int()
        rows, cols = C.c_int64(), C.c_int64()
        ctx._check(lib.clr_matrix_info(handle, C.byref(nrb), C.byref(ncb), C.byref(rows),
                                       C.byref(cols), None))
        self.nrb, self.ncb = nrb.value, ncb.value
        self.rows, self.cols = rows.value, cols.value

    def close(self):
        # a matrix outliving its context (closed first) is left to it: the native
        # handle refers to the context, which no longer exists
        if getattr(self, "_h", None):
            if getattr(self.ctx, "_h", None):
                lib.clr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.rows, self.cols)

    def meta(self):
        nb = self.nrb * self.ncb
        kind = np.zeros(nb, dtype=np.int8)
        rank = np.zeros(nb, dtype=np.int32)
        norm = np.zeros(nb, dtype=np.float64)
        self.ctx._check(lib.clr_get_meta(self.ctx._h, self._h,
                                         kind.ctypes.data_as(C.POINTER(C.c_int8)),
                                         rank.ctypes.data_as(C.POINTER(C.c_int)),
                                         norm.ctypes.data_as(C.POINTER(C.c_double))))
        return (kind.reshape(self.nrb, self.ncb), rank.reshape(self.nrb, self.ncb),
                norm.reshape(self.nrb, self.ncb))

    def stored_elements(self) -> int:
        s = C.c_int64()
        self.ctx._check(lib.clr_matrix_info(self._h, None, None, None, None, C.byref(s)))
        return s.value

    def arena(self):
        """(capacity in doubles, bytes of the device allocation) of this matrix's storage."""
        cap = C.c_int64()
        nbytes = C.c_size_t()
        self.ctx._check(lib.clr_matrix_arena(self._h, C.byref(cap), C.byref(nbytes)))
        return cap.value, nbytes.value

    def compact(self) -> "CLRMatrix":
        """Repack the storage so that the arena holds exactly the stored elements."""
        self.ctx._check(lib.clr_compact(self.ctx._h, self._h))
        return self

    def to_dense(self):
        torch = _torch()
        buf = torch.empty((self.cols, self.rows), dtype=torch.float64, device="cuda")
        self.ctx._check(lib.clr_to_dense(self.ctx._h, self._h, C.c_void_p(buf.data_ptr()),
                                         C.c_int64(self.rows)))
        return buf.t()

    def block(self, I: int, J: int, m: int, n: int, kind: int, rank: int):
        """Factors of block (I, J): ("D", D) or ("L", U, V) as torch tensors."""
        torch = _torch()
        if kind == 1:
            d = torch.empty((n, m), dtype=torch.float64, device="cuda")
            self.ctx._check(lib.clr_get_block(self.ctx._h, self._h, I, J, C.c_void_p(d.data_ptr()), None))
            return ("D", d.t())
        u = torch.empty((rank, m), dtype=torch.float64, device="cuda")
        v = torch.empty((rank, n), dtype=torch.float64, device="cuda")
        self.ctx._check(lib.clr_get_block(self.ctx._h, self._h, I, J, C.c_void_p(u.data_ptr()),
                                          C.c_void_p(v.data_ptr())))
        return ("L", u.t(), v.t())


# ---------------------------------------------------------------------------
# torch.autograd entry points.  The differentiable inputs are the dense forms
# of the CLR operands (the matrices the handles represent); gradients are
# restricted to the operands' stored blocks, and truncation is treated as the
# identity in the backward pass.
# ---------------------------------------------------------------------------

_FN = {}


def _functions():
    if _FN:
        return _FN
    torch = _torch()

    class GemmFn(torch.autograd.Function):
        @staticmethod
        def forward(fctx, a_dense, b_dense, ctx, A, B, kw):
            Cm = ctx.gemm(A, B, **kw)
            fctx.clr = (ctx, A, B, float(kw.get("alpha", 1.0)))
            return Cm.to_dense().contiguous()

        @staticmethod
        def backward(fctx, gC):
            ctx, A, B, alpha = fctx.clr
            dA, dB = ctx.gemm_backward(A, B, gC.contiguous(), alpha, fctx.needs_input_grad[0],
                                       fctx.needs_input_grad[1])
            return dA, dB, None, None, None, None

    class SqrtInvFn(torch.autograd.Function):
        @staticmethod
        def forward(fctx, s_dense, ctx, S, iters, checkpoint_every, kw):
            W, _st = ctx.sqrt_inv(S, fixed_iters=iters, **kw)
            fctx.clr = (ctx, S, iters, checkpoint_every, kw)
            return W.to_dense().contiguous()

        @staticmethod
        def backward(fctx, gW):
            ctx, S, iters, every, kw = fctx.clr
            dS, _W = ctx.sqrt_inv_backward(S, gW.contiguous(), iters, every, **kw)
            return dS, None, None, None, None, None

    _FN["gemm"] = GemmFn
    _FN["sqrt_inv"] = SqrtInvFn
    return _FN


def _check_stand_in(name, t, M: CLRMatrix, verify_tol):
    """A dense stand-in must have its handle's shape, be FP64 on the GPU and,
    with verify_tol set, equal the matrix the handle represents to that
    relative Frobenius tolerance (the product's result depends on the
    handle only, so a mismatched stand-in would get a gradient that belongs
    to another matrix)."""
    torch = _torch()
    if tuple(t.shape) != (M.rows, M.cols):
        raise ValueError(f"{name}: shape {tuple(t.shape)} does not match the handle's "
                         f"{(M.rows, M.cols)}")
    if t.dtype != torch.float64 or not t.is_cuda:
        raise ValueError(f"{name}: expected a float64 tensor on the GPU, got {t.dtype} on {t.device}")
    if verify_tol is not None:
        ref = M.to_dense()
        err = float(torch.linalg.norm(t.detach() - ref)) / max(float(torch.linalg.norm(ref)), 1e-300)
        if err > verify_tol:
            raise ValueError(f"{name}: differs from the matrix its handle represents by {err:.3e} "
                             f"(relative Frobenius) > {verify_tol:.1e}")


def gemm_dense(ctx: Context, A: CLRMatrix, B: CLRMatrix, a_dense, b_dense, verify_tol=None, **kw):
    """Dense C = A B (CLR product) differentiable w.r.t. a_dense / b_dense.

    a_dense and b_dense stand for the matrices A and B represent: the values
    are taken from the handles and gradients come from the library's adjoint.
    Shapes, dtype and device are always checked; with verify_tol the values
    are compared with the handles' dense forms too (ValueError beyond it)."""
    _check_stand_in("a_dense", a_dense, A, verify_tol)
    _check_stand_in("b_dense", b_dense, B, verify_tol)
    return _functions()["gemm"].apply(a_dense, b_dense, ctx, A, B, kw)


def sqrt_inv_dense(ctx: Context, S: CLRMatrix, s_dense, iters: int, checkpoint_every: int = 5,
                   verify_tol=None, **kw):
    """Dense W = S^-1/2 after `iters` unrolled iterations, differentiable w.r.t. s_dense
    (a stand-in for the matrix S represents, checked as in gemm_dense)."""
    _check_stand_in("s_dense", s_dense, S, verify_tol)
    return _functions()["sqrt_inv"].apply(s_dense, ctx, S, iters, checkpoint_every, kw)
