"""The allocation-free identity residual against the allocating one, through the C ABI."""
import ctypes as C
import math
import sys

import numpy as np
import pytest

from workloads import line_n512, scaled_workload

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _noalloc(lib, ctx, X, out):
    return lib.clr_identity_residual_noalloc(ctx._h, X._h, C.c_void_p(out.data_ptr()))


def test_identity_residual_noalloc_matches_allocating_call(torch):
    """Two calls in a row on one device, the second on a matrix with fewer blocks (so the fixed
    array still holds the first call's longer list of terms), each equal to clr_identity_residual
    to the FP64 bar; a matrix with more blocks than the fixed array is refused."""
    import paper_1509_00309_amd as clr
    from paper_1509_00309_amd._abi import lib
    ctx = clr.Context()
    big = scaled_workload("lattice", 1536, seed=140)
    Sb = ctx.compress(torch.from_numpy(big.dense()).cuda(), big.sizes, big.sizes, big.tol, 1e-10)
    alpha = 1.0 / float(np.max(np.sum(Sb.meta()[2], axis=1)))
    Xb = ctx.gemm(Sb, Sb, big.tol, big.eps_sp, alpha=alpha)        # an iterate-like X
    small = line_n512()
    Xs = ctx.compress(torch.from_numpy(small.dense()).cuda(), small.sizes, small.sizes, small.tol,
                      1e-10)
    nb_big, nb_small = len(big.sizes) ** 2, len(small.sizes) ** 2
    assert nb_small < nb_big
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    for X, nb, slot in ((Xb, nb_big, 0), (Xs, nb_small, 1)):
        log(f"noalloc residual: {nb} blocks")
        assert _noalloc(lib, ctx, X, out[slot:]) == 0
        ref = ctx.identity_residual(X)           # synchronises the context stream
        got = float(out[slot].item())
        log(f"  noalloc {got:.17e}  allocating {ref:.17e}")
        assert math.isfinite(got) and ref > 0
        assert abs(got - ref) <= 1e-12 * ref
    # the binding's wrapper gives the same value
    got = float(ctx.identity_residual_noalloc(Xs, out[:1])[0].item())
    assert abs(got - ctx.identity_residual(Xs)) <= 1e-12 * got
    # more blocks than the fixed array holds: refused before any launch
    n = 257
    sizes = [1] * n
    Z = ctx.create(sizes, sizes, np.zeros((n, n), dtype=np.int8), np.zeros((n, n), dtype=np.int32),
                   {}, {})
    before = out.clone()
    assert _noalloc(lib, ctx, Z, out) == 3            # CLR_ERR_CAPACITY
    torch.cuda.synchronize()
    assert torch.equal(out.isnan(), before.isnan()) and torch.equal(out[~out.isnan()],
                                                                    before[~before.isnan()])
