"""GPU parity of the HIP path (through the C ABI) against the FP64 CPU oracle."""
import math
import sys

import numpy as np
import pytest

import oracle as orc
import parity
from workloads import (batch_product, line_n512, lattice_3d, kernel_matrix, points_1d, points_3d, random_blocks,
                       rng_for, scaled_workload, sizes_weighted)

pytestmark = pytest.mark.gpu

FP64_BOUND = 1e-12


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_1509_00309_amd as clr
    return clr.Context()


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_from_random(ctx, torch, rc):
    f0 = {k: torch.from_numpy(v).cuda() for k, v in rc.f0.items()}
    f1 = {k: torch.from_numpy(v).cuda() for k, v in rc.f1.items()}
    return ctx.create(rc.row_sizes, rc.col_sizes, rc.kind, rc.rank, f0, f1)


def orc_from_random(rc):
    return orc.from_factors(rc.row_sizes, rc.col_sizes, rc.kind, rc.f0, rc.f1)


# ---------------------------------------------------------------------------
# Boundary: ingest, round trip, norms
# ---------------------------------------------------------------------------

def test_create_roundtrip_dense_bit_exact(ctx, torch):
    log("create/to_dense round trip, dense blocks")
    rc = random_blocks(101, [17, 33, 5], [9, 40, 16, 1], p_zero=0.3, p_dense=1.0)
    M = gpu_from_random(ctx, torch, rc)
    got = M.to_dense().cpu().numpy()
    ref = orc.to_dense(orc_from_random(rc))
    assert np.array_equal(got, ref)
    kind, rank, norm = M.meta()
    assert np.array_equal(kind, rc.kind)


def test_create_lowrank_norms(ctx, torch):
    log("create low-rank blocks, norms")
    rc = random_blocks(102, [30, 45, 12, 64], [50, 20, 33], p_zero=0.1, p_dense=0.3)
    M = gpu_from_random(ctx, torch, rc)
    O = orc_from_random(rc)
    got = M.to_dense().cpu().numpy()
    ref = orc.to_dense(O)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    _k, _r, norm = M.meta()
    on = O.norms()
    assert np.max(np.abs(norm - on) / np.maximum(on, 1e-300)) < 1e-13


def test_create_rejects_bad_input(ctx, torch):
    import paper_1509_00309_amd as clr
    rc = random_blocks(103, [8, 8], [8, 8], p_zero=0.0, p_dense=1.0)
    bad = rc.f0[(0, 0)].copy()
    bad[0, 0] = np.nan
    rc.f0[(0, 0)] = bad
    with pytest.raises(clr.ClrError) as e:
        gpu_from_random(ctx, torch, rc)
    assert e.value.code == 4
    rc = random_blocks(104, [8, 8], [8, 8], p_zero=0.0, p_dense=1.0)
    with pytest.raises(clr.ClrError) as e:
        f0 = {k: torch.from_numpy(v).cuda() for k, v in rc.f0.items()}
        ctx.create(rc.row_sizes, rc.col_sizes, rc.kind, rc.rank, f0, {}, norms=np.ones((2, 2)))
    assert e.value.code == 7


# ---------------------------------------------------------------------------
# Compression of an input (drop, diagonal dense, truncated SVD, dense switch)
# ---------------------------------------------------------------------------

def test_compress_line_n512(ctx, torch):
    log("compress line_n512 (N=512, 1D)")
    wl = line_n512()
    Sd = wl.dense()
    G = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    O = orc.compress(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10)
    E = orc.compress(Sd, wl.sizes, wl.sizes, 0.0, 1e-10)
    rep = parity.compare(G, O, wl.tol, exact=E)
    log("  " + parity.summary(rep))
    parity.assert_parity(rep, FP64_BOUND, nblocks=64)
    assert rep.max_norm_rel < 1e-12


def test_compress_rectangular_blocks_and_edges(ctx, torch):
    """Blocks with m < n and m > n (both Jacobi orientations), size-1 blocks, tol = 0."""
    log("compress rectangular / size-1 blocks")
    rng = rng_for(105)
    rows, cols = [1, 37, 96, 150], [80, 1, 23, 130]
    pts_r = rng.uniform(0, 30, size=(sum(rows), 1))
    pts_c = rng.uniform(0, 30, size=(sum(cols), 1))
    from workloads import kernel_block
    Sd = kernel_block(np.sort(pts_r, axis=0), np.sort(pts_c, axis=0), 0.05)
    for tol in (1e-6, 1e-10, 0.0):
        G = ctx.compress(torch.from_numpy(Sd).cuda(), rows, cols, tol, 1e-12)
        O = orc.compress(Sd, rows, cols, tol, 1e-12)
        E = orc.compress(Sd, rows, cols, 0.0, 1e-12)
        rep = parity.compare(G, O, tol, exact=E)
        log("  " + parity.summary(rep))
        parity.assert_parity(rep, FP64_BOUND, nblocks=16)


def _check_rrqr(G, Sd, O, rows, cols, tol):
    """RRQR construction against the oracle's: kinds and ranks agree (a rank may differ only at a
    cut within 1e-6 of the threshold); every factored block satisfies U^T U = I and V = M^T U
    (the rows of R), its error is within tol ||M||, and its reconstruction matches the oracle's
    unless the two took different pivots at a near tie."""
    kind, rank, norm = G.meta()
    ro = np.concatenate([[0], np.cumsum(rows)])
    co = np.concatenate([[0], np.cumsum(cols)])
    ko = O.kinds()
    same = differ = 0
    for i in range(len(rows)):
        for j in range(len(cols)):
            M = Sd[ro[i]:ro[i + 1], co[j]:co[j + 1]]
            nm = np.linalg.norm(M)
            k = int(kind[i, j])
            ob = O.blocks.get((i, j))
            if k != int(ko[i, j]) or (k == 2 and int(rank[i, j]) != ob.rank):
                r, _X, _W, tails = orc.rrqr_truncate(M, tol)
                near = [abs(tails[x] - tol * nm) <= 1e-6 * tol * nm for x in range(len(tails))]
                assert any(near), (i, j, k, int(ko[i, j]), int(rank[i, j]))
                differ += 1
                continue
            if k != 2:
                continue
            _t, U, V = G.block(i, j, rows[i], cols[j], 2, int(rank[i, j]))
            U, V = U.cpu().numpy(), V.cpu().numpy()
            r = U.shape[1]
            assert np.linalg.norm(U.T @ U - np.eye(r)) <= 1e-13 * r
            assert np.linalg.norm(V - M.T @ U) <= 1e-13 * nm
            assert np.linalg.norm(M - U @ V.T) <= tol * nm * (1 + 1e-9)
            if np.linalg.norm(U @ V.T - ob.dense()) <= 1e-12 * nm:
                same += 1
            else:
                differ += 1
    return same, differ


def test_compress_rrqr(ctx, torch):
    """clr_compress with the paper's rank-revealing QR: register-size, LDS and global-scratch
    working sets, rectangular blocks, against the oracle's column-pivoted QR."""
    log("compress by RRQR")
    wl = line_n512()
    Sd = wl.dense()
    G = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10, method="rrqr")
    O = orc.compress_rrqr(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10)
    same, differ = _check_rrqr(G, Sd, O, wl.sizes, wl.sizes, wl.tol)
    log(f"  line N=512: {same} factored blocks equal to the oracle's, {differ} at pivot ties")
    assert differ <= max(1, 0.1 * (same + differ))
    rng = rng_for(151)
    rows, cols = [1, 37, 96, 150, 200], [80, 1, 23, 130, 300]
    pts_r = rng.uniform(0, 30, size=(sum(rows), 1))
    pts_c = rng.uniform(0, 30, size=(sum(cols), 1))
    from workloads import kernel_block
    Sr = kernel_block(np.sort(pts_r, axis=0), np.sort(pts_c, axis=0), 0.05)
    for tol in (1e-6, 1e-10):
        G = ctx.compress(torch.from_numpy(Sr).cuda(), rows, cols, tol, 1e-12, method="rrqr")
        O = orc.compress_rrqr(Sr, rows, cols, tol, 1e-12)
        same, differ = _check_rrqr(G, Sr, O, rows, cols, tol)
        log(f"  rectangular tol {tol}: {same} equal, {differ} at pivot ties")
        assert differ <= max(1, 0.1 * (same + differ))
    # the default stays the SVD
    G = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    rep = parity.compare(G, orc.compress(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10), wl.tol)
    log("  " + parity.summary(rep))
    parity.assert_parity(rep, FP64_BOUND, nblocks=64)


def test_kernel_matrix_generator(ctx, torch):
    """clr_kernel_matrix against the seeded host generator: the Coulomb-like kernel bit for bit
    (r^2 rounded step by step, correctly rounded sqrt and division), the overlap-like kernel
    within exp's last-bit rounding; the CLR matrix built from the device-generated input equals
    the one built from the host matrix, and meets the FP64 bar against the oracle's."""
    import paper_1509_00309_amd as clr
    log("kernel matrix generator")
    wl = scaled_workload("coulomb", 1536, seed=161)
    pts = torch.from_numpy(wl.points).cuda()
    G = ctx.kernel_matrix(pts, "coulomb", wl.a, wl.diag)
    got, ref = G.cpu().numpy(), wl.dense()
    assert G.shape == ref.shape and np.array_equal(got, ref)
    A = ctx.compress(G, wl.sizes, wl.sizes, wl.tol, 1e-10)
    B = ctx.compress(torch.from_numpy(ref).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    for x, y in zip(A.meta(), B.meta()):
        assert np.array_equal(x, y)
    assert torch.equal(A.to_dense(), B.to_dense())
    rep = parity.compare(A, orc.compress(ref, wl.sizes, wl.sizes, wl.tol, 1e-10), wl.tol)
    log("  " + parity.summary(rep))
    parity.assert_parity(rep, FP64_BOUND, nblocks=len(wl.sizes) ** 2)

    wl = scaled_workload("lattice", 1536, seed=162)
    G = ctx.kernel_matrix(torch.from_numpy(wl.points).cuda(), "gaussian", wl.a, wl.diag)
    got, ref = G.cpu().numpy(), wl.dense()
    log(f"  gaussian: {int(np.sum(got != ref))} of {got.size} entries differ in the last bits")
    assert np.all(np.abs(got - ref) <= 4.5e-16 * np.abs(ref))
    S = ctx.compress(G, wl.sizes, wl.sizes, wl.tol, 1e-10)
    rep = parity.compare(S, orc.compress(ref, wl.sizes, wl.sizes, wl.tol, 1e-10), wl.tol)
    log("  " + parity.summary(rep))
    parity.assert_parity(rep, FP64_BOUND, nblocks=len(wl.sizes) ** 2)

    # rectangular, one dimension, distinct row and column points, no diagonal shift
    x = points_1d(rng_for(163), 520, 1.0, 0.2)
    from workloads import kernel_block
    G = ctx.kernel_matrix(torch.from_numpy(x[:300]).cuda(), "gaussian", 0.05, 0.0,
                          col_points=torch.from_numpy(x[100:]).cuda())
    ref = kernel_block(x[:300], x[100:], 0.05)
    assert G.shape == (300, 420)
    # far entries underflow to zero on both sides
    assert np.all(np.abs(G.cpu().numpy() - ref) <= 4.5e-16 * np.abs(ref) + 1e-300)

    # two dimensions, the Coulomb-like kernel with a diagonal shift, rectangular by columns
    from workloads import coulomb_block
    p2 = rng_for(164).uniform(0, 10, size=(200, 2))
    G = ctx.kernel_matrix(torch.from_numpy(p2).cuda(), "coulomb", 0.7, 0.3,
                          col_points=torch.from_numpy(p2[:150]).cuda())
    ref = coulomb_block(p2, p2[:150], 0.7)
    ref[np.arange(150), np.arange(150)] += 0.3
    assert G.shape == (200, 150) and np.array_equal(G.cpu().numpy(), ref)

    # argument errors are reported, nothing is launched
    with pytest.raises(clr.ClrError):
        ctx.kernel_matrix(pts, "coulomb", 0.0, 0.1)
    with pytest.raises(clr.ClrError):
        ctx.kernel_matrix(torch.zeros((4, 4), dtype=torch.float64, device="cuda"), "gaussian")


# ---------------------------------------------------------------------------
# The product
# ---------------------------------------------------------------------------

def test_gemm_dense_limit_exact(ctx, torch):
    """tol = 0, eps_sp = 0, all blocks dense: the product equals the dense FP64 product."""
    log("gemm dense limit")
    rc_a = random_blocks(106, [48, 160, 17, 129], [100, 33, 160], p_zero=0.0, p_dense=1.0)
    rc_b = random_blocks(107, [100, 33, 160], [64, 150, 7], p_zero=0.0, p_dense=1.0)
    A, B = gpu_from_random(ctx, torch, rc_a), gpu_from_random(ctx, torch, rc_b)
    C = ctx.gemm(A, B, tol=0.0, eps_sp=0.0)
    got = C.to_dense().cpu().numpy()
    ref = orc.to_dense(orc_from_random(rc_a)) @ orc.to_dense(orc_from_random(rc_b))
    assert np.sqrt(np.sum((got - ref) ** 2)) / np.sqrt(np.sum(ref ** 2)) < 1e-14


@pytest.mark.parametrize("seed", [110, 111, 112])
def test_gemm_all_product_kinds_untruncated(ctx, torch, seed):
    """Mixed zero/dense/low-rank blocks, tol = 0: every product kind and both accumulation paths."""
    log(f"gemm random kinds untruncated seed={seed}")
    rows, inner, cols = [40, 96, 23, 150], [64, 30, 128, 77], [50, 96, 33, 140]
    rc_a = random_blocks(seed, rows, inner, p_zero=0.2, p_dense=0.25)
    rc_b = random_blocks(seed + 50, inner, cols, p_zero=0.2, p_dense=0.25)
    A, B = gpu_from_random(ctx, torch, rc_a), gpu_from_random(ctx, torch, rc_b)
    C, st = ctx.gemm(A, B, tol=0.0, eps_sp=0.0, alpha=0.75, stats=True)
    Oa, Ob = orc_from_random(rc_a), orc_from_random(rc_b)
    Oc = orc.gemm(Oa, Ob, 0.0, 0.0, alpha=0.75)
    rep = parity.compare(C, Oc, 0.0, operands=(Oa, Ob, 0.75))
    log("  " + parity.summary(rep))
    parity.assert_parity(rep, FP64_BOUND, nblocks=16)
    assert st.n_ld + st.n_dl + st.n_ll > 0


@pytest.mark.parametrize("seed", [120, 121])
def test_gemm_all_product_kinds_truncated(ctx, torch, seed):
    log(f"gemm random kinds truncated seed={seed}")
    rows, inner, cols = [40, 96, 23, 150], [64, 30, 128, 77], [50, 96, 33, 140]
    rc_a = random_blocks(seed, rows, inner, p_zero=0.2, p_dense=0.25, max_rank=6)
    rc_b = random_blocks(seed + 50, inner, cols, p_zero=0.2, p_dense=0.25, max_rank=6)
    A, B = gpu_from_random(ctx, torch, rc_a), gpu_from_random(ctx, torch, rc_b)
    tol = 1e-3
    C = ctx.gemm(A, B, tol=tol, eps_sp=1e-12)
    Oa, Ob = orc_from_random(rc_a), orc_from_random(rc_b)
    Oc = orc.gemm(Oa, Ob, tol, 1e-12)
    E = orc.gemm(Oa, Ob, 0.0, 1e-12)
    rep = parity.compare(C, Oc, tol, exact=E, operands=(Oa, Ob))
    log("  " + parity.summary(rep))
    parity.assert_parity(rep, FP64_BOUND, nblocks=16)


def test_gemm_screening_modes(ctx, torch):
    """Norms spread over decades; absolute and per-area screening drop the same blocks as the oracle."""
    log("gemm screening")
    rows = [20, 31, 17, 25, 22, 30]
    rc_a = random_blocks(130, rows, rows, p_zero=0.05, p_dense=0.5, scale_decay=4.0)
    rc_b = random_blocks(131, rows, rows, p_zero=0.05, p_dense=0.5, scale_decay=4.0)
    A, B = gpu_from_random(ctx, torch, rc_a), gpu_from_random(ctx, torch, rc_b)
    Oa, Ob = orc_from_random(rc_a), orc_from_random(rc_b)
    for screen, eps in (("abs", 1e-3), ("area", 1e-6)):
        C = ctx.gemm(A, B, tol=0.0, eps_sp=eps, screen=screen)
        Oc = orc.gemm(Oa, Ob, 0.0, eps, screen)
        kind_g, _, _ = C.meta()
        assert np.array_equal(kind_g, Oc.kinds()), screen
        rep = parity.compare(C, Oc, 0.0, operands=(Oa, Ob))
        log("  " + parity.summary(rep))
        parity.assert_parity(rep, FP64_BOUND, nblocks=36)


def test_gemm_everything_screened(ctx, torch):
    rc = random_blocks(132, [8, 9], [8, 9], p_zero=0.0, p_dense=1.0)
    A = gpu_from_random(ctx, torch, rc)
    C = ctx.gemm(A, A, tol=0.0, eps_sp=1e30)
    kind, _, _ = C.meta()
    assert np.all(kind == 0)
    assert np.all(C.to_dense().cpu().numpy() == 0.0)


def test_gemm_shape_mismatch(ctx, torch):
    import paper_1509_00309_amd as clr
    a = random_blocks(133, [8, 9], [8, 9], p_zero=0.0, p_dense=1.0)
    b = random_blocks(134, [9, 8], [8, 9], p_zero=0.0, p_dense=1.0)
    A, B = gpu_from_random(ctx, torch, a), gpu_from_random(ctx, torch, b)
    with pytest.raises(clr.ClrError) as e:
        ctx.gemm(A, B, 0.0, 0.0)
    assert e.value.code == 2


def test_gemm_line_n512(ctx, torch):
    log("gemm line_n512 S*S")
    wl = line_n512()
    Sd = wl.dense()
    S = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    O = orc.compress(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10)
    C = ctx.gemm(S, S, wl.tol, wl.eps_sp)
    Oc = orc.gemm(O, O, wl.tol, wl.eps_sp)
    E = orc.gemm(O, O, 0.0, wl.eps_sp)
    rep = parity.compare(C, Oc, wl.tol, exact=E, operands=(O, O))
    log("  " + parity.summary(rep))
    parity.assert_parity(rep, FP64_BOUND, nblocks=64)


def test_gemm_3d_scaled(ctx, torch):
    """Overlap-like 3D matrix (the N = 8192 physics) at N = 1536: several dozen blocks, ragged sizes."""
    log("gemm 3D scaled N=1536")
    wl = scaled_workload("lattice", 1536, seed=140)
    Sd = wl.dense()
    S = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    O = orc.compress(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10)
    C, st = ctx.gemm(S, S, wl.tol, wl.eps_sp, stats=True)
    Oc = orc.gemm(O, O, wl.tol, wl.eps_sp)
    E = orc.gemm(O, O, 0.0, wl.eps_sp)
    rep = parity.compare(C, Oc, wl.tol, exact=E, operands=(O, O))
    nb = len(wl.sizes) ** 2
    log("  " + parity.summary(rep))
    parity.assert_parity(rep, FP64_BOUND, nblocks=nb)
    log(f"  blocks={nb} computed={st.computed} dense={st.out_dense} lr={st.out_lowrank} "
        f"err={rep.rel_err:.2e} ambiguous={len(rep.ambiguous)}")


@pytest.mark.parametrize("kind,n", [("morton", 2048), ("coulomb", 1536)])
def test_gemm_low_rank_regime(ctx, torch, kind, n):
    """Rank-sparse inputs: Morton-ordered compact clusters of the 3D Gaussian workload and a
    Coulomb-like 1/sqrt(r^2 + 1) kernel; most result blocks take the low-rank recompression path."""
    log(f"gemm low-rank regime: {kind} N={n}")
    wl = scaled_workload(kind, n, seed=150)
    Sd = wl.dense()
    S = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    O = orc.compress(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10)
    C, st = ctx.gemm(S, S, wl.tol, wl.eps_sp, stats=True)
    Oc = orc.gemm(O, O, wl.tol, wl.eps_sp)
    E = orc.gemm(O, O, 0.0, wl.eps_sp)
    rep = parity.compare(C, Oc, wl.tol, exact=E, operands=(O, O))
    nb = len(wl.sizes) ** 2
    log(f"  blocks={nb} computed={st.computed} dense={st.out_dense} lr={st.out_lowrank} "
        f"err={rep.rel_err:.2e} ambiguous={len(rep.ambiguous)}")
    assert st.out_lowrank > st.out_dense
    log("  " + parity.summary(rep))
    parity.assert_parity(rep, FP64_BOUND, nblocks=nb)


def _bitwise_same(A, B):
    ka, ra, na = A.meta()
    kb, rb, nb = B.meta()
    assert np.array_equal(ka, kb) and np.array_equal(ra, rb) and np.array_equal(na, nb)
    assert np.array_equal(A.to_dense().cpu().numpy(), B.to_dense().cpu().numpy())


@pytest.mark.parametrize("tol", [1e-6, 1e-8])
def test_dense_certificate_changes_nothing(torch, tol):
    """Blocks proved dense from their Gram matrix skip the SVD: the product is bit for bit the one
    computed without the proof (3D workload at N = 1536, blocks of the register engine)."""
    import paper_1509_00309_amd as clr
    log(f"dense certificate on/off, 3D N=1536, tol {tol}")
    wl = scaled_workload("lattice", 1536, seed=146, tol=tol)
    Sd = wl.dense()
    c = clr.Context()
    S = c.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, tol, 1e-10)
    C_on, st_on = c.gemm(S, S, tol, wl.eps_sp, stats=True)
    c.set_dense_certificate(False)
    C_off, st_off = c.gemm(S, S, tol, wl.eps_sp, stats=True)
    log(f"  certified {st_on.certified_dense} of {st_on.out_dense} dense; bidiagonalisation flops "
        f"{st_on.flops_rec_engine:.3e} vs {st_off.flops_rec_engine:.3e} without the proof")
    assert 0 < st_on.certified_dense <= st_on.out_dense
    assert st_off.certified_dense == 0
    assert st_on.flops_rec_engine < st_off.flops_rec_engine
    _bitwise_same(C_on, C_off)


@pytest.mark.parametrize("sizes", [[120, 230, 64, 300, 150], [120, 400, 64, 340, 150]])
def test_dense_certificate_general_kernel(torch, sizes):
    """Blocks whose long edge exceeds 160 go to the general recompression kernel; the certificate
    proves the dense ones there as well: short edges up to 319 from a 160-column subset, beyond
    that (400 x 340 here) by the left-looking form.  Compression (dense and low-rank results) and
    the product are unchanged by it and match the oracle."""
    import paper_1509_00309_amd as clr
    log(f"dense certificate, general-kernel blocks, sizes {sizes}")
    n = sum(sizes)
    Sd3 = kernel_matrix(points_3d(rng_for(148), n, 1.5, 0.3), 0.3, 0.1)   # dense blocks
    Sd1 = kernel_matrix(points_1d(rng_for(149), n, 1.0, 0.2), 0.05, 0.1)  # low-rank blocks
    c = clr.Context()
    for Sd, tol in ((Sd3, 1e-6), (Sd1, 1e-6), (Sd1, 1e-8)):
        c.set_dense_certificate(True)
        G_on = c.compress(torch.from_numpy(Sd).cuda(), sizes, sizes, tol, 1e-12)
        c.set_dense_certificate(False)
        G_off = c.compress(torch.from_numpy(Sd).cuda(), sizes, sizes, tol, 1e-12)
        _bitwise_same(G_on, G_off)
        O = orc.compress(Sd, sizes, sizes, tol, 1e-12)
        E = orc.compress(Sd, sizes, sizes, 0.0, 1e-12)
        rep = parity.compare(G_on, O, tol, exact=E)
        log("  " + parity.summary(rep))
        parity.assert_parity(rep, FP64_BOUND, nblocks=25)
    c.set_dense_certificate(True)
    S = c.compress(torch.from_numpy(Sd3).cuda(), sizes, sizes, 1e-6, 1e-12)
    C, st = c.gemm(S, S, 1e-6, 1e-10, stats=True)
    c.set_dense_certificate(False)
    C_off, st_off = c.gemm(S, S, 1e-6, 1e-10, stats=True)
    c.set_dense_certificate(True)
    _bitwise_same(C, C_off)
    kinds = C.meta()[0]
    nb = len(sizes)
    # dense off-diagonal results by short edge: up to 160 (the full Gram matrix), beyond
    small = sum(1 for i in range(nb) for j in range(nb)
                if i != j and kinds[i, j] == 1 and min(sizes[i], sizes[j]) <= 160)
    big = sum(1 for i in range(nb) for j in range(nb)
              if i != j and kinds[i, j] == 1 and min(sizes[i], sizes[j]) > 160)
    log(f"  product: certified {st.certified_dense} of {st.out_dense} dense "
        f"({small} off-diagonal with short edge <= 160, {big} beyond)")
    assert big > 0 and small < st.certified_dense <= small + big
    assert st_off.certified_dense == 0
    O = orc.compress(Sd3, sizes, sizes, 1e-6, 1e-12)
    rep = parity.compare(C, orc.gemm(O, O, 1e-6, 1e-10), 1e-6, exact=orc.gemm(O, O, 0.0, 1e-10),
                         operands=(O, O))
    log("  " + parity.summary(rep))
    parity.assert_parity(rep, FP64_BOUND, nblocks=25)


def test_axpby_ns_combination(ctx, torch):
    """T = (-10 X + 3 X^2 + 15 I)/8 (Eq. (9)) with low-rank, dense and identity terms."""
    log("axpby (NS T)")
    wl = line_n512()
    Sd = wl.dense()
    S = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    O = orc.compress(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10)
    a = orc.default_alpha(O)
    X = ctx.gemm(S, S, wl.tol, wl.eps_sp, alpha=a)
    Q = ctx.gemm(X, X, wl.tol, wl.eps_sp)
    T = ctx.axpby(-10 / 8, X, 3 / 8, Q, 15 / 8, wl.tol, wl.eps_sp)
    Ox = orc.gemm(O, O, wl.tol, wl.eps_sp, alpha=a)
    Oq = orc.gemm(Ox, Ox, wl.tol, wl.eps_sp)
    Ot = orc.ns_T(Ox, Oq, wl.tol, wl.eps_sp)
    scale = 1.25 * Ox.norms() + 0.375 * Oq.norms() + 1.875 * np.diag(np.sqrt(np.array(wl.sizes, float)))
    rep = parity.compare(T, Ot, wl.tol, floor=1e-2 * scale)
    log("  " + parity.summary(rep))
    parity.assert_parity(rep, FP64_BOUND, nblocks=64)


def test_sqrt_inv_line_n512(ctx, torch):
    log("sqrt_inv line_n512")
    wl = line_n512()
    Sd = wl.dense()
    S = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    O = orc.compress(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10)
    W, st = ctx.sqrt_inv(S, wl.tol, wl.eps_sp, conv_tol=wl.extra["conv_tol"],
                         allow_not_converged=True)
    Ow, info = orc.sqrt_inv(O, wl.tol, wl.eps_sp, conv_tol=wl.extra["conv_tol"])
    assert st.iterations == info.iterations
    rep = parity.compare(W, Ow, wl.tol)
    log(f"  iters={st.iterations} internal={st.internal_residual:.2e} "
        f"explicit={st.explicit_residual:.2e} err={rep.rel_err:.2e}")
    log("  " + parity.summary(rep))
    parity.assert_parity(rep, FP64_BOUND, nblocks=64)
    assert abs(st.explicit_residual - info.explicit[-1][1]) <= 1e-12
    assert bool(st.converged) == (info.status == "converged")


def test_sqrt_inv_wide_lattice_3d(ctx, torch):
    """S^-1/2 on the 3-D wide-lattice physics of the N = 32768 workload (spacing 1.2,
    exp(-0.2 r^2) + 0.05 delta, kappa ~ 620) at N = 1536 in 12 uneven clusters (64..170 points,
    so blocks above 160 take the general recompression kernel), tol 1e-8, conv_tol 1e-8: the
    same iteration count and status as the oracle, its explicit residual, and its W block by
    block at the FP64 bar."""
    log("sqrt_inv wide 3D lattice N=1536")
    wl = scaled_workload("wide", 1536)
    Sd = wl.dense()
    S = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    O = orc.compress(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10)
    conv = wl.extra["conv_tol"]
    W, st = ctx.sqrt_inv(S, wl.tol, wl.eps_sp, conv_tol=conv, allow_not_converged=True)
    Ow, info = orc.sqrt_inv(O, wl.tol, wl.eps_sp, conv_tol=conv)
    log(f"  GPU: iters={st.iterations} converged={st.converged} internal={st.internal_residual:.2e} "
        f"explicit={st.explicit_residual:.2e}; oracle: iters={info.iterations} {info.status} "
        f"explicit={info.explicit[-1][1]:.2e}")
    assert st.iterations == info.iterations
    assert bool(st.converged) == (info.status == "converged")
    assert abs(st.explicit_residual - info.explicit[-1][1]) <= 1e-12
    assert abs(st.internal_residual - info.internal[-1]) <= 1e-12
    rep = parity.compare(W, Ow, wl.tol)
    log("  " + parity.summary(rep))
    parity.assert_parity(rep, FP64_BOUND, nblocks=len(wl.sizes) ** 2)


def _same_clr(torch, A, B):
    """Two CLR matrices with equal kinds, ranks, norms and dense values, bit for bit."""
    ka, ra, na = A.meta()
    kb, rb, nb = B.meta()
    assert np.array_equal(ka, kb) and np.array_equal(ra, rb)
    assert np.array_equal(na, nb)
    assert torch.equal(A.to_dense(), B.to_dense())


@pytest.mark.parametrize("case,precision,margin", [("line", "fp64", 0.0), ("wide", "fp64", 0.0),
                                                    ("wide", "mixed", 0.0), ("line", "fp64", 0.01)])
def test_sqrt_inv_graph_replay_bit_exact(ctx, torch, case, precision, margin):
    """S^-1/2 with each iteration replayed from a recorded HIP graph (the four products, the
    combination of Eq. (9) and the residual terms, list lengths kept on the device) equals the
    directly run iteration bit for bit: W's kinds, ranks, norms and values, the iteration
    count, status and both residuals.  Margin 0.01 gives the graph lists too small for the
    second iteration, so the device flags the overflow, that iteration is redone directly and
    the graphs are recorded again (at least four recordings), still with equal results.  The
    iterates fill in as Z_n approaches S^-1/2, so lists can also outgrow the default margin
    (measured: the line workload re-records twice at margin 1.5)."""
    log(f"sqrt_inv graph replay {case} {precision} margin {margin}")
    wl = line_n512() if case == "line" else scaled_workload("wide", 1536)
    Sd = wl.dense()
    S = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    conv = wl.extra["conv_tol"]
    kw = dict(conv_tol=conv, precision=precision, allow_not_converged=True)
    if precision == "mixed":
        kw["max_iter"] = 14
    W0, s0 = ctx.sqrt_inv(S, wl.tol, wl.eps_sp, **kw)
    W1, s1 = ctx.sqrt_inv(S, wl.tol, wl.eps_sp, graph=True, graph_margin=margin, **kw)
    log(f"  direct: iters={s0.iterations} internal={s0.internal_residual:.3e} "
        f"explicit={s0.explicit_residual:.3e}; graph: iters={s1.iterations} "
        f"replays={s1.graph_replays} captures={s1.graph_captures}")
    assert s1.iterations == s0.iterations and s1.converged == s0.converged
    assert s1.internal_residual == s0.internal_residual
    assert s1.explicit_residual == s0.explicit_residual
    assert abs(s1.flops_products - s0.flops_products) <= 1e-12 * s0.flops_products
    _same_clr(torch, W0, W1)
    # every directly run iteration (the first, and each one whose lists overflowed) is followed
    # by two recordings; every other iteration is a replay
    assert s1.graph_captures % 2 == 0 and s1.graph_captures >= 2
    assert s1.graph_replays + s1.graph_captures // 2 == s0.iterations
    if margin == 0.0:
        assert s1.graph_replays >= 1
    else:
        assert s1.graph_captures >= 4


def test_sqrt_inv_graph_replay_bit_exact_n8192(ctx, torch):
    """Graph replay against the direct iteration on the N = 8192 wide 3-D lattice (64 clusters) at
    3 fixed iterations.  The graph's workspace is separate from the one direct calls reuse (its
    buffers hold other data), so a kernel whose result depended on what a buffer held before (once: an
    uninitialised flag of the product's recompression items, which sent random blocks to the
    column-pivoted-QR truncation) shows up as a difference here."""
    from workloads import lattice_3d_wide
    wl = lattice_3d_wide(8192, 64)
    S = ctx.compress(torch.from_numpy(wl.dense()).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    W0, s0 = ctx.sqrt_inv(S, wl.tol, wl.eps_sp, fixed_iters=3)
    W1, s1 = ctx.sqrt_inv(S, wl.tol, wl.eps_sp, fixed_iters=3, graph=True)
    log(f"  N=8192 graph replays={s1.graph_replays} captures={s1.graph_captures} "
        f"internal {s0.internal_residual:.17e} / {s1.internal_residual:.17e}")
    assert s1.graph_replays == 2 and s1.internal_residual == s0.internal_residual
    _same_clr(torch, W0, W1)


def test_sqrt_inv_graph_fixed_iterations_and_rejections(ctx, torch):
    """Graph replay with a fixed iteration count equals the direct run; the precision schedule
    and the INT8 form are rejected with graph replay."""
    from paper_1509_00309_amd._abi import ClrError
    wl = line_n512()
    S = ctx.compress(torch.from_numpy(wl.dense()).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    W0, s0 = ctx.sqrt_inv(S, wl.tol, wl.eps_sp, fixed_iters=6)
    W1, s1 = ctx.sqrt_inv(S, wl.tol, wl.eps_sp, fixed_iters=6, graph=True)
    assert s1.graph_replays + s1.graph_captures // 2 == 6
    assert s1.internal_residual == s0.internal_residual
    _same_clr(torch, W0, W1)
    with pytest.raises(ClrError):
        ctx.sqrt_inv(S, wl.tol, wl.eps_sp, precision="mixed", reduced_below=0.3, graph=True)
    with pytest.raises(ClrError):
        ctx.sqrt_inv(S, wl.tol, wl.eps_sp, precision="ozaki", graph=True)


@pytest.mark.parametrize("reduced_below", [0.3, 0.03])
def test_mixed_sqrt_inv_schedule_wide_lattice_3d(ctx, torch, reduced_below):
    """Reduced-precision S^-1/2 with the precision schedule: FP64 products until
    ||X_n - I||_F/sqrt(N) <= reduced_below, then X_n in FP64 and the other products on FP32
    MFMA in the correction form (T_n = I + D_n).  On the 3-D wide-lattice cut (N = 1536,
    kappa ~ 620, tol 1e-8) it converges like the FP64 oracle and its W is within 10 x tol of the
    oracle's, block by block; the unscheduled FP32 form stays above that (measured 3e-6 at
    N = 8192)."""
    log(f"mixed sqrt_inv with schedule below {reduced_below}, wide 3D lattice N=1536")
    wl = scaled_workload("wide", 1536)
    Sd = wl.dense()
    S = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    O = orc.compress(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10)
    conv = wl.extra["conv_tol"]
    W, st = ctx.sqrt_inv(S, wl.tol, wl.eps_sp, conv_tol=conv, precision="mixed",
                         reduced_below=reduced_below, correction=True)
    Ow, info = orc.sqrt_inv(O, wl.tol, wl.eps_sp, conv_tol=conv)
    log(f"  GPU mixed: iters={st.iterations} converged={st.converged} "
        f"explicit={st.explicit_residual:.2e}; oracle: iters={info.iterations} {info.status}")
    assert info.status == "converged" and st.converged
    assert abs(st.iterations - info.iterations) <= 1
    assert st.explicit_residual <= conv
    rep = parity.compare(W, Ow, wl.tol, ambiguous_rel=0.05)
    log("  " + parity.summary(rep))
    # Whole matrix within 10 x tol.  Per block: the far blocks of W (norms down to 1e-4 of the
    # diagonal ones) carry the absolute rounding of the FP32 products, which is not proportional
    # to their own norm; switching at 0.3 leaves 9.9e-8 of its norm on the worst one (block
    # (0, 11)), switching at 0.03 leaves 1e-10.
    parity.assert_parity(rep, 10 * wl.tol, nblocks=len(wl.sizes) ** 2, max_ambiguous_frac=0.05,
                         block_bound=(10 if reduced_below <= 0.03 else 100) * wl.tol,
                         norm_bound=10 * wl.tol)


def test_mixed_gemm_3d_scaled(ctx, torch):
    """FP32-MFMA products with FP64 accumulation: within 10 x tol of the FP64 oracle for the
    whole matrix, block by block and in the norm table; kinds and ranks equal the oracle's except
    at cuts within 5 % of the threshold (FP32 rounding moves singular values by ~1e-8 ||C||)."""
    log("mixed gemm 3D scaled")
    wl = scaled_workload("lattice", 1536, seed=141)
    Sd = wl.dense()
    S = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    O = orc.compress(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10)
    Oc = orc.gemm(O, O, wl.tol, wl.eps_sp)
    E = orc.gemm(O, O, 0.0, wl.eps_sp)
    nb = len(wl.sizes) ** 2
    for split in (0, 1):
        C = ctx.gemm(S, S, wl.tol, wl.eps_sp, precision="mixed", split=split)
        rep = parity.compare(C, Oc, wl.tol, exact=E, ambiguous_rel=0.05, operands=(O, O))
        log(f"  split={split} " + parity.summary(rep))
        parity.assert_parity(rep, 10 * wl.tol, nblocks=nb, max_ambiguous_frac=0.05)


def test_ozaki_gemm_3d_scaled(ctx, torch):
    """Dense accumulation on INT8 MFMA by operand splitting: with 7 digits the product meets the
    FP64 bar against the oracle (ambiguous cuts judged on the exact product); with 4 digits it
    stays within 10 x tol.  Items are at most 64 x 64, so blocks of 96..160 span several."""
    log("ozaki gemm 3D scaled")
    wl = scaled_workload("lattice", 1536, seed=142)
    Sd = wl.dense()
    S = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    O = orc.compress(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10)
    Oc = orc.gemm(O, O, wl.tol, wl.eps_sp)
    E = orc.gemm(O, O, 0.0, wl.eps_sp)
    C = ctx.gemm(S, S, wl.tol, wl.eps_sp, precision="ozaki", split=7)
    rep = parity.compare(C, Oc, wl.tol, exact=E, operands=(O, O))
    nb = len(wl.sizes) ** 2
    log(f"  7 digits: err={rep.rel_err:.2e} ambiguous={len(rep.ambiguous)}")
    log("  " + parity.summary(rep))
    parity.assert_parity(rep, FP64_BOUND, nblocks=nb)
    ref = orc.to_dense(Oc)
    C4 = ctx.gemm(S, S, wl.tol, wl.eps_sp, precision="ozaki", split=4)
    got = C4.to_dense().cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    log(f"  4 digits: err={err:.2e}")
    assert err <= 10 * wl.tol


def test_ozaki_digit_error_bound(ctx, torch):
    """Element-wise bound of the operand-split arithmetic.  With every block dense and no
    truncation, an item's inner range is the plain inner index, cut into 64-wide chunks.  For a
    chunk scaled by 2^e <= 2 max|x| (rows) and 2^f <= 2 max|y| (columns), S digits leave at
    most (S + 3) 2^(-7S) 2^(e+f) per inner index (remainders and dropped digit products), so
        |C_ij - (A B)_ij| <= sum_c 4 * 64 (S + 3) 2^(-7S) max_c|A_i.| max_c|B_.j| + FP64 slack.
    Entries span four decades, so a wrong digit weight or exponent breaks the bound."""
    log("ozaki digit error bound")
    rng = rng_for(181)
    rs, ks, cs = [64, 50], [100, 92], [64, 30]
    M, K, N = sum(rs), sum(ks), sum(cs)
    Ad = rng.standard_normal((M, K)) * 10.0 ** rng.uniform(-2, 2, size=(M, K))
    Bd = rng.standard_normal((K, N)) * 10.0 ** rng.uniform(-2, 2, size=(K, N))
    A = ctx.compress(torch.from_numpy(Ad).cuda(), rs, ks, 0.0, 0.0)
    B = ctx.compress(torch.from_numpy(Bd).cuda(), ks, cs, 0.0, 0.0)
    for Mx in (A, B):
        assert np.all(Mx.meta()[0] == 1)
    ref = Ad @ Bd
    absprod = np.abs(Ad) @ np.abs(Bd)
    nch = (K + 63) // 64
    mx = np.stack([np.abs(Ad[:, 64 * c:64 * c + 64]).max(axis=1) for c in range(nch)], axis=1)
    my = np.stack([np.abs(Bd[64 * c:64 * c + 64, :]).max(axis=0) for c in range(nch)], axis=0)
    chunk_bound = mx @ my   # sum over chunks of max|x| max|y|
    prev = None
    for S in (2, 4, 7):
        C = ctx.gemm(A, B, 0.0, 0.0, precision="ozaki", split=S)
        err = np.abs(C.to_dense().cpu().numpy() - ref)
        bound = 4 * 64 * (S + 3) * 2.0 ** (-7 * S) * chunk_bound \
            + (K + 4 * S * nch) * 2.0 ** -53 * absprod
        worst = float(np.max(err / bound))
        rel = float(np.linalg.norm(err) / np.linalg.norm(ref))
        log(f"  S={S}: relative error {rel:.2e}, largest error / bound {worst:.3f}")
        assert worst <= 1.0
        if prev is not None:
            assert rel < prev
        prev = rel


def test_ozaki_sqrt_inv_line_n512(ctx, torch):
    """S^-1/2 with every dense accumulation in the operand-split form (7 digits): the same
    iteration count and the oracle's result to the FP64 iteration's bar."""
    log("ozaki sqrt_inv line_n512")
    wl = line_n512()
    Sd = wl.dense()
    S = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    O = orc.compress(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10)
    W, st = ctx.sqrt_inv(S, wl.tol, wl.eps_sp, conv_tol=wl.extra["conv_tol"], precision="ozaki",
                         allow_not_converged=True)
    Ow, info = orc.sqrt_inv(O, wl.tol, wl.eps_sp, conv_tol=wl.extra["conv_tol"])
    assert st.iterations == info.iterations
    rep = parity.compare(W, Ow, wl.tol)
    log(f"  iters={st.iterations} explicit={st.explicit_residual:.2e} err={rep.rel_err:.2e}")
    log("  " + parity.summary(rep))
    parity.assert_parity(rep, FP64_BOUND, nblocks=64)
    assert abs(st.explicit_residual - info.explicit[-1][1]) <= 1e-12


def test_ozaki_batch_matches_single_products(ctx, torch):
    """The operand-split form in a planned batch (one launch per phase) equals the products one
    by one in the same form, bit for bit."""
    log("ozaki batch vs single products")
    ops = _batch_operands(ctx, torch)
    As, Bs = [a for a, _ in ops], [b for _, b in ops]
    Cs = ctx.gemm_batch(As, Bs, 1e-8, 1e-10, precision="ozaki")
    for (A, B), Cb in zip(ops, Cs):
        C1 = ctx.gemm(A, B, 1e-8, 1e-10, precision="ozaki")
        assert np.array_equal(Cb.to_dense().cpu().numpy(), C1.to_dense().cpu().numpy())
        for x, y in zip(Cb.meta(), C1.meta()):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("seed", [171, 172])
def test_ozaki_gemm_all_kinds_untruncated(ctx, torch, seed):
    """Every block kind and ragged edges (items cut at 64, partial 16-tiles, inner ranges that
    end inside a 64-chunk), no truncation: 7 digits against the oracle's product."""
    import paper_1509_00309_amd as clr
    log(f"ozaki all kinds seed={seed}")
    rs, ks, cs = [40, 130, 17, 71], [25, 150, 9, 70, 66], [31, 129, 12]
    ra = random_blocks(seed, rs, ks, p_zero=0.2, p_dense=0.5, max_rank=8)
    rb = random_blocks(seed + 50, ks, cs, p_zero=0.2, p_dense=0.5, max_rank=8)
    A, B = gpu_from_random(ctx, torch, ra), gpu_from_random(ctx, torch, rb)
    OA, OB = orc_from_random(ra), orc_from_random(rb)
    C = ctx.gemm(A, B, 0.0, 0.0, precision="ozaki", split=7, alpha=0.7)
    ref = orc.to_dense(orc.gemm(OA, OB, 0.0, 0.0, alpha=0.7))
    got = C.to_dense().cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    log(f"  err={err:.2e}")
    assert err <= 1e-12
    with pytest.raises(clr.ClrError):
        ctx.gemm(A, B, 0.0, 0.0, precision="ozaki", split=9)


# ---------------------------------------------------------------------------
# Adjoints
# ---------------------------------------------------------------------------

def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("seed", [301, 302])
def test_gemm_backward_matches_oracle(ctx, torch, seed):
    """dA = alpha dC B^T, dB = alpha A^T dC on the stored blocks, all block kinds."""
    log(f"gemm backward seed={seed}")
    rs, ks, cs = [40, 17, 64, 33], [25, 48, 9, 70, 16], [31, 64, 12]
    ra = random_blocks(seed, rs, ks, p_zero=0.3, p_dense=0.4, max_rank=8)
    rb = random_blocks(seed + 50, ks, cs, p_zero=0.3, p_dense=0.4, max_rank=8)
    A, B = gpu_from_random(ctx, torch, ra), gpu_from_random(ctx, torch, rb)
    OA, OB = orc_from_random(ra), orc_from_random(rb)
    dC = rng_for(seed + 99).standard_normal((sum(rs), sum(cs)))
    alpha = 0.7
    dA, dB = ctx.gemm_backward(A, B, torch.from_numpy(dC).cuda(), alpha)
    rA, rB = orc.gemm_vjp(OA, OB, dC, alpha)
    eA, eB = _rel(dA.cpu().numpy(), rA), _rel(dB.cpu().numpy(), rB)
    log(f"  dA err {eA:.2e} dB err {eB:.2e}")
    assert eA <= FP64_BOUND and eB <= FP64_BOUND
    # zero blocks of A and B get exactly zero gradient
    mA, mB = orc.structure_mask(OA), orc.structure_mask(OB)
    assert np.all(dA.cpu().numpy()[mA == 0] == 0.0) and np.all(dB.cpu().numpy()[mB == 0] == 0.0)
    only_a, none_b = ctx.gemm_backward(A, B, torch.from_numpy(dC).cuda(), alpha, want_b=False)
    assert none_b is None and np.array_equal(only_a.cpu().numpy(), dA.cpu().numpy())


def test_sqrt_inv_backward_matches_oracle(ctx, torch):
    """dS through unrolled iterations (straight-through truncation) vs the oracle's VJP."""
    log("sqrt_inv backward line_n512")
    wl = line_n512()
    Sd = wl.dense()
    S = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    O = orc.compress(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10)
    mask = orc.structure_mask(O)
    Wbar = rng_for(5101).standard_normal(Sd.shape) * mask
    iters = 6
    dS, W = ctx.sqrt_inv_backward(S, torch.from_numpy(Wbar).cuda(), iters, 2, wl.tol, wl.eps_sp)
    ref, Ow, _info = orc.sqrt_inv_vjp(O, Wbar, iters, wl.tol, wl.eps_sp)
    err = _rel(dS.cpu().numpy(), ref)
    werr = _rel(W.to_dense().cpu().numpy(), orc.to_dense(Ow))
    log(f"  dS err {err:.2e}  W err {werr:.2e}")
    assert werr <= FP64_BOUND
    assert err <= FP64_BOUND
    assert np.all(dS.cpu().numpy()[mask == 0] == 0.0)
    # checkpoint spacing does not change the result (iterates are recomputed exactly)
    dS1, _ = ctx.sqrt_inv_backward(S, torch.from_numpy(Wbar).cuda(), iters, 1, wl.tol, wl.eps_sp)
    dS4, _ = ctx.sqrt_inv_backward(S, torch.from_numpy(Wbar).cuda(), iters, 4, wl.tol, wl.eps_sp)
    assert np.array_equal(dS1.cpu().numpy(), dS.cpu().numpy())
    assert np.array_equal(dS4.cpu().numpy(), dS.cpu().numpy())


def test_autograd_entry_points(ctx, torch):
    """torch.autograd through gemm_dense / sqrt_inv_dense equals the direct adjoint calls."""
    import paper_1509_00309_amd as clr
    log("autograd entry points")
    rs = [24, 40, 16]
    ra = random_blocks(401, rs, rs, p_zero=0.2, p_dense=0.5, max_rank=6)
    rb = random_blocks(402, rs, rs, p_zero=0.2, p_dense=0.5, max_rank=6)
    A, B = gpu_from_random(ctx, torch, ra), gpu_from_random(ctx, torch, rb)
    a = A.to_dense().clone().requires_grad_(True)
    b = B.to_dense().clone().requires_grad_(True)
    Cd = clr.gemm_dense(ctx, A, B, a, b, tol=0.0, eps_sp=0.0)
    Wt = torch.from_numpy(rng_for(403).standard_normal(Cd.shape)).cuda()
    (Cd * Wt).sum().backward()
    dA, dB = ctx.gemm_backward(A, B, Wt)
    assert torch.equal(a.grad, dA) and torch.equal(b.grad, dB)
    wl = line_n512()
    S = ctx.compress(torch.from_numpy(wl.dense()).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    s = S.to_dense().clone().requires_grad_(True)
    W = clr.sqrt_inv_dense(ctx, S, s, 4, 2, tol=wl.tol, eps_sp=wl.eps_sp)
    Wb = torch.from_numpy(rng_for(404).standard_normal(W.shape)).cuda()
    (W * Wb).sum().backward()
    dS, _ = ctx.sqrt_inv_backward(S, Wb, 4, 2, wl.tol, wl.eps_sp)
    assert torch.equal(s.grad, dS)


def test_torch_allocator_hook(torch):
    """A context whose matrices and work lists come from torch's caching allocator
    (clr_set_allocator through Context.use_torch_allocator) computes the same product, combination
    and S^-1/2 (direct and graph-replayed) bit for bit as one on hipMalloc; its matrices show up in
    torch's allocated bytes and are returned when released."""
    import gc
    import paper_1509_00309_amd as clr
    wl = line_n512()
    Sd = torch.from_numpy(wl.dense()).cuda()
    c1, c2 = clr.Context(), clr.Context()
    try:
        _torch_allocator_case(torch, clr, wl, Sd, c1, c2)
    finally:
        gc.collect()
        c2.close()
        c1.close()


def _torch_allocator_case(torch, clr, wl, Sd, c1, c2):
    import gc
    c2.use_torch_allocator()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    S1 = c1.compress(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10)
    S2 = c2.compress(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10)
    torch.cuda.synchronize()
    grown = torch.cuda.memory_allocated() - base
    _cap2, bytes2 = S2.arena()
    assert grown >= bytes2 > 0, (grown, bytes2)   # at least S2's storage (packed arena)
    _same_clr(torch, S1, S2)
    _same_clr(torch, c1.gemm(S1, S1, wl.tol, wl.eps_sp), c2.gemm(S2, S2, wl.tol, wl.eps_sp))
    _same_clr(torch, c1.axpby(0.5, S1, -0.25, S1, 1.0, wl.tol, wl.eps_sp),
              c2.axpby(0.5, S2, -0.25, S2, 1.0, wl.tol, wl.eps_sp))
    conv = wl.extra["conv_tol"]
    for graph in (False, True):
        W1, s1 = c1.sqrt_inv(S1, wl.tol, wl.eps_sp, conv_tol=conv, graph=graph,
                             allow_not_converged=True)
        W2, s2 = c2.sqrt_inv(S2, wl.tol, wl.eps_sp, conv_tol=conv, graph=graph,
                             allow_not_converged=True)
        assert s1.iterations == s2.iterations and s1.explicit_residual == s2.explicit_residual
        _same_clr(torch, W1, W2)
    del S2, W2
    gc.collect()
    c2.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - base < grown, "matrices not returned to torch"
    del S1, W1


def test_autograd_stand_in_checks(ctx, torch):
    """The dense stand-ins of gemm_dense / sqrt_inv_dense are checked against their handles:
    shape and dtype always, values on request."""
    import paper_1509_00309_amd as clr
    rs = [24, 40, 16]
    ra = random_blocks(405, rs, rs, p_zero=0.2, p_dense=0.5, max_rank=6)
    A = gpu_from_random(ctx, torch, ra)
    a = A.to_dense().clone().requires_grad_(True)
    with pytest.raises(ValueError, match="shape"):
        clr.gemm_dense(ctx, A, A, a[:, :-1], a, tol=0.0, eps_sp=0.0)
    with pytest.raises(ValueError, match="float64"):
        clr.gemm_dense(ctx, A, A, a.float(), a, tol=0.0, eps_sp=0.0)
    other = (a.detach() + 1e-3 * torch.ones_like(a)).requires_grad_(True)
    with pytest.raises(ValueError, match="differs"):
        clr.gemm_dense(ctx, A, A, other, a, verify_tol=1e-12, tol=0.0, eps_sp=0.0)
    Cd = clr.gemm_dense(ctx, A, A, a, a, verify_tol=1e-14, tol=0.0, eps_sp=0.0)
    assert Cd.shape == a.shape
    with pytest.raises(ValueError, match="differs"):
        clr.sqrt_inv_dense(ctx, A, other, 2, 1, verify_tol=1e-12, tol=1e-8, eps_sp=1e-10)


# ---------------------------------------------------------------------------
# Batches: one launch per phase, HIP graph replay
# ---------------------------------------------------------------------------

def _batch_operands(ctx, torch):
    ops = []
    for seed in (501, 502):
        rs, ks, cs = [40, 17, 64], [25, 48, 9, 70], [31, 64, 12, 20]
        ra = random_blocks(seed, rs, ks, p_zero=0.3, p_dense=0.4, max_rank=8)
        rb = random_blocks(seed + 50, ks, cs, p_zero=0.3, p_dense=0.4, max_rank=8)
        ops.append((gpu_from_random(ctx, torch, ra), gpu_from_random(ctx, torch, rb)))
    wl = line_n512()
    S = ctx.compress(torch.from_numpy(wl.dense()).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    ops.append((S, S))
    wl3 = scaled_workload("lattice", 1536, seed=143)
    S3 = ctx.compress(torch.from_numpy(wl3.dense()).cuda(), wl3.sizes, wl3.sizes, wl3.tol, 1e-10)
    ops.append((S3, S3))
    return ops


def test_gemm_batch_matches_single_products(ctx, torch):
    """A batch of products of different blockings equals the products one by one, bit for bit."""
    log("gemm batch vs single products")
    ops = _batch_operands(ctx, torch)
    As, Bs = [a for a, _ in ops], [b for _, b in ops]
    Cs, st = ctx.gemm_batch(As, Bs, 1e-8, 1e-10, stats=True)
    total = 0.0
    for (A, B), Cb in zip(ops, Cs):
        C1, s1 = ctx.gemm(A, B, 1e-8, 1e-10, stats=True)
        assert np.array_equal(Cb.to_dense().cpu().numpy(), C1.to_dense().cpu().numpy())
        kb, rb, nb = Cb.meta()
        k1, r1, n1 = C1.meta()
        assert np.array_equal(kb, k1) and np.array_equal(rb, r1) and np.array_equal(nb, n1)
        total += s1.flops_products
    assert abs(st.flops_products - total) <= 1e-9 * total
    log(f"  {len(ops)} products, {st.computed} blocks, {st.flops_products:.3e} flops")


def test_gemm_batch_against_oracle(ctx, torch):
    """Three products of different blockings and physics in one planned batch (one launch per
    phase for all, replayed as a HIP graph): the 3-D lattice at N = 1536, the 1-D line at
    N = 512 and a product of the 256-product batch (N = 2577, clusters up to 197, so dense
    blocks with short edges above 160), all truncated at 1e-8, each against the oracle block by
    block."""
    log("gemm batch against the oracle")
    tol, eps = 1e-8, 1e-10
    mats, orcs, nbs = [], [], []
    for wl in (scaled_workload("lattice", 1536, seed=147), line_n512(), batch_product(5)):
        Sd = wl.dense()
        mats.append(ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10))
        orcs.append(orc.compress(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10))
        nbs.append(len(wl.sizes) ** 2)
    plan = ctx.plan(mats, mats, tol, eps, graph=True)
    for _ in range(2):
        plan.execute()
    for C, O, nb in zip(plan.outputs, orcs, nbs):
        rep = parity.compare(C, orc.gemm(O, O, tol, eps), tol, exact=orc.gemm(O, O, 0.0, eps),
                             operands=(O, O))
        log("  " + parity.summary(rep))
        parity.assert_parity(rep, FP64_BOUND, nblocks=nb)
    plan.close()


def test_plan_graph_replay(ctx, torch):
    """A plan recorded as a HIP graph gives the eager result on every replay."""
    log("plan graph replay")
    ops = _batch_operands(ctx, torch)
    As, Bs = [a for a, _ in ops], [b for _, b in ops]
    ref = [c.to_dense().cpu().numpy() for c in ctx.gemm_batch(As, Bs, 1e-8, 1e-10)]
    plan = ctx.plan(As, Bs, 1e-8, 1e-10, graph=True)
    for rep in range(3):
        plan.execute()
        got = [c.to_dense().cpu().numpy() for c in plan.outputs]
        for g, r in zip(got, ref):
            assert np.array_equal(g, r), f"replay {rep} differs"
        # unrelated eager work between replays
        X = ctx.gemm(As[0], Bs[0], 0.0, 0.0)
        del X
        torch.cuda.synchronize()
    plan.close()


def test_tile_edges_and_autotune(ctx, torch):
    """Item edges, one per launch class or one per shape class, change launch shapes only:
    results are bit-identical; the autotuner returns admissible edges (launch classes, then
    every shape class) and leaves them set."""
    log("tile edges and autotune")
    wl = scaled_workload("lattice", 1536, seed=144)
    S = ctx.compress(torch.from_numpy(wl.dense()).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    ref = ctx.gemm(S, S, wl.tol, wl.eps_sp).to_dense().cpu().numpy()
    for de, te in ((32, 64), (96, 48), (64, 32)):
        ctx.set_tile_edges("fp64", de, te)
        got = ctx.gemm(S, S, wl.tol, wl.eps_sp).to_dense().cpu().numpy()
        assert np.array_equal(got, ref), (de, te)
    import paper_1509_00309_amd as clr
    with pytest.raises(clr.ClrError):
        ctx.set_tile_edges("fp64", 40, 0)
    # per shape class: every class table gives the same result, bit for bit
    for dense, thin in (([32, 48, 64, 96, 112, 160], [16, 32, 48, 64, 16]),
                        ([160, 16, 32, 48, 64, 80], [64, 16, 32, 16, 48])):
        ctx.set_tile_classes("fp64", dense, thin)
        assert ctx.get_tile_classes("fp64") == (dense, thin)
        got = ctx.gemm(S, S, wl.tol, wl.eps_sp).to_dense().cpu().numpy()
        assert np.array_equal(got, ref), (dense, thin)
    with pytest.raises(clr.ClrError):
        ctx.set_tile_classes("fp64", [32, 48, 64, 96, 112, 176], [16, 32, 48, 64, 16])
    res = ctx.autotune(S, S, wl.tol, wl.eps_sp)
    log(f"  autotune: {res}")
    assert res["dense_edge"] in (32, 64, 96, 128, 160) and res["thin_edge"] in (32, 64)
    assert all(e in (32, 64, 96, 128, 160) for e in res["dense_classes"])
    assert all(e in (16, 32, 48, 64) for e in res["thin_classes"])
    assert ctx.get_tile_classes("fp64") == (res["dense_classes"], res["thin_classes"])
    got = ctx.gemm(S, S, wl.tol, wl.eps_sp).to_dense().cpu().numpy()
    assert np.array_equal(got, ref)
    ctx.set_tile_edges("fp64", 0, 0)


# ---------------------------------------------------------------------------
# Full size (the benchmark's workload and launch configuration), largest block
# edge, and the adjoint against finite differences and the eigen-gradient
# ---------------------------------------------------------------------------

def test_construction_rrqr_full_size_sampled(ctx, torch):
    """The N = 8192 input as the construction leg of bench.py builds it, but generated on the
    device: 28 sampled blocks of the generated matrix against the host generator, and of the
    RRQR-compressed matrix against the oracle's column-pivoted QR one block at a time (kind,
    rank, U^T U = I, V = M^T U, the error bound, and the oracle's reconstruction unless a
    pivot near-tie or a cut on the threshold separates them)."""
    log("construction by RRQR, N=8192, sampled blocks")
    wl = lattice_3d(8192)
    Sd = wl.dense()
    G = ctx.kernel_matrix(torch.from_numpy(wl.points).cuda(), "gaussian", wl.a, wl.diag)
    S = ctx.compress(G, wl.sizes, wl.sizes, wl.tol, 1e-10, method="rrqr")
    kind, rank, _norm = S.meta()
    offs = wl.offsets()
    nb = len(wl.sizes)
    rng = rng_for(8193)
    picks = [(i, i) for i in rng.choice(nb, 4, replace=False)]
    picks += [(i, min(nb - 1, i + 1)) for i in rng.choice(nb, 8, replace=False)]
    picks += [(int(rng.integers(nb)), int(rng.integers(nb))) for _ in range(16)]
    same = differ = 0
    for (i, j) in picks:
        M = Sd[offs[i]:offs[i + 1], offs[j]:offs[j + 1]]
        g = G[offs[i]:offs[i + 1], offs[j]:offs[j + 1]].cpu().numpy()
        assert np.all(np.abs(g - M) <= 4.5e-16 * np.abs(M) + 1e-300)
        m, n = M.shape
        nm = np.linalg.norm(M)
        r, _X, _W, tails = orc.rrqr_truncate(M, wl.tol)
        want = 0 if nm < 1e-10 else (1 if i == j or 2 * r > min(m, n) else 2)
        k = int(kind[i, j])
        if k != want or (k == 2 and int(rank[i, j]) != r):
            assert any(abs(t - wl.tol * nm) <= 1e-6 * wl.tol * nm for t in tails), \
                (i, j, k, want, int(rank[i, j]), r)
            differ += 1
            continue
        if k != 2:
            continue
        _t, U, V = S.block(i, j, m, n, 2, int(rank[i, j]))
        U, V = U.cpu().numpy(), V.cpu().numpy()
        assert np.linalg.norm(U.T @ U - np.eye(U.shape[1])) <= 1e-13 * U.shape[1]
        assert np.linalg.norm(V - M.T @ U) <= 1e-13 * nm
        assert np.linalg.norm(M - U @ V.T) <= wl.tol * nm * (1 + 1e-9)
        if np.linalg.norm(U @ V.T - _X @ _W.T) <= 1e-12 * nm:
            same += 1
        else:
            differ += 1
    log(f"  {len(picks)} blocks: {same} factored blocks equal to the oracle's, {differ} at ties")
    assert differ <= 2


@pytest.mark.parametrize("name,precision", [("lattice_3d", "fp64"), ("lattice_3d_morton", "fp64"),
                                            ("coulomb_3d_morton", "fp64"), ("lattice_3d", "ozaki")])
def test_gemm_full_size_sampled(ctx, torch, name, precision):
    """The N = 8192 workloads exactly as bench.py times them (the 3D lattice product in the FP64
    and operand-split forms, and the two low-rank-regime products); 32 result blocks recomputed
    one by one by the oracle (kinds, ranks and values)."""
    import workloads
    log(f"gemm full size N=8192 ({name}, {precision}), sampled blocks")
    wl = getattr(workloads, name)(8192)
    Sd = wl.dense()
    S = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    C = ctx.gemm(S, S, wl.tol, wl.eps_sp, precision=precision)
    kind, rank, _norm = C.meta()
    Dg = C.to_dense().cpu().numpy()
    O = orc.compress(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10)
    offs = wl.offsets()
    nb = len(wl.sizes)
    rng = rng_for(8192)
    picks = [(i, i) for i in rng.choice(nb, 4, replace=False)]
    picks += [(i, min(nb - 1, i + 1)) for i in rng.choice(nb, 8, replace=False)]
    picks += [(int(rng.integers(nb)), int(rng.integers(nb))) for _ in range(20)]
    num = den = 0.0
    worst = 0.0
    seen = {0: 0, 1: 0, 2: 0}
    ambiguous = 0
    est = parity.operand_scale(O, O)
    for (i, j) in picks:
        ob = orc.gemm_block(O, O, i, j, wl.tol, wl.eps_sp)
        m, n = wl.sizes[i], wl.sizes[j]
        ref = ob.dense() if ob is not None else np.zeros((m, n))
        got = Dg[offs[i]:offs[i + 1], offs[j]:offs[j + 1]]
        ok = 0 if ob is None else (1 if ob.kind == "D" else 2)
        seen[int(kind[i, j])] += 1
        if int(kind[i, j]) != ok or (ok == 2 and int(rank[i, j]) != ob.rank):
            # a cut on a tie of the truncation rule: judged on the untruncated block
            eb = orc.gemm_block(O, O, i, j, 0.0, wl.eps_sp)
            rk = [int(rank[i, j]) if kind[i, j] else 0, ob.rank if ok == 2 else 0]
            assert eb is not None and parity.ambiguous_cut(eb.dense(), wl.tol, rk), \
                (i, j, int(kind[i, j]), ok, int(rank[i, j]), ob.rank if ob else 0)
            ambiguous += 1
            continue
        num += float(np.sum((got - ref) ** 2))
        den += float(np.sum(ref ** 2))
        if ok:   # each block against max(||C_IJ||, 1e-2 est_IJ), as parity.compare does
            bref = max(math.sqrt(float(np.sum(ref ** 2))), 1e-2 * float(est[i, j]))
            worst = max(worst, math.sqrt(float(np.sum((got - ref) ** 2))) / bref)
    err = math.sqrt(num / den)
    log(f"  {len(picks)} blocks (kinds {seen}, {ambiguous} ambiguous cuts), rel err {err:.2e}, "
        f"worst block {worst:.2e}")
    assert ambiguous <= 1
    assert err <= FP64_BOUND
    # The operand-split form quantises each 64-deep chunk of a row (column) against the chunk's
    # largest entry, so a small term sharing a chunk with a large one keeps an absolute error of
    # about 2^-49 of that entry: about 1e-11 est_IJ, a large relative error for a block far below
    # its operand scale.  Its block bar is therefore 1e-8, the whole-sample bar the FP64 one.
    assert worst <= (FP64_BOUND if precision == "fp64" else 1e-8)


def test_gemm_largest_block_edge(ctx, torch):
    """Blocks up to the largest supported edge (512) take the general recompression path."""
    log("gemm with 512-edge blocks")
    rs, ks = [512, 300, 48], [512, 200]
    ra = random_blocks(601, rs, ks, p_zero=0.0, p_dense=0.5, max_rank=24)
    rb = random_blocks(602, ks, rs, p_zero=0.0, p_dense=0.5, max_rank=24)
    A, B = gpu_from_random(ctx, torch, ra), gpu_from_random(ctx, torch, rb)
    OA, OB = orc_from_random(ra), orc_from_random(rb)
    for tol in (1e-8, 0.0):
        C = ctx.gemm(A, B, tol, 1e-10)
        Oc = orc.gemm(OA, OB, tol, 1e-10)
        rep = parity.compare(C, Oc, tol, operands=(OA, OB))
        log(f"  tol={tol:g} err={rep.rel_err:.2e}")
        log("  " + parity.summary(rep))
        parity.assert_parity(rep, FP64_BOUND, nblocks=9)



def test_gemm_many_terms_per_block(ctx, torch):
    """Result blocks with more inner terms than the grouped GEMM caches in LDS (256): their
    term descriptors are read from global memory on every slab.  FP64 to the oracle's bar;
    the mixed forms on the same path within FP32 rounding of the FP64 product (random
    N(0,1) operands over ~1500 inner indices, so not the 10 x tol bar of the decaying
    workloads)."""
    log("gemm with 300 inner blocks")
    rs, cs = [40, 24], [32, 17]
    ks = [3 + (7 * i) % 5 for i in range(300)]
    ra = random_blocks(611, rs, ks, p_zero=0.02, p_dense=0.5, max_rank=2)
    rb = random_blocks(612, ks, cs, p_zero=0.02, p_dense=0.5, max_rank=2)
    terms = ((ra.kind != 0).astype(int) @ (rb.kind != 0).astype(int))
    assert terms.max() > 256, terms
    A, B = gpu_from_random(ctx, torch, ra), gpu_from_random(ctx, torch, rb)
    OA, OB = orc_from_random(ra), orc_from_random(rb)
    for tol in (1e-8, 0.0):
        C = ctx.gemm(A, B, tol, 1e-10)
        Oc = orc.gemm(OA, OB, tol, 1e-10)
        rep = parity.compare(C, Oc, tol, operands=(OA, OB))
        log(f"  tol={tol:g} " + parity.summary(rep))
        parity.assert_parity(rep, FP64_BOUND, nblocks=4)
    ref = ctx.gemm(A, B, 0.0, 1e-10).to_dense()
    for split in (0, 1):
        Cm = ctx.gemm(A, B, 0.0, 1e-10, precision="mixed", split=split).to_dense()
        err = float(torch.linalg.norm(Cm - ref) / torch.linalg.norm(ref))
        log(f"  mixed split={split} rel err vs FP64 {err:.2e}")
        assert err < 1e-5

def _alpha_of(S):
    _k, _r, norm = S.meta()
    return 1.0 / float(np.max(np.sum(norm, axis=1)))


def test_sqrt_inv_backward_finite_differences(ctx, torch):
    """dS by the adjoint vs central differences (h = 1e-6) on 32 stored entries,
    truncation off, alpha held fixed."""
    log("sqrt_inv backward vs finite differences")
    wl = line_n512()
    Sd = wl.dense()
    S = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, 0.0, 1e-10)
    alpha = _alpha_of(S)
    kind, _r, _n = S.meta()
    offs = wl.offsets()
    mask = np.zeros_like(Sd)
    for I in range(len(wl.sizes)):
        for J in range(len(wl.sizes)):
            if kind[I, J]:
                mask[offs[I]:offs[I + 1], offs[J]:offs[J + 1]] = 1.0
    Wbar = rng_for(7101).standard_normal(Sd.shape) * mask
    iters = 6
    dS, _ = ctx.sqrt_inv_backward(S, torch.from_numpy(Wbar).cuda(), iters, 2, 0.0, 0.0, alpha=alpha)
    dS = dS.cpu().numpy()
    rng = rng_for(7102)
    idx = np.argwhere(mask > 0)
    pick = idx[rng.choice(len(idx), 32, replace=False)]
    h = 1e-6

    def loss(M):
        X = ctx.compress(torch.from_numpy(M).cuda(), wl.sizes, wl.sizes, 0.0, 1e-10)
        W, _st = ctx.sqrt_inv(X, 0.0, 0.0, fixed_iters=iters, alpha=alpha)
        return float(np.sum(Wbar * W.to_dense().cpu().numpy()))

    fd, ad = [], []
    for (i, j) in pick:
        Sp, Sm = Sd.copy(), Sd.copy()
        Sp[i, j] += h
        Sm[i, j] -= h
        fd.append((loss(Sp) - loss(Sm)) / (2 * h))
        ad.append(dS[i, j])
    fd, ad = np.array(fd), np.array(ad)
    err = float(np.max(np.abs(fd - ad)) / np.max(np.abs(ad)))
    log(f"  max |fd - adjoint| / max |adjoint| = {err:.2e}")
    assert err <= 1e-6


def test_sqrt_inv_backward_eigen_gradient(ctx, torch):
    """Converged iteration (truncation off): dS equals the Daleckii-Krein gradient of
    S^-1/2, Q (Gamma o (Q^T Wbar Q)) Q^T with Gamma_ij = -1/(sqrt(l_i) sqrt(l_j)
    (sqrt(l_i) + sqrt(l_j))), on S's stored blocks."""
    log("sqrt_inv backward vs Daleckii-Krein")
    wl = scaled_workload("lattice", 768, nclusters=6, seed=145)
    Sd = wl.dense()
    S = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, 0.0, 1e-10)
    kind, _r, _n = S.meta()
    offs = wl.offsets()
    mask = np.zeros_like(Sd)
    for I in range(len(wl.sizes)):
        for J in range(len(wl.sizes)):
            if kind[I, J]:
                mask[offs[I]:offs[I + 1], offs[J]:offs[J + 1]] = 1.0
    Wbar = rng_for(7201).standard_normal(Sd.shape) * mask
    dS, W = ctx.sqrt_inv_backward(S, torch.from_numpy(Wbar).cuda(), 20, 5, 0.0, 0.0)
    lam, Q = np.linalg.eigh(Sd)
    sq = np.sqrt(lam)
    gam = -1.0 / (np.outer(sq, sq) * (sq[:, None] + sq[None, :]))
    ref = (Q @ (gam * (Q.T @ Wbar @ Q)) @ Q.T) * mask
    err = float(np.linalg.norm(dS.cpu().numpy() - ref) / np.linalg.norm(ref))
    werr = float(np.linalg.norm(W.to_dense().cpu().numpy() - (Q / sq) @ Q.T) / np.linalg.norm((Q / sq) @ Q.T))
    log(f"  dS vs eigen-gradient {err:.2e}, W vs eigh {werr:.2e}")
    assert werr <= 1e-10
    assert err <= 1e-8


def test_sqrt_inv_backward_eigen_gradient_n4096(ctx, torch):
    """The differentiation workload at its size: N = 4096, 32 clusters, tol 1e-8, 20 unrolled
    iterations with a checkpoint every 5, Wbar ~ N(0, 1) masked to S's blocks.  dS against the
    Daleckii-Krein gradient of the dense S^-1/2 of the same compressed S (FP64 eigendecomposition
    on the host) and W against S^-1/2, each within 1e-7 (measured: 5.2e-9 and 2.5e-9; the
    truncation at 1e-8 per product sets that level)."""
    from workloads import adjoint_n4096
    log("sqrt_inv backward N=4096 (tol 1e-8, 20 iterations, checkpoint 5) vs Daleckii-Krein")
    wl = adjoint_n4096()
    S = ctx.compress(torch.from_numpy(wl.dense()).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    kind, _r, _n = S.meta()
    offs = wl.offsets()
    mask = np.zeros((wl.n, wl.n))
    for I in range(len(wl.sizes)):
        for J in range(len(wl.sizes)):
            if kind[I, J]:
                mask[offs[I]:offs[I + 1], offs[J]:offs[J + 1]] = 1.0
    Wbar = wl.extra["weights"] * mask
    dS, W = ctx.sqrt_inv_backward(S, torch.from_numpy(Wbar).cuda(), wl.extra["iters"],
                                  wl.extra["checkpoint_every"], wl.tol, wl.eps_sp)
    Sc = S.to_dense().cpu().numpy()
    lam, Q = np.linalg.eigh(0.5 * (Sc + Sc.T))
    sq = np.sqrt(lam)
    gam = -1.0 / (np.outer(sq, sq) * (sq[:, None] + sq[None, :]))
    ref = (Q @ (gam * (Q.T @ Wbar @ Q)) @ Q.T) * mask
    wref = (Q / sq) @ Q.T
    err = float(np.linalg.norm(dS.cpu().numpy() - ref) / np.linalg.norm(ref))
    werr = float(np.linalg.norm(W.to_dense().cpu().numpy() - wref) / np.linalg.norm(wref))
    log(f"  dS vs eigen-gradient {err:.2e}, W vs eigh {werr:.2e}")
    assert np.all(dS.cpu().numpy()[mask == 0] == 0.0)
    assert werr <= 1e-7
    assert err <= 1e-7


def _blocks_of(M, sizes):
    """Every stored block of M as host arrays (through the block accessor)."""
    kind, rank, _n = M.meta()
    out = {}
    for I in range(len(sizes)):
        for J in range(len(sizes)):
            if kind[I, J]:
                f = M.block(I, J, sizes[I], sizes[J], int(kind[I, J]), int(rank[I, J]))
                out[(I, J)] = [x.cpu().numpy() for x in f[1:]]
    return out


def test_packed_storage_and_compaction(ctx, torch):
    """Storage follows the ranks.  Created and compressed matrices are packed (arena = stored
    elements: m n per dense block, (m + n) r per factored block); a product reserves per block the
    most its result can store (between the stored elements and N^2) and compaction gives the rest
    back.  Layout changes nothing else: after compaction the values, kinds, ranks, norms and every
    block are bit for bit the same, and a product of compacted operands equals the product of the
    planned ones bit for bit."""
    log("packed storage: create, compress, product room, compaction")
    rc = random_blocks(160, [30, 45, 12, 64], [50, 20, 33], p_zero=0.2, p_dense=0.4)
    M = gpu_from_random(ctx, torch, rc)
    cap, nbytes = M.arena()
    assert cap == M.stored_elements() and nbytes >= 8 * cap
    wl = scaled_workload("morton", 2048, seed=151)
    Sd = wl.dense()
    S = ctx.compress(torch.from_numpy(Sd).cuda(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    cap_s, _ = S.arena()
    log(f"  compressed S: arena {cap_s} doubles = stored, {cap_s / wl.n ** 2:.3f} of N^2")
    assert cap_s == S.stored_elements() < wl.n ** 2
    C = ctx.gemm(S, S, wl.tol, wl.eps_sp)
    cap_c, _ = C.arena()
    stored = C.stored_elements()
    log(f"  product room {cap_c} doubles for {stored} stored ({cap_c / wl.n ** 2:.3f} of N^2)")
    assert stored <= cap_c <= wl.n ** 2
    dense0 = C.to_dense().cpu().numpy()
    meta0 = C.meta()
    blocks0 = _blocks_of(C, wl.sizes)
    P0 = ctx.gemm(C, S, wl.tol, wl.eps_sp)
    C.compact()
    assert C.arena()[0] == stored
    assert np.array_equal(C.to_dense().cpu().numpy(), dense0)
    for a, b in zip(C.meta(), meta0):
        assert np.array_equal(a, b)
    blocks1 = _blocks_of(C, wl.sizes)
    assert blocks1.keys() == blocks0.keys()
    for key in blocks0:
        for x, y in zip(blocks1[key], blocks0[key]):
            assert np.array_equal(x, y)
    P1 = ctx.gemm(C, S, wl.tol, wl.eps_sp)
    _bitwise_same(P0, P1)
    # compacting a packed matrix keeps it as it is
    C.compact()
    assert C.arena()[0] == stored
    assert np.array_equal(C.to_dense().cpu().numpy(), dense0)
