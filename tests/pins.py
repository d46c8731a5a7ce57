"""Pins that tie the CPU oracle to facts fixed by the paper and by mathematics.

Each ``pin_*`` function runs one check against the oracle module passed in and
returns the worst error it saw (0 for exact checks).  The test suite asserts
each is below its bound; the mutation tests plant a mistake in a copy of the
oracle and assert that at least one pin then fails.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from workloads import line_n512, random_blocks, rng_for


# ---------------------------------------------------------------------------
# Independent references (no oracle code)
# ---------------------------------------------------------------------------

def triple_loop(A, B):
    """Textbook C_ij = sum_k A_ik B_kj with Python floats, ascending k."""
    n, kdim = len(A), len(A[0])
    m = len(B[0])
    C = [[0.0] * m for _ in range(n)]
    for i in range(n):
        for j in range(m):
            s = 0.0
            for k in range(kdim):
                s += A[i][k] * B[k][j]
            C[i][j] = s
    return C


def integer_clr(seed, row_sizes, col_sizes, p_zero=0.2, p_dense=0.4):
    """Random CLR factors with small-integer entries so every product is exact in FP64."""
    rc = random_blocks(seed, row_sizes, col_sizes, p_zero=p_zero, p_dense=p_dense)
    rng = rng_for(seed + 17)
    for key in list(rc.f0):
        rc.f0[key] = rng.integers(-3, 4, size=rc.f0[key].shape).astype(np.float64)
    for key in list(rc.f1):
        rc.f1[key] = rng.integers(-3, 4, size=rc.f1[key].shape).astype(np.float64)
    return rc


def dense_from_factors(rc):
    ro = np.concatenate([[0], np.cumsum(rc.row_sizes)]).astype(int)
    co = np.concatenate([[0], np.cumsum(rc.col_sizes)]).astype(int)
    out = np.zeros((ro[-1], co[-1]))
    for (i, j), f in rc.f0.items():
        blk = f if rc.kind[i, j] == 1 else f @ rc.f1[(i, j)].T
        out[ro[i]:ro[i + 1], co[j]:co[j + 1]] = blk
    return out


def random_orthogonal(rng, n):
    """Householder product of n random reflectors (an orthogonal matrix, no LAPACK)."""
    Q = np.eye(n)
    for _ in range(n):
        v = rng.standard_normal(n)
        v /= np.sqrt(v @ v)
        Q = Q - 2.0 * np.outer(Q @ v, v)
    return Q


def ns_scalar(lam, alpha, iters):
    """Scalar form of Eqs. (8)-(11) for a 1x1 matrix lam: returns sqrt(alpha) z_n."""
    y, z = lam, 1.0
    for _ in range(iters):
        x = alpha * y * z
        t = (-10.0 * x + 3.0 * x * x + 15.0) / 8.0
        z, y = z * t, t * y
    return math.sqrt(alpha) * z


# ---------------------------------------------------------------------------
# Pins
# ---------------------------------------------------------------------------

def pin_triple_loop_exact(orc, seed=11):
    """Integer-valued inputs, tol = 0, eps_sp = 0: the CLR product equals the triple loop exactly."""
    rows, inner, cols = [3, 5, 2, 4], [4, 2, 6], [5, 3, 4, 2]
    ra = integer_clr(seed, rows, inner)
    rb = integer_clr(seed + 1, inner, cols)
    A = orc.from_factors(ra.row_sizes, ra.col_sizes, ra.kind, ra.f0, ra.f1)
    B = orc.from_factors(rb.row_sizes, rb.col_sizes, rb.kind, rb.f0, rb.f1)
    C = orc.to_dense(orc.gemm(A, B, tol=0.0, eps_sp=0.0))
    ref = np.array(triple_loop(dense_from_factors(ra).tolist(), dense_from_factors(rb).tolist()))
    return float(np.max(np.abs(C - ref)))


def pin_product_kinds(orc, seed=12):
    """Each block product (DD, LD, DL, LL, both absorb sides) equals the dense product (Eq. (4))."""
    rng = rng_for(seed)
    worst = 0.0
    m, k, n = 7, 9, 6
    cases = []
    Ad, Bd = rng.standard_normal((m, k)), rng.standard_normal((k, n))
    Ua, Va = rng.standard_normal((m, 3)), rng.standard_normal((k, 3))
    Ub, Vb = rng.standard_normal((k, 2)), rng.standard_normal((n, 2))
    Ub4, Vb4 = rng.standard_normal((k, 4)), rng.standard_normal((n, 4))
    Ub3, Vb3 = rng.standard_normal((k, 3)), rng.standard_normal((n, 3))
    a_d = orc.Block("D", D=Ad)
    a_l = orc.Block("L", U=Ua, V=Va)
    for b in [orc.Block("D", D=Bd), orc.Block("L", U=Ub, V=Vb), orc.Block("L", U=Ub4, V=Vb4),
              orc.Block("L", U=Ub3, V=Vb3)]:
        for a in (a_d, a_l):
            cases.append((a, b))
    for a, b in cases:
        term = orc.block_product(a, b, alpha=1.5)
        got = term[1] if term[0] == "D" else term[1] @ term[2].T
        ref = 1.5 * (a.dense() @ b.dense())
        worst = max(worst, float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
        if a.kind == "L" and b.kind == "L":
            # output rank = min(r_A, r_B) (Eq. (4) and the text after it)
            if term[1].shape[1] != min(a.rank, b.rank):
                return math.inf
            # the tie goes to the W side: U factor is alpha * U_A itself
            if a.rank == b.rank and not np.array_equal(term[1], 1.5 * a.U):
                return math.inf
    return worst


def spectrum_matrix(rng, m, n, s):
    Q1 = random_orthogonal(rng, m)[:, : len(s)]
    Q2 = random_orthogonal(rng, n)[:, : len(s)]
    return (Q1 * s) @ Q2.T


def pin_eckart_young(orc, seed=13):
    """Truncation keeps the smallest admissible rank and its error equals the dropped tail."""
    rng = rng_for(seed)
    worst = 0.0
    m, n = 12, 10
    s = np.array([3.0, 1.0, 0.5, 0.2, 1e-2, 3e-3, 1e-4, 2e-5, 1e-6, 1e-8])
    D = spectrum_matrix(rng, m, n, s)
    normc = math.sqrt(float(np.sum(s ** 2)))
    for tol in (1e-1, 3e-2, 1e-3, 1e-5):
        tails = [math.sqrt(float(np.sum(s[r:] ** 2))) for r in range(len(s) + 1)]
        r_ref = min(r for r in range(len(s) + 1) if tails[r] <= tol * normc)
        r = orc.truncation_rank(s, tol, normc)
        if r != r_ref:
            return math.inf
        blk = orc.combine(m, n, [("D", D)], tol, 0.0, False)
        if 2 * r_ref > min(m, n):
            if blk.kind != "D":
                return math.inf
            continue
        if blk.kind != "L" or blk.rank != r_ref:
            return math.inf
        err = float(np.sqrt(np.sum((D - blk.U @ blk.V.T) ** 2)))
        worst = max(worst, abs(err - tails[r_ref]) / normc)
        worst = max(worst, abs(blk.norm - math.sqrt(float(np.sum(s[:r_ref] ** 2)))) / normc)
        # U orthonormal (X = Q_r convention)
        worst = max(worst, float(np.max(np.abs(blk.U.T @ blk.U - np.eye(r_ref)))))
    return worst


def pin_lowrank_recompression(orc, seed=14):
    """Concatenated factors recompress to the true rank and reproduce the sum (Eqs. (5)-(7))."""
    rng = rng_for(seed)
    m, n = 40, 80
    basis_u = rng.standard_normal((m, 5))
    basis_v = rng.standard_normal((n, 5))
    pieces = []
    for r in (3, 4, 5):            # R_cat = 12, 2*12 < 40: stays on the low-rank path
        pieces.append(("L", basis_u @ rng.standard_normal((5, r)), basis_v @ rng.standard_normal((5, r))))
    ref = sum(p[1] @ p[2].T for p in pieces)
    blk = orc.combine(m, n, pieces, 1e-12, 0.0, False)
    if blk is None or blk.kind != "L" or blk.rank != 5:
        return math.inf
    worst = float(np.max(np.abs(blk.U @ blk.V.T - ref)) / np.max(np.abs(ref)))
    worst = max(worst, abs(blk.norm - float(np.sqrt(np.sum(ref ** 2)))) / float(np.sqrt(np.sum(ref ** 2))))
    return worst


def pin_screening(orc, seed=15):
    """Norm estimates bound the exact block norms; screened blocks are exactly those below tau."""
    rows, inner, cols = [6, 5, 7, 4, 6], [5, 6, 4, 7], [6, 5, 7, 4, 6]
    ra = random_blocks(seed, rows, inner, p_zero=0.1, scale_decay=3.0)
    rb = random_blocks(seed + 1, inner, cols, p_zero=0.1, scale_decay=3.0)
    A = orc.from_factors(ra.row_sizes, ra.col_sizes, ra.kind, ra.f0, ra.f1)
    B = orc.from_factors(rb.row_sizes, rb.col_sizes, rb.kind, rb.f0, rb.f1)
    exact = orc.gemm(A, B, tol=0.0, eps_sp=0.0)
    Ad, Bd = dense_from_factors(ra), dense_from_factors(rb)
    ro = np.concatenate([[0], np.cumsum(rows)])
    co = np.concatenate([[0], np.cumsum(cols)])
    ko = np.concatenate([[0], np.cumsum(inner)])
    tau = 1e-2
    screened = orc.gemm(A, B, tol=0.0, eps_sp=tau)
    worst = 0.0
    for i in range(len(rows)):
        for j in range(len(cols)):
            blk = Ad[ro[i]:ro[i + 1]] @ Bd[:, co[j]:co[j + 1]]
            true_norm = float(np.sqrt(np.sum(blk ** 2)))
            est = 0.0
            for k in range(len(inner)):
                na = float(np.sqrt(np.sum(Ad[ro[i]:ro[i + 1], ko[k]:ko[k + 1]] ** 2)))
                nb = float(np.sqrt(np.sum(Bd[ko[k]:ko[k + 1], co[j]:co[j + 1]] ** 2)))
                est += na * nb
            if true_norm > est * (1 + 1e-12):
                return math.inf
            kept = (i, j) in screened.blocks
            if kept != (est >= tau and true_norm >= tau):
                return math.inf
            if (i, j) in exact.blocks:
                worst = max(worst, abs(exact.blocks[(i, j)].norm - true_norm) / max(true_norm, 1e-300))
    return worst


def pin_ns_coefficients(orc):
    """Eq. (9) on 1x1 blocks: T = (-10 x + 3 x^2 + 15)/8 for exact rational x (coefficients from the paper)."""
    worst = 0.0
    for x in (Fraction(1, 2), Fraction(3, 4), Fraction(1, 1), Fraction(5, 4), Fraction(1, 8)):
        xf = float(x)
        X = orc.OMatrix([1], [1], {(0, 0): orc.Block("D", D=np.array([[xf]]), norm=abs(xf))})
        Q = orc.OMatrix([1], [1], {(0, 0): orc.Block("D", D=np.array([[xf * xf]]), norm=xf * xf)})
        T = orc.ns_T(X, Q, tol=0.0, eps_sp=0.0)
        ref = (Fraction(-10) * x + 3 * x * x + 15) / 8
        worst = max(worst, abs(float(T.blocks[(0, 0)].D[0, 0]) - float(ref)))
    return worst


def pin_ns_diagonal(orc):
    """Diagonal S reduces Eqs. (8)-(11) to independent scalar recurrences."""
    lam = [0.15, 0.4, 0.9, 1.7, 2.5, 0.6]
    sizes = [2, 3, 1]
    D = np.diag(lam)
    S = orc.compress(D, sizes, sizes, tol=0.0, drop=0.0)
    alpha = 0.37
    worst = 0.0
    for iters in (1, 2, 5, 12):
        W, _info = orc.sqrt_inv(S, tol=0.0, eps_sp=0.0, fixed_iters=iters, alpha=alpha)
        Wd = orc.to_dense(W)
        ref = np.diag([ns_scalar(l, alpha, iters) for l in lam])
        worst = max(worst, float(np.max(np.abs(Wd - ref))))
    # converged value is lam^-1/2
    W, _ = orc.sqrt_inv(S, tol=0.0, eps_sp=0.0, fixed_iters=12, alpha=alpha)
    worst = max(worst, float(np.max(np.abs(np.diag(orc.to_dense(W)) - np.array(lam) ** -0.5))))
    return worst


def pin_sqrt_inv_eigh(orc):
    """S^-1/2 of the 1D N = 512 overlap-like matrix against an eigendecomposition of the same S."""
    wl = line_n512()
    S = orc.compress(wl.dense(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    W, info = orc.sqrt_inv(S, wl.tol, wl.eps_sp, conv_tol=wl.extra["conv_tol"])
    Sd = orc.to_dense(S)
    lam, Q = np.linalg.eigh(0.5 * (Sd + Sd.T))
    ref = (Q * lam ** -0.5) @ Q.T
    err = float(np.sqrt(np.sum((orc.to_dense(W) - ref) ** 2)) / np.sqrt(np.sum(ref ** 2)))
    return err, info


def pin_cubic_rate(orc):
    """Third-order contraction.  For 1x1 S the error e = 1 - x obeys e' = (5/8) e^3 + O(e^4)
    (expand x p(x)^2 with p(x) = (15 - 10x + 3x^2)/8); for N x N S the measure
    a = ||X - I||_F / sqrt(N) satisfies a' <= (5/8) N a^3 to leading order (all error in one
    eigenvalue is the worst case).  Returns (worst scalar deviation from 5/8, worst matrix
    ratio a'/((5/8) N a^3), residual history)."""
    worst_scalar = 0.0
    for lam in (0.95, 1.05, 0.98):
        S1 = orc.compress(np.array([[lam]]), [1], [1], tol=0.0, drop=0.0)
        _W, info = orc.sqrt_inv(S1, tol=0.0, eps_sp=0.0, fixed_iters=2, alpha=1.0)
        e0, e1 = info.internal[0], info.internal[1]
        worst_scalar = max(worst_scalar, abs(e1 / e0 ** 3 - 5.0 / 8.0))
    rng = rng_for(16)
    n = 30
    Q = random_orthogonal(rng, n)
    lam = np.linspace(0.3, 3.0, n)
    Sd = (Q * lam) @ Q.T
    sizes = [10, 12, 8]
    S = orc.compress(Sd, sizes, sizes, tol=0.0, drop=0.0)
    _W, info = orc.sqrt_inv(S, tol=0.0, eps_sp=0.0, fixed_iters=8)
    e = info.internal
    worst = 0.0
    for a, b in zip(e[:-1], e[1:]):
        if 1e-4 < a < 0.05:
            worst = max(worst, b / (0.625 * n * a ** 3))
    return worst_scalar, worst, e


def pin_dense_limit(orc):
    """tol -> 0, eps_sp -> 0: the CLR product is the dense product (Sec. 4.1, accuracy knobs)."""
    wl = line_n512()
    Sd = wl.dense()
    S = orc.compress(Sd, wl.sizes, wl.sizes, tol=0.0, drop=0.0)
    C = orc.to_dense(orc.gemm(S, S, tol=0.0, eps_sp=0.0))
    ref = Sd @ Sd
    return float(np.sqrt(np.sum((C - ref) ** 2)) / np.sqrt(np.sum(ref ** 2)))


def pin_default_alpha(orc):
    """alpha = 1 / max_I sum_J ||S_IJ||_F (the block-Gershgorin reading of Sec. 4.2's condition
    ||alpha S - I||_2 <= 1), on hand-set block norms whose row sums (3.75, 2.5, 4.0) and column
    sums (4.5, 2.0, 3.75) differ, so a column-sum, a max-norm or a smaller alpha all fail.
    Returns |alpha - 1/4|; the exact value is a power of two, so the check is exact."""
    def blk(v):
        return orc.Block("D", D=np.array([[v]]), norm=abs(v))
    blocks = {(0, 0): blk(1.0), (0, 1): blk(2.0), (0, 2): blk(0.75),
              (1, 0): blk(-0.5), (1, 2): blk(2.0),
              (2, 0): blk(3.0), (2, 2): blk(-1.0)}
    S = orc.OMatrix([1, 1, 1], [1, 1, 1], blocks)
    return abs(orc.default_alpha(S) - 0.25)


def pin_screening_area(orc, seed=19):
    """Per-area screening (tau = eps_sp * m * n, the paper's literal threshold of Sec. 4.1): with
    blocks of very different areas, the kept blocks are exactly those whose norm estimate is at
    least eps_sp * m * n (brute force over all pairs), and a kept block equals the exact sum."""
    rows, inner, cols = [2, 9, 4, 12], [5, 3, 8], [11, 2, 6, 3]
    ra = random_blocks(seed, rows, inner, p_zero=0.1, scale_decay=2.0)
    rb = random_blocks(seed + 1, inner, cols, p_zero=0.1, scale_decay=2.0)
    A = orc.from_factors(ra.row_sizes, ra.col_sizes, ra.kind, ra.f0, ra.f1)
    B = orc.from_factors(rb.row_sizes, rb.col_sizes, rb.kind, rb.f0, rb.f1)
    Ad, Bd = dense_from_factors(ra), dense_from_factors(rb)
    ro = np.concatenate([[0], np.cumsum(rows)])
    co = np.concatenate([[0], np.cumsum(cols)])
    ko = np.concatenate([[0], np.cumsum(inner)])
    est = np.zeros((len(rows), len(cols)))
    for i in range(len(rows)):
        for j in range(len(cols)):
            for k in range(len(inner)):
                na = float(np.sqrt(np.sum(Ad[ro[i]:ro[i + 1], ko[k]:ko[k + 1]] ** 2)))
                nb = float(np.sqrt(np.sum(Bd[ko[k]:ko[k + 1], co[j]:co[j + 1]] ** 2)))
                est[i, j] += na * nb
    area = np.outer(rows, cols).astype(float)
    # a threshold per unit area that separates the blocks: the median of est / area
    eps = float(np.median(est / area))
    C = orc.gemm(A, B, tol=0.0, eps_sp=eps, screen="area")
    worst = 0.0
    nkept = 0
    for i in range(len(rows)):
        for j in range(len(cols)):
            want = est[i, j] >= eps * area[i, j]
            exact = Ad[ro[i]:ro[i + 1]] @ Bd[:, co[j]:co[j + 1]]
            nrm = float(np.sqrt(np.sum(exact ** 2)))
            want = want and nrm >= eps * area[i, j]      # dropped after compute if below tau
            if ((i, j) in C.blocks) != want:
                return math.inf
            if want:
                nkept += 1
                d = C.blocks[(i, j)].dense() - exact
                worst = max(worst, float(np.sqrt(np.sum(d ** 2))) / nrm)
    if nkept == 0 or nkept == len(rows) * len(cols):
        return math.inf   # the case must screen some blocks and keep others
    return worst


def ns_scalar_residuals(lam, alpha, iters):
    """Internal residuals of Eqs. (8)-(11) for diagonal S = diag(lam): x_n = alpha lam z_n^2
    (X_n = alpha Y_n Z_n with Y_n = lam z_n for diagonal iterates), and the explicit residual of
    W = sqrt(alpha) z_{n+1}: sqrt(mean((alpha lam z_{n+1}^2 - 1)^2))."""
    lam = np.asarray(lam, dtype=np.float64)
    z = np.ones_like(lam)
    internal, explicit = [], []
    for _ in range(iters):
        x = alpha * lam * z * z
        internal.append(float(np.sqrt(np.mean((x - 1.0) ** 2))))
        z = z * (15.0 - 10.0 * x + 3.0 * x * x) / 8.0
        explicit.append(float(np.sqrt(np.mean((alpha * lam * z * z - 1.0) ** 2))))
    return internal, explicit


def pin_stop_statuses(orc):
    """The stopping rule (reading C9 of Sec. 4.2's iteration) on cases whose outcome is fixed by
    the scalar recurrence, not by rounding:
      converged: diagonal S, no truncation; the run stops after the first iteration whose
        internal residual is <= conv_tol (its explicit residual is then far below conv_tol);
      diverged: alpha = 2.5 / lambda_max, outside ||alpha S - I||_2 <= 1, so x p(x)^2 grows
        without bound from x = 2.5 (p(2.5) > 1); stops after the third iteration;
      stalled: a 1-D overlap-like matrix truncated at tol 1e-4 per product with an unreachable
        target (conv_tol 1e-15): the truncation keeps W's explicit residual near 1e-5, and the
        internal residual settles at its own floor and grows in two consecutive iterations.
    Returns a list of (case, ok, detail)."""
    out = []
    lam = [0.2, 0.5, 0.9, 1.3, 1.7, 0.35]
    sizes = [2, 3, 1]
    S = orc.compress(np.diag(lam), sizes, sizes, tol=0.0, drop=0.0)
    alpha = 0.5
    conv = 1e-10
    internal, explicit = ns_scalar_residuals(lam, alpha, 30)
    n_stop = next(i for i, r in enumerate(internal) if r <= conv)
    clear = internal[n_stop] < 0.1 * conv and (n_stop == 0 or internal[n_stop - 1] > 10 * conv) \
        and explicit[n_stop] < 0.1 * conv
    _W, info = orc.sqrt_inv(S, 0.0, 0.0, conv_tol=conv, alpha=alpha)
    out.append(("converged", clear and info.status == "converged" and info.iterations == n_stop + 1,
                (info.status, info.iterations, n_stop + 1)))
    _W, info = orc.sqrt_inv(S, 0.0, 0.0, conv_tol=conv, alpha=2.5 / max(lam))
    out.append(("diverged", info.status == "diverged" and info.iterations == 3,
                (info.status, info.iterations)))
    from workloads import kernel_matrix, points_1d
    Sd = kernel_matrix(points_1d(rng_for(22), 96, 1.0, 0.2), 0.5, 0.1)
    S2 = orc.compress(Sd, [16] * 6, [16] * 6, 1e-4, 1e-12)
    W, info = orc.sqrt_inv(S2, 1e-4, 1e-12, conv_tol=1e-15)
    Wd, Sc = orc.to_dense(W), orc.to_dense(S2)
    expl = float(np.sqrt(np.sum((Wd @ Sc @ Wd - np.eye(96)) ** 2)) / math.sqrt(96))
    r = info.internal
    grew = len(r) >= 3 and r[-1] > r[-2] > r[-3] and r[-1] < 0.5
    out.append(("stalled", info.status == "stalled" and expl > 1e-6 and grew,
                (info.status, info.iterations, expl)))
    return out
