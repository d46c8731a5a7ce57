"""Plain FP64 CPU oracle for the clustered low-rank (CLR) block product and S^-1/2.

TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may import,
call or execute this module; it exists so that tests, the smoke check and the
benchmark's CPU-baseline leg can check the GPU path against an independent,
slow, obviously-correct implementation written from the paper
(Calvin, Lewis & Valeev, "Scalable Task-Based Algorithm for Multiplication of
Block-Rank-Sparse Matrices", IA^3 2015).  It shares no code with the GPU path.

Every function below follows one passage of the paper:

* CLR representation, Sec. 4.1: each block is zero, dense, or X W^T with
  X m x r and W n x r; a block whose rank exceeds half of full rank is kept
  in full (dense) form.
* Low-rank x low-rank product, Sec. 4.1 Eq. (4): Z = (W^A)^T X^B, contracted
  with X^A or W^B so that the output rank is the smaller one.
* Low-rank addition, Sec. 4.1 Eq. (5): concatenation of the factors.
* Recompression, Sec. 4.1 Eqs. (6)-(7): QR of X and W, core M = R^X (R^W)^T,
  low-rank decomposition of M, X' = Q^X X^M, W' = Q^W W^M.
* Screening, Sec. 4.1 (last paragraph): a result block is computed only when
  its Frobenius-norm estimate (triangle inequality + submultiplicativity) is
  not below the threshold.
* Iterative square-root inverse, Sec. 4.2 Eqs. (8)-(11): coupled third-order
  Newton-Schulz with Z_0 = I, Y_0 = M, result sqrt(alpha) Z.

Readings of points the paper leaves open (each applied identically by the GPU
path and listed in the design notes):

* Screening direction: the printed inequality is inverted relative to its
  stated purpose; a block is computed iff est >= tau (ties computed).
* tau is absolute (tau = eps_sp) by default; ``screen="area"`` uses
  eps_sp * m * n, the paper's per-area form.
* Truncation: the low-rank decomposition is a truncated SVD (the paper builds
  its factors by rank-revealing QR).  The kept rank is the smallest r with
  sqrt(sum_{i>r} sigma_i^2) <= tol * ||C_IJ||_F (relative per block; the tail
  is accumulated from the smallest singular value upward).  tol == 0 means
  "no truncation": blocks are kept exactly as accumulated.
* Dense storage iff 2 r > min(m, n); diagonal blocks of square-blocked
  matrices are always dense.  A block's accumulation is done densely iff it is
  such a diagonal block, or any contribution is dense, or the concatenated
  rank R satisfies 2 R >= min(m, n).
* After accumulation a block whose exact norm is below tau is dropped; a
  block whose accumulated value is exactly zero is a zero block.
* Factor convention: X (here U) carries the orthonormal basis, W (here V)
  carries the singular values, as X = Q_r in the paper.
* Construction by rank-revealing QR (``compress_rrqr``, the paper's own
  factorisation of an input block): column pivoting of the block M itself,
  M P = Q R, with the same relative per-block truncation: the smallest r with
  ||M - Q_r R_r P^T||_F = ||R[r:, :]||_F <= tol * ||M||_F.
* Ties in the low-rank x low-rank absorb rule go to the W side (V_B Z^T).
* alpha defaults to 1 / max_I sum_J ||S_IJ||_F (a block-Gershgorin bound on
  the largest eigenvalue, so ||alpha S - I||_2 <= 1 for symmetric positive S).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Block",
    "OMatrix",
    "from_factors",
    "compress",
    "compress_rrqr",
    "rrqr_truncate",
    "to_dense",
    "truncation_rank",
    "combine",
    "block_product",
    "gemm",
    "gemm_block",
    "ns_T",
    "identity",
    "scale",
    "default_alpha",
    "offdiag_identity_residual",
    "explicit_residual",
    "sqrt_inv",
    "gemm_vjp",
    "sqrt_inv_vjp",
    "structure_mask",
    "GemmStats",
]


# ---------------------------------------------------------------------------
# Representation (Sec. 4.1)
# ---------------------------------------------------------------------------

@dataclass
class Block:
    """One stored block: dense ``D`` (m x n) or low-rank ``U @ V.T`` (U m x r, V n x r)."""

    kind: str                       # "D" or "L"
    D: Optional[np.ndarray] = None
    U: Optional[np.ndarray] = None
    V: Optional[np.ndarray] = None
    norm: float = 0.0

    @property
    def rank(self) -> int:
        if self.kind == "D":
            return int(min(self.D.shape))
        return int(self.U.shape[1])

    def dense(self) -> np.ndarray:
        if self.kind == "D":
            return self.D
        return self.U @ self.V.T


@dataclass
class OMatrix:
    row_sizes: List[int]
    col_sizes: List[int]
    blocks: Dict[Tuple[int, int], Block]

    @property
    def nrb(self) -> int:
        return len(self.row_sizes)

    @property
    def ncb(self) -> int:
        return len(self.col_sizes)

    @property
    def shape(self) -> Tuple[int, int]:
        return int(sum(self.row_sizes)), int(sum(self.col_sizes))

    def square_blocked(self) -> bool:
        return list(self.row_sizes) == list(self.col_sizes)

    def offsets(self):
        ro = np.concatenate([[0], np.cumsum(self.row_sizes)]).astype(int)
        co = np.concatenate([[0], np.cumsum(self.col_sizes)]).astype(int)
        return ro, co

    def kinds(self) -> np.ndarray:
        k = np.zeros((self.nrb, self.ncb), dtype=np.int8)
        for (i, j), b in self.blocks.items():
            k[i, j] = 1 if b.kind == "D" else 2
        return k

    def ranks(self) -> np.ndarray:
        r = np.zeros((self.nrb, self.ncb), dtype=np.int32)
        for (i, j), b in self.blocks.items():
            r[i, j] = b.rank
        return r

    def norms(self) -> np.ndarray:
        r = np.zeros((self.nrb, self.ncb), dtype=np.float64)
        for (i, j), b in self.blocks.items():
            r[i, j] = b.norm
        return r


def frob(x: np.ndarray) -> float:
    return float(np.sqrt(np.sum(x * x)))


def to_dense(M: OMatrix) -> np.ndarray:
    ro, co = M.offsets()
    out = np.zeros(M.shape, dtype=np.float64)
    for (i, j), b in M.blocks.items():
        out[ro[i]:ro[i + 1], co[j]:co[j + 1]] = b.dense()
    return out


def from_factors(row_sizes: Sequence[int], col_sizes: Sequence[int], kind: np.ndarray,
                 f0: dict, f1: dict) -> OMatrix:
    """Wrap given factors as a CLR matrix (no compression); norms are exact block norms."""
    blocks = {}
    for i in range(len(row_sizes)):
        for j in range(len(col_sizes)):
            k = int(kind[i, j])
            if k == 0:
                continue
            if k == 1:
                D = np.array(f0[(i, j)], dtype=np.float64)
                blocks[(i, j)] = Block("D", D=D, norm=frob(D))
            else:
                U = np.array(f0[(i, j)], dtype=np.float64)
                V = np.array(f1[(i, j)], dtype=np.float64)
                blocks[(i, j)] = Block("L", U=U, V=V, norm=frob(U @ V.T))
    return OMatrix(list(row_sizes), list(col_sizes), blocks)


# ---------------------------------------------------------------------------
# Truncation and recompression (Sec. 4.1, Eqs. (5)-(7))
# ---------------------------------------------------------------------------

def truncation_rank(sigma: np.ndarray, tol: float, normc: float) -> int:
    """Smallest r with sqrt(sum_{i>=r} sigma_i^2) <= tol * normc (sigma descending)."""
    n = len(sigma)
    tails = np.zeros(n + 1, dtype=np.float64)
    acc = 0.0
    for i in range(n - 1, -1, -1):
        acc += float(sigma[i]) * float(sigma[i])
        tails[i] = acc
    bound = tol * normc
    for r in range(n + 1):
        if math.sqrt(tails[r]) <= bound:
            return r
    return n


def combine(m: int, n: int, contribs: List[tuple], tol: float, tau: float,
            force_dense: bool) -> Optional[Block]:
    """Accumulate the contributions of one result block and recompress it.

    ``contribs`` holds ("D", D) and ("L", U, V) terms in accumulation order.
    Low-rank terms are concatenated (Eq. (5)); the concatenation is recompressed
    through QR of both factors, the core M = R_U R_V^T and its truncated SVD
    (Eqs. (6)-(7)).  A block that must be accumulated densely is truncated by
    the SVD of the dense sum.  Returns None for a zero (dropped) block.
    """
    rcat = sum(c[1].shape[1] for c in contribs if c[0] == "L")
    any_dense = any(c[0] == "D" for c in contribs)
    mn = min(m, n)
    if force_dense or any_dense or 2 * rcat >= mn:
        D = np.zeros((m, n), dtype=np.float64)
        for c in contribs:
            if c[0] == "D":
                D += c[1]
            else:
                D += c[1] @ c[2].T
        normc = frob(D)
        if normc < tau or normc == 0.0:
            return None
        if force_dense or tol == 0.0:
            return Block("D", D=D, norm=normc)
        U, s, Vt = np.linalg.svd(D, full_matrices=False)
        r = truncation_rank(s, tol, normc)
        if r == 0:
            return None
        if 2 * r > mn:
            return Block("D", D=D, norm=normc)
        return Block("L", U=U[:, :r].copy(), V=(Vt[:r].T * s[:r]).copy(),
                     norm=math.sqrt(float(np.sum(s[:r] ** 2))))
    Ucat = np.concatenate([c[1] for c in contribs], axis=1)
    Vcat = np.concatenate([c[2] for c in contribs], axis=1)
    if tol == 0.0:
        normc = frob(Ucat @ Vcat.T)
        if normc < tau or normc == 0.0:
            return None
        return Block("L", U=Ucat, V=Vcat, norm=normc)
    QU, RU = np.linalg.qr(Ucat)
    QV, RV = np.linalg.qr(Vcat)
    M = RU @ RV.T
    normc = frob(M)
    if normc < tau or normc == 0.0:
        return None
    Um, s, Vmt = np.linalg.svd(M)
    r = truncation_rank(s, tol, normc)
    if r == 0:
        return None
    return Block("L", U=QU @ Um[:, :r], V=QV @ (Vmt[:r].T * s[:r]),
                 norm=math.sqrt(float(np.sum(s[:r] ** 2))))


def compress(S: np.ndarray, row_sizes: Sequence[int], col_sizes: Sequence[int], tol: float,
             drop: float) -> OMatrix:
    """CLR form of a dense matrix: drop blocks with norm < drop, truncate the rest (Sec. 4.1)."""
    ro = np.concatenate([[0], np.cumsum(row_sizes)]).astype(int)
    co = np.concatenate([[0], np.cumsum(col_sizes)]).astype(int)
    square = list(row_sizes) == list(col_sizes)
    blocks = {}
    for i in range(len(row_sizes)):
        for j in range(len(col_sizes)):
            D = np.array(S[ro[i]:ro[i + 1], co[j]:co[j + 1]], dtype=np.float64)
            b = combine(D.shape[0], D.shape[1], [("D", D)], tol, drop, square and i == j)
            if b is not None:
                blocks[(i, j)] = b
    return OMatrix(list(row_sizes), list(col_sizes), blocks)


def rrqr_truncate(M: np.ndarray, tol: float) -> Tuple[int, np.ndarray, np.ndarray, np.ndarray]:
    """Rank-revealing QR of one block (Sec. 4.1): M P = Q R by Householder QR with column
    pivoting (LAPACK's greedy rule: the remaining column of largest norm goes next), then the
    smallest r whose dropped part ||R[r:, :]||_F is <= tol * ||M||_F.

    Returns (r, X, W, tails) with M ~ X W^T, X = Q[:, :r] (orthonormal), W^T = R[:r] P^T, and
    tails[k] = ||R[k:, :]||_F for k = 0 .. min(m, n).
    """
    import scipy.linalg as sl
    Q, R, piv = sl.qr(M, mode="economic", pivoting=True)
    k = R.shape[0]
    tails = np.zeros(k + 1, dtype=np.float64)
    acc = 0.0
    for i in range(k - 1, -1, -1):
        acc += float(np.sum(R[i, i:] ** 2))
        tails[i] = math.sqrt(acc)
    bound = tol * frob(M)
    r = next(i for i in range(k + 1) if tails[i] <= bound)
    Wt = np.zeros((r, M.shape[1]), dtype=np.float64)
    Wt[:, piv] = R[:r, :]
    return r, Q[:, :r].copy(), Wt.T.copy(), tails


def compress_rrqr(S: np.ndarray, row_sizes: Sequence[int], col_sizes: Sequence[int], tol: float,
                  drop: float) -> OMatrix:
    """CLR form of a dense matrix built with the paper's rank-revealing QR (Sec. 4.1): blocks
    with norm < drop are dropped, diagonal blocks of a square blocking stay dense, the others
    are truncated by ``rrqr_truncate`` and stored dense iff 2 r > min(m, n)."""
    ro = np.concatenate([[0], np.cumsum(row_sizes)]).astype(int)
    co = np.concatenate([[0], np.cumsum(col_sizes)]).astype(int)
    square = list(row_sizes) == list(col_sizes)
    blocks = {}
    for i in range(len(row_sizes)):
        for j in range(len(col_sizes)):
            D = np.array(S[ro[i]:ro[i + 1], co[j]:co[j + 1]], dtype=np.float64)
            normc = frob(D)
            if normc < drop or normc == 0.0:
                continue
            if (square and i == j) or tol == 0.0:
                blocks[(i, j)] = Block("D", D=D, norm=normc)
                continue
            r, X, W, _tails = rrqr_truncate(D, tol)
            if r == 0:
                continue
            if 2 * r > min(D.shape):
                blocks[(i, j)] = Block("D", D=D, norm=normc)
            else:
                blocks[(i, j)] = Block("L", U=X, V=W, norm=frob(X @ W.T))
    return OMatrix(list(row_sizes), list(col_sizes), blocks)


# ---------------------------------------------------------------------------
# Block products (Sec. 4.1, Eq. (4)) and the CLR GEMM
# ---------------------------------------------------------------------------

def block_product(a: Block, b: Block, alpha: float = 1.0) -> tuple:
    """alpha * A_IK @ B_KJ as a dense or low-rank term."""
    if a.kind == "D" and b.kind == "D":
        return ("D", alpha * (a.D @ b.D))
    if a.kind == "L" and b.kind == "D":
        return ("L", alpha * a.U, b.D.T @ a.V)
    if a.kind == "D" and b.kind == "L":
        return ("L", alpha * (a.D @ b.U), b.V)
    Z = a.V.T @ b.U                              # r_A x r_B core
    if b.rank < a.rank:
        return ("L", alpha * (a.U @ Z), b.V)     # output rank r_B
    return ("L", alpha * a.U, b.V @ Z.T)         # output rank r_A (ties here)


@dataclass
class GemmStats:
    computed: int = 0
    screened: int = 0
    dropped: int = 0
    triples: int = 0
    flops_dd: float = 0.0
    flops_ld: float = 0.0
    flops_dl: float = 0.0
    flops_ll: float = 0.0
    flops_densify: float = 0.0


def block_tau(eps_sp: float, m: int, n: int, screen: str) -> float:
    return eps_sp * m * n if screen == "area" else eps_sp


def gemm_block(A: OMatrix, B: OMatrix, i: int, j: int, tol: float, eps_sp: float,
               screen: str = "abs", alpha: float = 1.0,
               stats: Optional[GemmStats] = None) -> Optional[Block]:
    """Result block (i, j) of alpha * A @ B: screening, products, accumulation, recompression."""
    m, n = A.row_sizes[i], B.col_sizes[j]
    square = list(A.row_sizes) == list(B.col_sizes)
    klist = [k for k in range(A.ncb) if (i, k) in A.blocks and (k, j) in B.blocks]
    if not klist:
        return None
    est = 0.0
    for k in klist:
        est += A.blocks[(i, k)].norm * B.blocks[(k, j)].norm
    est *= abs(alpha)
    tau = block_tau(eps_sp, m, n, screen)
    if est < tau:
        if stats is not None:
            stats.screened += 1
        return None
    contribs = []
    for k in klist:
        a, b = A.blocks[(i, k)], B.blocks[(k, j)]
        contribs.append(block_product(a, b, alpha))
        if stats is not None:
            kk = A.col_sizes[k]
            stats.triples += 1
            if a.kind == "D" and b.kind == "D":
                stats.flops_dd += 2.0 * m * kk * n
            elif a.kind == "L" and b.kind == "D":
                stats.flops_ld += 2.0 * a.rank * kk * n
            elif a.kind == "D" and b.kind == "L":
                stats.flops_dl += 2.0 * m * kk * b.rank
            else:
                side = m if b.rank < a.rank else n
                stats.flops_ll += 2.0 * kk * a.rank * b.rank + 2.0 * side * a.rank * b.rank
    blk = combine(m, n, contribs, tol, tau, square and i == j)
    if stats is not None:
        rcat = sum(c[1].shape[1] for c in contribs if c[0] == "L")
        if (square and i == j) or any(c[0] == "D" for c in contribs) or 2 * rcat >= min(m, n):
            stats.flops_densify += 2.0 * m * n * rcat
        stats.computed += 1
        if blk is None:
            stats.dropped += 1
    return blk


def gemm(A: OMatrix, B: OMatrix, tol: float, eps_sp: float, screen: str = "abs",
         alpha: float = 1.0, stats: Optional[GemmStats] = None) -> OMatrix:
    """C = alpha * A @ B in CLR arithmetic: screening, block products, accumulation, recompression."""
    if list(A.col_sizes) != list(B.row_sizes):
        raise ValueError("inner blockings differ")
    blocks = {}
    for i in range(A.nrb):
        for j in range(B.ncb):
            blk = gemm_block(A, B, i, j, tol, eps_sp, screen, alpha, stats)
            if blk is not None:
                blocks[(i, j)] = blk
    return OMatrix(list(A.row_sizes), list(B.col_sizes), blocks)


# ---------------------------------------------------------------------------
# Newton-Schulz square-root inverse (Sec. 4.2, Eqs. (8)-(11))
# ---------------------------------------------------------------------------

def identity(sizes: Sequence[int]) -> OMatrix:
    blocks = {}
    for i, m in enumerate(sizes):
        blocks[(i, i)] = Block("D", D=np.eye(m), norm=math.sqrt(m))
    return OMatrix(list(sizes), list(sizes), blocks)


def scale(M: OMatrix, s: float) -> OMatrix:
    blocks = {}
    for key, b in M.blocks.items():
        if b.kind == "D":
            blocks[key] = Block("D", D=s * b.D, norm=abs(s) * b.norm)
        else:
            blocks[key] = Block("L", U=s * b.U, V=b.V.copy(), norm=abs(s) * b.norm)
    return OMatrix(list(M.row_sizes), list(M.col_sizes), blocks)


def ns_T(X: OMatrix, Q: OMatrix, tol: float, eps_sp: float, screen: str = "abs") -> OMatrix:
    """T = (-10 X + 3 X^2 + 15 I) / 8 blockwise (Eq. (9)), with Q = X^2 given."""
    blocks = {}
    for i in range(X.nrb):
        m = X.row_sizes[i]
        for j in range(X.ncb):
            n = X.col_sizes[j]
            contribs = []
            est = 0.0
            if (i, j) in X.blocks:
                b = X.blocks[(i, j)]
                est += (10.0 / 8.0) * b.norm
                contribs.append(("D", (-10.0 / 8.0) * b.D) if b.kind == "D"
                                else ("L", (-10.0 / 8.0) * b.U, b.V))
            if (i, j) in Q.blocks:
                b = Q.blocks[(i, j)]
                est += (3.0 / 8.0) * b.norm
                contribs.append(("D", (3.0 / 8.0) * b.D) if b.kind == "D"
                                else ("L", (3.0 / 8.0) * b.U, b.V))
            if i == j:
                est += (15.0 / 8.0) * math.sqrt(m)
                contribs.append(("D", (15.0 / 8.0) * np.eye(m)))
            if not contribs:
                continue
            tau = block_tau(eps_sp, m, n, screen)
            if est < tau:
                continue
            blk = combine(m, n, contribs, tol, tau, i == j)
            if blk is not None:
                blocks[(i, j)] = blk
    return OMatrix(list(X.row_sizes), list(X.col_sizes), blocks)


def default_alpha(S: OMatrix) -> float:
    """1 / max_I sum_J ||S_IJ||_F: block-Gershgorin bound, keeps ||alpha S - I||_2 <= 1."""
    rows = np.zeros(S.nrb)
    for (i, _j), b in S.blocks.items():
        rows[i] += b.norm
    return 1.0 / float(np.max(rows))


def offdiag_identity_residual(X: OMatrix) -> float:
    """||X - I||_F / sqrt(N)."""
    N = X.shape[0]
    return frob(to_dense(X) - np.eye(N)) / math.sqrt(N)


def explicit_residual(W: OMatrix, S: OMatrix) -> float:
    """||W S W - I||_F / sqrt(N) from the dense forms, exact (untruncated) FP64 products."""
    Wd, Sd = to_dense(W), to_dense(S)
    N = Wd.shape[0]
    return frob(Wd @ Sd @ Wd - np.eye(N)) / math.sqrt(N)


@dataclass
class SqrtInvInfo:
    iterations: int
    alpha: float
    internal: List[float]
    explicit: List[Tuple[int, float]]
    status: str


def sqrt_inv(S: OMatrix, tol: float, eps_sp: float, conv_tol: float = 1e-10,
             max_iter: int = 50, fixed_iters: int = 0, alpha: Optional[float] = None,
             screen: str = "abs", keep_iterates: bool = False):
    """W = S^-1/2 by the coupled third-order Newton-Schulz iteration, Eqs. (8)-(11).

    Per iteration: X_n = alpha Y_n Z_n; T_n = (-10 X_n + 3 X_n^2 + 15 I)/8;
    Z_{n+1} = Z_n T_n; Y_{n+1} = T_n Y_n; result sqrt(alpha) Z.
    Stopping (fixed_iters == 0): once ||X_n - I||_F/sqrt(N) <= conv_tol the
    explicit residual ||W S W - I||_F/sqrt(N) of W = sqrt(alpha) Z_{n+1} is
    evaluated; stop when it is <= conv_tol ("converged"), or when it failed
    to halve since the previous evaluation ("stalled"); when ||X_n - I||
    grew in two consecutive iterations while above conv_tol, stop with
    "diverged" if it exceeds 0.5 and "stalled" otherwise; stop at max_iter.
    """
    if alpha is None:
        alpha = default_alpha(S)
    Z = identity(S.row_sizes)
    Y = S
    internal: List[float] = []
    explicit: List[Tuple[int, float]] = []
    iterates = []
    status = "max_iter"
    n_iter = fixed_iters if fixed_iters > 0 else max_iter
    it = 0
    for it in range(n_iter):
        X = gemm(Y, Z, tol, eps_sp, screen, alpha=alpha)
        Q = gemm(X, X, tol, eps_sp, screen)
        T = ns_T(X, Q, tol, eps_sp, screen)
        if keep_iterates:
            iterates.append((Y, Z, X, T))
        Zn = gemm(Z, T, tol, eps_sp, screen)
        Yn = gemm(T, Y, tol, eps_sp, screen)
        r = offdiag_identity_residual(X)
        internal.append(r)
        Z, Y = Zn, Yn
        if fixed_iters > 0:
            continue
        if r <= conv_tol:
            e = explicit_residual(scale(Z, math.sqrt(alpha)), S)
            explicit.append((it, e))
            if e <= conv_tol:
                status = "converged"
                break
            if len(explicit) >= 2 and e > 0.5 * explicit[-2][1]:
                status = "stalled"
                break
        elif len(internal) >= 3 and internal[-1] > internal[-2] > internal[-3]:
            # In exact arithmetic the residual falls monotonically once
            # ||alpha S - I||_2 < 1 (Sec. 4.2); growth while it is small is the
            # truncation / precision floor, growth beyond 0.5 is divergence.
            status = "diverged" if internal[-1] > 0.5 else "stalled"
            break
    if fixed_iters > 0:
        status = "fixed"
    W = scale(Z, math.sqrt(alpha))
    info = SqrtInvInfo(iterations=it + 1, alpha=alpha, internal=internal, explicit=explicit,
                       status=status)
    if keep_iterates:
        return W, info, iterates
    return W, info


# ---------------------------------------------------------------------------
# Adjoints (straight-through truncation; gradients on the stored structure)
# ---------------------------------------------------------------------------

def structure_mask(M: OMatrix) -> np.ndarray:
    ro, co = M.offsets()
    mask = np.zeros(M.shape, dtype=np.float64)
    for (i, j) in M.blocks:
        mask[ro[i]:ro[i + 1], co[j]:co[j + 1]] = 1.0
    return mask


def gemm_vjp(A: OMatrix, B: OMatrix, dC: np.ndarray, alpha: float = 1.0):
    """dA = alpha dC B^T and dB = alpha A^T dC, each restricted to the stored blocks."""
    Ad, Bd = to_dense(A), to_dense(B)
    dA = alpha * (dC @ Bd.T) * structure_mask(A)
    dB = alpha * (Ad.T @ dC) * structure_mask(B)
    return dA, dB


def sqrt_inv_vjp(S: OMatrix, Wbar: np.ndarray, iters: int, tol: float, eps_sp: float,
                 alpha: Optional[float] = None, screen: str = "abs"):
    """dL/dS for L = sum(Wbar * S^-1/2) through ``iters`` unrolled iterations.

    Reverse of Eqs. (8)-(11) with alpha held constant and the truncation
    treated as the identity:
      Zbar_K = sqrt(alpha) Wbar, Ybar_K = 0; for n = K-1..0:
      Tbar = Z_n^T Zbar_{n+1} + Ybar_{n+1} Y_n^T
      Zbar_n = Zbar_{n+1} T_n^T,  Ybar_n = T_n^T Ybar_{n+1}
      Xbar = -(10/8) Tbar + (3/8)(Tbar X_n^T + X_n^T Tbar)
      Ybar_n += alpha Xbar Z_n^T,  Zbar_n += alpha Y_n^T Xbar
    and dS = Ybar_0 on S's stored blocks.
    """
    if alpha is None:
        alpha = default_alpha(S)
    W, info, its = sqrt_inv(S, tol, eps_sp, fixed_iters=iters, alpha=alpha, screen=screen,
                            keep_iterates=True)
    Zb = math.sqrt(alpha) * Wbar
    Yb = np.zeros_like(Wbar)
    for (Y, Z, X, T) in reversed(its):
        Yd, Zd, Xd, Td = to_dense(Y), to_dense(Z), to_dense(X), to_dense(T)
        Tb = Zd.T @ Zb + Yb @ Yd.T
        Zb_new = Zb @ Td.T
        Yb_new = Td.T @ Yb
        Xb = -(10.0 / 8.0) * Tb + (3.0 / 8.0) * (Tb @ Xd.T + Xd.T @ Tb)
        Yb_new = Yb_new + alpha * (Xb @ Zd.T)
        Zb_new = Zb_new + alpha * (Yd.T @ Xb)
        Zb, Yb = Zb_new, Yb_new
    return Yb * structure_mask(S), W, info
