"""Seeded synthetic inputs shared by the CLR library's tests, its benchmark and the oracle.

This module produces raw inputs only: point sets, cluster (block) sizes, dense
kernel matrices built from those points, and random dense/low-rank block factors.
It holds none of the method's arithmetic (no products, no factorisations, no
truncation, no screening), so the GPU path and the CPU oracle can both consume
exactly the same bytes without sharing any of the computation they are
compared on.

Workloads stand in for the paper's quantum-chemistry overlap matrices (Sec. 4.2:
190 water molecules, 141 basis functions each, natural 141-blocking, an
exponentially decaying kernel).  Those integrals are not available, so the
matrices here are Gaussian-kernel "overlap-like" matrices on jittered point
sets, clustered into contiguous blocks of 96..160 points.

Recipe (all draws from ``numpy.random.Generator(PCG64(seed))``):

* 1D: x_i = i*spacing + U(-jit, jit), i < N.
* 3D: n_s = smallest integer with n_s**3 >= N; point idx sits at lattice site
  (idx // n_s**2, (idx // n_s) % n_s, idx % n_s) * spacing + U(-jit, jit)**3.
  Clusters are contiguous runs of idx ("lattice order", k fastest).
* Jitter is drawn first, shape (N, d); cluster sizes afterwards.
* Kernel: S_ij = exp(-a * |x_i - x_j|**2) + d * delta_ij.
* Low-rank regime: the same lattice sites visited in Morton (Z-curve) order of
  their integer coordinates, so that contiguous clusters are compact boxes
  instead of lattice slabs; and a slowly decaying Coulomb-like kernel
  S_ij = 1 / sqrt(|x_i - x_j|**2 + delta**2) + d * delta_ij on those sites.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Workload",
    "rng_for",
    "points_1d",
    "points_3d",
    "lattice_side",
    "sizes_until",
    "sizes_pm",
    "sizes_weighted",
    "kernel_matrix",
    "kernel_block",
    "coulomb_block",
    "coulomb_matrix",
    "morton_order",
    "points_3d_morton",
    "line_n512",
    "lattice_3d",
    "batch_product",
    "dense_limit",
    "lattice_3d_wide",
    "adjoint_n4096",
    "scaled_workload",
    "lattice_3d_morton",
    "coulomb_3d_morton",
    "random_blocks",
    "RandomCLR",
]


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Workload:
    """A synthetic overlap-like matrix: points, kernel parameters and blocking."""

    name: str
    points: np.ndarray          # (N, d) float64
    sizes: List[int]            # cluster sizes, sum == N
    a: float                    # Gaussian exponent (Coulomb-like kernel: the softening length)
    diag: float                 # diagonal shift d
    tol: float                  # relative truncation tolerance
    eps_sp: float               # screening threshold
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.points.shape[0])

    def dense(self) -> np.ndarray:
        if self.extra.get("kernel") == "coulomb":
            return coulomb_matrix(self.points, self.a, self.diag)
        return kernel_matrix(self.points, self.a, self.diag)

    def offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)


def points_1d(rng: np.random.Generator, n: int, spacing: float, jit: float) -> np.ndarray:
    jitter = rng.uniform(-jit, jit, size=(n, 1))
    base = (np.arange(n, dtype=np.float64) * spacing)[:, None]
    return base + jitter


def lattice_side(n: int) -> int:
    """Smallest integer n_s with n_s**3 >= n (integer search, no cube root)."""
    s = 1
    while s * s * s < n:
        s += 1
    return s


def points_3d(rng: np.random.Generator, n: int, spacing: float, jit: float) -> np.ndarray:
    jitter = rng.uniform(-jit, jit, size=(n, 3))
    ns = lattice_side(n)
    idx = np.arange(n, dtype=np.int64)
    site = np.stack([idx // (ns * ns), (idx // ns) % ns, idx % ns], axis=1).astype(np.float64)
    return site * spacing + jitter


def morton_order(n: int) -> np.ndarray:
    """Lattice indices 0..n-1 (site (idx // ns**2, (idx // ns) % ns, idx % ns)) sorted by the
    Morton code of their integer coordinates: bit b of i, j, k goes to bit 3b + 2, 3b + 1, 3b."""
    ns = lattice_side(n)
    idx = np.arange(n, dtype=np.int64)
    ijk = [idx // (ns * ns), (idx // ns) % ns, idx % ns]
    code = np.zeros(n, dtype=np.int64)
    for b in range(int(ns).bit_length()):
        for shift, c in ((2, ijk[0]), (1, ijk[1]), (0, ijk[2])):
            code |= ((c >> b) & 1) << (3 * b + shift)
    return np.argsort(code, kind="stable")


def points_3d_morton(rng: np.random.Generator, n: int, spacing: float, jit: float) -> np.ndarray:
    """points_3d (same draws), visited in Morton order of their lattice sites."""
    return points_3d(rng, n, spacing, jit)[morton_order(n)]


def sizes_until(rng: np.random.Generator, n: int, lo: int, hi: int) -> List[int]:
    """Draw sizes ~ U{lo..hi} until they reach n; the last cluster takes the remainder."""
    out: List[int] = []
    total = 0
    while total < n:
        s = int(rng.integers(lo, hi + 1))
        if total + s >= n:
            s = n - total
        out.append(s)
        total += s
    return out


def sizes_pm(rng: np.random.Generator, center: int, half_count: int, spread: int) -> List[int]:
    """Multiset {center +- d_i} for d_i ~ U{-spread..spread}, shuffled (sums to 2*center*half_count)."""
    d = rng.integers(-spread, spread + 1, size=half_count)
    sizes = np.concatenate([center + d, center - d]).astype(np.int64)
    rng.shuffle(sizes)
    return [int(s) for s in sizes]


def sizes_weighted(rng: np.random.Generator, n: int, count: int) -> List[int]:
    """Uneven sizes: w ~ U(0.5, 1.5)**count, s = floor(n*w/sum w), remainder +1 to the first clusters."""
    w = rng.uniform(0.5, 1.5, size=count)
    s = np.floor(n * w / w.sum()).astype(np.int64)
    rem = int(n - s.sum())
    s[:rem] += 1
    return [int(v) for v in s]


def kernel_block(xi: np.ndarray, xj: np.ndarray, a: float) -> np.ndarray:
    """exp(-a |x_i - x_j|^2) for two point sets (no diagonal shift)."""
    d2 = np.zeros((xi.shape[0], xj.shape[0]), dtype=np.float64)
    for c in range(xi.shape[1]):
        diff = xi[:, c][:, None] - xj[:, c][None, :]
        d2 += diff * diff
    return np.exp(-a * d2)


def coulomb_block(xi: np.ndarray, xj: np.ndarray, delta: float) -> np.ndarray:
    """1 / sqrt(|x_i - x_j|^2 + delta^2) for two point sets (no diagonal shift)."""
    d2 = np.full((xi.shape[0], xj.shape[0]), delta * delta, dtype=np.float64)
    for c in range(xi.shape[1]):
        diff = xi[:, c][:, None] - xj[:, c][None, :]
        d2 += diff * diff
    return 1.0 / np.sqrt(d2)


def coulomb_matrix(points: np.ndarray, delta: float, diag: float, chunk: int = 4096) -> np.ndarray:
    """Dense S_ij = 1 / sqrt(|x_i - x_j|^2 + delta^2) + diag * delta_ij, built in row chunks."""
    n = points.shape[0]
    s = np.empty((n, n), dtype=np.float64)
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        s[r0:r1] = coulomb_block(points[r0:r1], points, delta)
    s[np.arange(n), np.arange(n)] += diag
    return s


def kernel_matrix(points: np.ndarray, a: float, diag: float, chunk: int = 4096) -> np.ndarray:
    """Dense S_ij = exp(-a |x_i - x_j|^2) + diag * delta_ij, built in row chunks."""
    n = points.shape[0]
    s = np.empty((n, n), dtype=np.float64)
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        s[r0:r1] = kernel_block(points[r0:r1], points, a)
    s[np.arange(n), np.arange(n)] += diag
    return s


# ---------------------------------------------------------------------------
# The named workloads.  Seeds: 1000 (line), 2000 (3-D lattice), 3000 + p
# (batch product p), 3999 (dense limit), 4000 (wide 3-D lattice), 5000 (adjoint).
# ---------------------------------------------------------------------------

def line_n512() -> Workload:
    """N = 512 points on a line, 8 clusters of the given sizes, a = 0.5, d = 0.1."""
    rng = rng_for(1000)
    pts = points_1d(rng, 512, 1.0, 0.2)
    sizes = [48, 80, 64, 72, 56, 64, 60, 68]
    return Workload("line-n512", pts, sizes, a=0.5, diag=0.1, tol=1e-8, eps_sp=1e-10,
                    extra={"conv_tol": 1e-10})


def lattice_3d(n: int = 8192, seed: int = 2000) -> Workload:
    """Jittered 3D lattice (spacing 1.5, jitter 0.3), a = 0.3, d = 0.1, clusters U{96..160}."""
    rng = rng_for(seed)
    pts = points_3d(rng, n, 1.5, 0.3)
    sizes = sizes_until(rng, n, 96, 160)
    return Workload(f"lattice3d-n{n}", pts, sizes, a=0.3, diag=0.1, tol=1e-6, eps_sp=1e-10)


def batch_product(p: int) -> Workload:
    """Product p of the batch: N ~ U{512..4096}, 16..48 clusters of uneven sizes, 3-D lattice physics, tol 1e-8."""
    rng = rng_for(3000 + p)
    n = int(rng.integers(512, 4097))
    c = int(rng.integers(16, 49))
    pts = points_3d(rng, n, 1.5, 0.3)
    sizes = sizes_weighted(rng, n, c)
    return Workload(f"batch-p{p}-n{n}", pts, sizes, a=0.3, diag=0.1, tol=1e-8, eps_sp=1e-10)


def dense_limit(n: int = 4096, nblocks: int = 32) -> Workload:
    """Full-rank dense limit: truncation and screening off, equal blocks."""
    rng = rng_for(3999)
    pts = points_3d(rng, n, 1.5, 0.3)
    sizes = [n // nblocks] * nblocks
    return Workload(f"dense-limit-n{n}", pts, sizes, a=0.3, diag=0.1, tol=0.0, eps_sp=0.0)


def lattice_3d_wide(n: int = 32768, nclusters: int = 256, seed: int = 4000) -> Workload:
    """3D lattice spacing 1.2, jitter 0.3, a = 0.2, d = 0.05, sizes {128 +- U{-32..32}}."""
    rng = rng_for(seed)
    pts = points_3d(rng, n, 1.2, 0.3)
    sizes = sizes_pm(rng, n // nclusters, nclusters // 2, 32)
    return Workload(f"wide3d-n{n}", pts, sizes, a=0.2, diag=0.05, tol=1e-8, eps_sp=1e-10,
                    extra={"conv_tol": 1e-8})


def adjoint_n4096(seed: int = 5000) -> Workload:
    """N = 4096, 32 clusters {128 +- d}, 3-D lattice physics, tol 1e-8; 20 fixed iterations."""
    rng = rng_for(seed)
    pts = points_3d(rng, 4096, 1.5, 0.3)
    sizes = sizes_pm(rng, 128, 16, 32)
    w = rng.standard_normal((4096, 4096))
    return Workload("adjoint3d-n4096", pts, sizes, a=0.3, diag=0.1, tol=1e-8, eps_sp=1e-10,
                    extra={"weights": w, "iters": 20, "checkpoint_every": 5})


def lattice_3d_morton(n: int = 8192, seed: int = 2000) -> Workload:
    """lattice_3d's points and physics in Morton order: compact clusters U{96..160}, far more
    low-rank blocks (the paper's rank-sparse regime)."""
    rng = rng_for(seed)
    pts = points_3d_morton(rng, n, 1.5, 0.3)
    sizes = sizes_until(rng, n, 96, 160)
    return Workload(f"morton3d-n{n}", pts, sizes, a=0.3, diag=0.1, tol=1e-6, eps_sp=1e-10)


def coulomb_3d_morton(n: int = 8192, seed: int = 6000) -> Workload:
    """Coulomb-like 1 / sqrt(r^2 + 1) + 0.1 delta on a Morton-ordered jittered lattice (spacing 1.0,
    jitter 0.3), clusters U{96..160}, tol 1e-6: no block is negligible, ranks decay slowly."""
    rng = rng_for(seed)
    pts = points_3d_morton(rng, n, 1.0, 0.3)
    sizes = sizes_until(rng, n, 96, 160)
    return Workload(f"coulomb3d-n{n}", pts, sizes, a=1.0, diag=0.1, tol=1e-6, eps_sp=1e-10,
                    extra={"kernel": "coulomb"})


def scaled_workload(kind: str, n: int, nclusters: Optional[int] = None, seed: int = 7000,
                    tol: Optional[float] = None) -> Workload:
    """Smaller copies of the 3D workloads (same physics) for parity tests the oracle finishes fast."""
    rng = rng_for(seed)
    if kind == "lattice":
        pts = points_3d(rng, n, 1.5, 0.3)
        sizes = sizes_until(rng, n, 96, 160) if nclusters is None else sizes_weighted(rng, n, nclusters)
        return Workload(f"lattice3d-small-n{n}", pts, sizes, 0.3, 0.1, 1e-6 if tol is None else tol, 1e-10)
    if kind == "wide":
        pts = points_3d(rng, n, 1.2, 0.3)
        nc = nclusters or max(2, n // 128)
        sizes = sizes_weighted(rng, n, nc)
        return Workload(f"wide3d-small-n{n}", pts, sizes, 0.2, 0.05, 1e-8 if tol is None else tol, 1e-10,
                        extra={"conv_tol": 1e-8})
    if kind == "morton":
        pts = points_3d_morton(rng, n, 1.5, 0.3)
        sizes = sizes_until(rng, n, 96, 160) if nclusters is None else sizes_weighted(rng, n, nclusters)
        return Workload(f"morton3d-small-n{n}", pts, sizes, 0.3, 0.1, 1e-6 if tol is None else tol, 1e-10)
    if kind == "coulomb":
        pts = points_3d_morton(rng, n, 1.0, 0.3)
        sizes = sizes_until(rng, n, 96, 160) if nclusters is None else sizes_weighted(rng, n, nclusters)
        return Workload(f"coulomb3d-small-n{n}", pts, sizes, 1.0, 0.1, 1e-6 if tol is None else tol, 1e-10,
                        extra={"kernel": "coulomb"})
    raise ValueError(kind)


# ---------------------------------------------------------------------------
# Random CLR factor sets (for product-kind and boundary tests)
# ---------------------------------------------------------------------------

@dataclass
class RandomCLR:
    """A block structure with per-block kind (0 zero, 1 dense, 2 low-rank) and raw factors.

    Dense blocks: ``f0[(I,J)]`` is m x n.  Low-rank blocks: ``f0`` is U (m x r) and
    ``f1`` is V (n x r); the block value is U @ V.T.  All arrays are float64.
    """

    row_sizes: List[int]
    col_sizes: List[int]
    kind: np.ndarray            # (nrb, ncb) int8
    rank: np.ndarray            # (nrb, ncb) int32
    f0: dict
    f1: dict


def random_blocks(seed: int, row_sizes: Sequence[int], col_sizes: Sequence[int],
                  p_zero: float = 0.2, p_dense: float = 0.3, max_rank: Optional[int] = None,
                  scale_decay: float = 0.0) -> RandomCLR:
    """Random CLR factors: kinds drawn per block, ranks ~ U{1..min(m,n)//2}, N(0,1) entries.

    ``scale_decay`` > 0 multiplies block (I,J) by exp(-scale_decay*|I-J|) so that
    norms spread over several decades, which exercises screening.
    """
    rng = rng_for(seed)
    nrb, ncb = len(row_sizes), len(col_sizes)
    kind = np.zeros((nrb, ncb), dtype=np.int8)
    rank = np.zeros((nrb, ncb), dtype=np.int32)
    f0, f1 = {}, {}
    for i in range(nrb):
        for j in range(ncb):
            m, n = int(row_sizes[i]), int(col_sizes[j])
            u = rng.uniform()
            scale = float(np.exp(-scale_decay * abs(i - j)))
            if u < p_zero:
                continue
            if u < p_zero + p_dense or min(m, n) < 2:
                kind[i, j] = 1
                rank[i, j] = min(m, n)
                f0[(i, j)] = scale * rng.standard_normal((m, n))
            else:
                hi = max(1, min(m, n) // 2)
                if max_rank is not None:
                    hi = max(1, min(hi, max_rank))
                r = int(rng.integers(1, hi + 1))
                kind[i, j] = 2
                rank[i, j] = r
                f0[(i, j)] = scale * rng.standard_normal((m, r))
                f1[(i, j)] = rng.standard_normal((n, r))
    return RandomCLR(list(map(int, row_sizes)), list(map(int, col_sizes)), kind, rank, f0, f1)
