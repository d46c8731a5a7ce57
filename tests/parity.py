"""Comparison of a GPU CLR result with the oracle's, block by block.

Discrete decisions (zero / dense / low rank, kept rank) must agree exactly,
except where the oracle's own truncation is ambiguous: the dropped tail at the
oracle's or the GPU's rank lies within relative 1e-6 of tol * ||C_IJ||_F, so
that either rank is correct up to rounding.  Values are compared three ways:

* per block: ||G_IJ - O_IJ||_F / ||O_IJ||_F for every block of equal kind and
  rank (the largest is reported), so that a wrong far block of small norm is
  not hidden by the O(1) diagonal blocks.  For a product, a block whose value
  is far below the norms of the terms it sums (est_IJ = |alpha| sum_K
  ||A_IK||_F ||B_KJ||_F, the screening estimate of Sec. 4.1) carries the
  rounding of those terms: two correct summation orders differ by a few ulp
  of est_IJ, which is a large multiple of ||C_IJ||_F when the terms cancel or
  the product of decaying blocks is small.  Such a block is judged against
  max(||O_IJ||_F, 1e-2 est_IJ), so an error of 1e-12 relative is at most
  about 90 ulp of est_IJ;
* the norm table (Sec. 4.1: the norms that screen the next product): the
  largest relative difference of the stored ||C_IJ||_F;
* the whole matrix: relative Frobenius error.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

import oracle as orc


@dataclass
class ParityReport:
    rel_err: float
    kind_mismatch: List[tuple] = field(default_factory=list)
    rank_mismatch: List[tuple] = field(default_factory=list)
    ambiguous: List[tuple] = field(default_factory=list)
    max_norm_rel: float = 0.0
    max_block_rel: float = 0.0
    worst_block: tuple = ()
    blocks_compared: int = 0


def tails_of(block: np.ndarray) -> np.ndarray:
    s = np.linalg.svd(block, compute_uv=False)
    t = np.zeros(len(s) + 1)
    acc = 0.0
    for i in range(len(s) - 1, -1, -1):
        acc += s[i] ** 2
        t[i] = acc
    return np.sqrt(t)


def ambiguous_cut(exact_block: np.ndarray, tol: float, ranks, rel: float = 1e-6) -> bool:
    """True when the dropped tail at one of the given ranks (or one below) lies within relative
    ``rel`` of tol * ||block||_F: either rank is then a correct cut up to the arithmetic's error."""
    t = tails_of(exact_block)
    bound = tol * math.sqrt(float(np.sum(exact_block ** 2)))
    for r in ranks:
        for rr in (r - 1, r):
            if 0 <= rr < len(t) and abs(t[rr] - bound) <= rel * bound:
                return True
    return False


def operand_scale(A: orc.OMatrix, B: orc.OMatrix, alpha: float = 1.0) -> np.ndarray:
    """est_IJ = |alpha| sum_K ||A_IK||_F ||B_KJ||_F from the oracle operands' block norms."""
    na, nb = A.norms(), B.norms()
    return abs(alpha) * (na @ nb)


def compare(gpu, omat: orc.OMatrix, tol: float, exact: Optional[orc.OMatrix] = None,
            dense_gpu: Optional[np.ndarray] = None, ambiguous_rel: float = 1e-6,
            operands=None, floor: Optional[np.ndarray] = None) -> ParityReport:
    """Block-by-block comparison.  ``ambiguous_rel`` is the relative distance of a truncation
    tail from the cut within which a kind or rank difference is accepted (1e-6 for the FP64
    form; reduced-precision forms perturb singular values by their own rounding, which needs a
    wider margin).  ``operands`` = (A, B[, alpha]) of a product: each block's error and norm
    are then measured against max(||O_IJ||_F, 1e-2 est_IJ); ``floor`` gives that lower limit
    of the reference norm per block directly (for a blockwise sum of several terms)."""
    if operands is not None:
        alpha = operands[2] if len(operands) > 2 else 1.0
        floor = 1e-2 * operand_scale(operands[0], operands[1], alpha)
    kind_g, rank_g, norm_g = gpu.meta()
    Dg = dense_gpu if dense_gpu is not None else gpu.to_dense().cpu().numpy()
    Do = orc.to_dense(omat)
    kind_o, rank_o, norm_o = omat.kinds(), omat.ranks(), omat.norms()
    ro, co = omat.offsets()
    rep = ParityReport(rel_err=0.0)
    diff = Dg - Do
    for i in range(omat.nrb):
        for j in range(omat.ncb):
            kg, ko = int(kind_g[i, j]), int(kind_o[i, j])
            same_kind = kg == ko
            same_rank = (kg != 2) or (int(rank_g[i, j]) == int(rank_o[i, j]))
            if same_kind and same_rank:
                blk = diff[ro[i]:ro[i + 1], co[j]:co[j + 1]]
                if ko == 0:
                    # a zero block is exactly zero on both sides
                    brel = 0.0 if not np.any(blk) else math.inf
                    nrel = 0.0 if norm_g[i, j] == 0.0 else math.inf
                else:
                    ob = Do[ro[i]:ro[i + 1], co[j]:co[j + 1]]
                    onorm = math.sqrt(float(np.sum(ob ** 2)))
                    ref = max(onorm, float(floor[i, j]) if floor is not None else 0.0, 1e-300)
                    brel = math.sqrt(float(np.sum(blk ** 2))) / ref
                    nrel = abs(norm_g[i, j] - norm_o[i, j]) / ref
                rep.blocks_compared += 1
                rep.max_norm_rel = max(rep.max_norm_rel, nrel)
                if brel > rep.max_block_rel:
                    rep.max_block_rel = brel
                    rep.worst_block = (i, j, kg, int(rank_g[i, j]))
                continue
            ok = False
            if exact is not None and (i, j) in exact.blocks and tol > 0:
                eb = exact.blocks[(i, j)].dense()
                rk = [int(rank_g[i, j]) if kg else 0, int(rank_o[i, j]) if ko else 0]
                ok = ambiguous_cut(eb, tol, rk, ambiguous_rel)
            if ok:
                rep.ambiguous.append((i, j, kg, ko, int(rank_g[i, j]), int(rank_o[i, j])))
                diff[ro[i]:ro[i + 1], co[j]:co[j + 1]] = 0.0
            elif not same_kind:
                rep.kind_mismatch.append((i, j, kg, ko))
            else:
                rep.rank_mismatch.append((i, j, int(rank_g[i, j]), int(rank_o[i, j])))
    ref = math.sqrt(float(np.sum(Do ** 2)))
    rep.rel_err = math.sqrt(float(np.sum(diff ** 2))) / max(ref, 1e-300)
    return rep


def summary(rep: ParityReport) -> str:
    return (f"err={rep.rel_err:.2e} block_max={rep.max_block_rel:.2e} (block {rep.worst_block}) "
            f"norm_max={rep.max_norm_rel:.2e} blocks={rep.blocks_compared} "
            f"ambiguous={len(rep.ambiguous)}")


def assert_parity(rep: ParityReport, bound: float, max_ambiguous_frac: float = 0.02,
                  nblocks: int = 1, block_bound: Optional[float] = None,
                  norm_bound: Optional[float] = None):
    """Kinds and ranks equal (up to ambiguous cuts), the whole-matrix error, every block's own
    relative error and the norm table within their bounds (each defaults to ``bound``)."""
    assert not rep.kind_mismatch, f"kind mismatches: {rep.kind_mismatch[:10]}"
    assert not rep.rank_mismatch, f"rank mismatches: {rep.rank_mismatch[:10]}"
    assert len(rep.ambiguous) <= max(1, max_ambiguous_frac * nblocks), rep.ambiguous[:10]
    assert rep.rel_err <= bound, f"relative Frobenius error {rep.rel_err:.3e} > {bound:.1e}"
    bb = bound if block_bound is None else block_bound
    assert rep.max_block_rel <= bb, \
        f"block {rep.worst_block}: relative error {rep.max_block_rel:.3e} > {bb:.1e}"
    nb = bound if norm_bound is None else norm_bound
    assert rep.max_norm_rel <= nb, f"norm table: relative difference {rep.max_norm_rel:.3e} > {nb:.1e}"
