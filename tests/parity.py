"""Comparison of a GPU CLR result with the oracle's, block by block.

Discrete decisions (zero / dense / low rank, kept rank) must agree exactly,
except where the oracle's own truncation is ambiguous: the dropped tail at the
oracle's or the GPU's rank lies within relative 1e-6 of tol * ||C_IJ||_F, so
that either rank is correct up to rounding.  Reconstructed values are compared
by relative Frobenius error over the whole matrix.
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


def tails_of(block: np.ndarray) -> np.ndarray:
    s = np.linalg.svd(block, compute_uv=False)
    t = np.zeros(len(s) + 1)
    acc = 0.0
    for i in range(len(s) - 1, -1, -1):
        acc += s[i] ** 2
        t[i] = acc
    return np.sqrt(t)


def ambiguous_cut(exact_block: np.ndarray, tol: float, ranks) -> bool:
    t = tails_of(exact_block)
    bound = tol * math.sqrt(float(np.sum(exact_block ** 2)))
    for r in ranks:
        for rr in (r - 1, r):
            if 0 <= rr < len(t) and abs(t[rr] - bound) <= 1e-6 * bound:
                return True
    return False


def compare(gpu, omat: orc.OMatrix, tol: float, exact: Optional[orc.OMatrix] = None,
            dense_gpu: Optional[np.ndarray] = None) -> ParityReport:
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
                if ko != 0:
                    rel = abs(norm_g[i, j] - norm_o[i, j]) / max(norm_o[i, j], 1e-300)
                    rep.max_norm_rel = max(rep.max_norm_rel, rel)
                continue
            ok = False
            if exact is not None and (i, j) in exact.blocks and tol > 0:
                eb = exact.blocks[(i, j)].dense()
                rk = [int(rank_g[i, j]) if kg else 0, int(rank_o[i, j]) if ko else 0]
                ok = ambiguous_cut(eb, tol, rk)
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


def assert_parity(rep: ParityReport, bound: float, max_ambiguous_frac: float = 0.02,
                  nblocks: int = 1):
    assert not rep.kind_mismatch, f"kind mismatches: {rep.kind_mismatch[:10]}"
    assert not rep.rank_mismatch, f"rank mismatches: {rep.rank_mismatch[:10]}"
    assert len(rep.ambiguous) <= max(1, max_ambiguous_frac * nblocks), rep.ambiguous[:10]
    assert rep.rel_err <= bound, f"relative Frobenius error {rep.rel_err:.3e} > {bound:.1e}"
