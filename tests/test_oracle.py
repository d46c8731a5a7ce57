"""CPU tests that pin the FP64 oracle to the paper and to mathematics (no GPU)."""
import copy
import math
import types

import numpy as np
import pytest

import oracle as orc
from oracle import clr_oracle
import pins
from workloads import line_n512, random_blocks, rng_for


def test_triple_loop_bit_exact():
    assert pins.pin_triple_loop_exact(orc) == 0.0


def test_product_kinds_match_dense():
    assert pins.pin_product_kinds(orc) < 1e-14


def test_eckart_young_truncation():
    assert pins.pin_eckart_young(orc) < 1e-13


def test_lowrank_recompression_true_rank():
    assert pins.pin_lowrank_recompression(orc) < 1e-12


def test_screening_bounds_and_brute_force():
    assert pins.pin_screening(orc) < 1e-12


def test_ns_coefficients_eq9():
    assert pins.pin_ns_coefficients(orc) < 1e-15


def test_ns_diagonal_scalar_recurrence():
    assert pins.pin_ns_diagonal(orc) < 1e-13


def test_ns_cubic_rate():
    scalar, worst, e = pins.pin_cubic_rate(orc)
    assert scalar < 0.1 * 5.0 / 8.0
    assert e[-1] < 1e-14
    assert 0.0 < worst < 1.2


def test_dense_limit_exact():
    assert pins.pin_dense_limit(orc) < 1e-14


def test_sqrt_inv_matches_eigh_line_n512():
    """With per-product truncation at relative 1e-8 the explicit residual settles near 1e-9, so
    the iteration ends "stalled" above the 1e-10 target; the internal measure reaches 1e-16."""
    err, info = pins.pin_sqrt_inv_eigh(orc)
    assert info.status in ("converged", "stalled"), info
    assert info.internal[-1] < 1e-14
    assert info.explicit[-1][1] <= 1e-8
    assert err < 1e-8


def test_alpha_gershgorin_bound():
    wl = line_n512()
    S = orc.compress(wl.dense(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    a = orc.default_alpha(S)
    Sd = orc.to_dense(S)
    lam = np.linalg.eigvalsh(0.5 * (Sd + Sd.T))
    assert np.max(np.abs(a * lam - 1.0)) <= 1.0


def test_default_alpha_hand_value():
    """alpha of hand-set block norms: 1 / max row sum = 1/4 exactly (not a column sum, not smaller)."""
    assert pins.pin_default_alpha(orc) == 0.0


def test_screening_area_brute_force():
    """Per-area screening (tau = eps_sp m n): kept blocks are exactly the brute-force ones."""
    assert pins.pin_screening_area(orc) < 1e-13


@pytest.mark.parametrize("case", ["converged", "diverged", "stalled"])
def test_stop_statuses(case):
    res = {name: (ok, detail) for name, ok, detail in pins.pin_stop_statuses(orc)}
    ok, detail = res[case]
    assert ok, detail


def test_compress_rules_line_n512():
    """Drop below 1e-10, diagonal blocks dense, off-diagonal truncated; dense iff 2r > min."""
    wl = line_n512()
    Sd = wl.dense()
    S = orc.compress(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10)
    ro, co = S.offsets()
    for i in range(S.nrb):
        for j in range(S.ncb):
            blk = Sd[ro[i]:ro[i + 1], co[j]:co[j + 1]]
            nrm = float(np.sqrt(np.sum(blk ** 2)))
            b = S.blocks.get((i, j))
            if nrm < 1e-10:
                assert b is None
                continue
            assert b is not None
            if i == j:
                assert b.kind == "D"
                continue
            s = np.linalg.svd(blk, compute_uv=False)
            r = orc.truncation_rank(s, wl.tol, nrm)
            assert (b.kind == "D") == (2 * r > min(blk.shape))
            err = float(np.sqrt(np.sum((b.dense() - blk) ** 2)))
            assert err <= wl.tol * nrm * (1 + 1e-8)


def test_gemm_truncation_error_bound():
    """Each computed C block is within tol * ||C_IJ|| of the exact screened sum (Eckart-Young per block)."""
    wl = line_n512()
    S = orc.compress(wl.dense(), wl.sizes, wl.sizes, wl.tol, 1e-10)
    C = orc.gemm(S, S, wl.tol, wl.eps_sp)
    E = orc.gemm(S, S, 0.0, wl.eps_sp)
    ro, co = C.offsets()
    for key, b in C.blocks.items():
        ex = E.blocks[key].dense()
        nrm = float(np.sqrt(np.sum(ex ** 2)))
        assert float(np.sqrt(np.sum((b.dense() - ex) ** 2))) <= wl.tol * nrm * (1 + 1e-8) + 1e-15


def test_gemm_vjp_finite_difference():
    rows, inner, cols = [4, 3], [3, 5], [4, 2]
    ra = random_blocks(21, rows, inner, p_zero=0.0, p_dense=1.0)
    rb = random_blocks(22, inner, cols, p_zero=0.0, p_dense=1.0)
    A = orc.from_factors(ra.row_sizes, ra.col_sizes, ra.kind, ra.f0, ra.f1)
    B = orc.from_factors(rb.row_sizes, rb.col_sizes, rb.kind, rb.f0, rb.f1)
    G = rng_for(23).standard_normal((7, 6))
    dA, dB = orc.gemm_vjp(A, B, G, alpha=0.7)
    Ad, Bd = orc.to_dense(A), orc.to_dense(B)
    h = 1e-6
    for (i, j) in [(0, 0), (3, 6), (6, 2)]:
        Ap, Am = Ad.copy(), Ad.copy()
        Ap[i, j] += h
        Am[i, j] -= h
        fd = (np.sum(G * (0.7 * Ap @ Bd)) - np.sum(G * (0.7 * Am @ Bd))) / (2 * h)
        assert abs(fd - dA[i, j]) < 1e-7 * max(1.0, abs(fd))


def _small_spd(seed, n, sizes):
    rng = rng_for(seed)
    pts = np.sort(rng.uniform(0, n * 0.7, n))[:, None]
    from workloads import kernel_matrix
    return kernel_matrix(pts, 0.5, 0.1)


def test_sqrt_inv_vjp_finite_difference():
    """tol = 0 keeps the unrolled map smooth: central differences match the adjoint."""
    sizes = [5, 7, 6]
    Sd = _small_spd(31, 18, sizes)
    S = orc.compress(Sd, sizes, sizes, tol=0.0, drop=0.0)
    Wbar = rng_for(32).standard_normal((18, 18))
    alpha = orc.default_alpha(S)
    iters = 6
    dS, _W, _ = orc.sqrt_inv_vjp(S, Wbar, iters, 0.0, 0.0, alpha=alpha)
    h = 1e-6
    rng = rng_for(33)
    for _ in range(6):
        i, j = int(rng.integers(0, 18)), int(rng.integers(0, 18))
        vals = []
        for sgn in (1, -1):
            P = Sd.copy()
            P[i, j] += sgn * h
            Sp = orc.compress(P, sizes, sizes, tol=0.0, drop=0.0)
            Wp, _ = orc.sqrt_inv(Sp, 0.0, 0.0, fixed_iters=iters, alpha=alpha)
            vals.append(np.sum(Wbar * orc.to_dense(Wp)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - dS[i, j]) < 1e-6 * max(1.0, np.max(np.abs(dS)))


def test_sqrt_inv_vjp_daleckii_krein():
    """At convergence the adjoint equals the exact derivative of S^-1/2 (Daleckii-Krein form)."""
    sizes = [5, 7, 6]
    Sd = _small_spd(41, 18, sizes)
    Sd = 0.5 * (Sd + Sd.T)
    S = orc.compress(Sd, sizes, sizes, tol=0.0, drop=0.0)
    Wbar = rng_for(42).standard_normal((18, 18))
    dS, _W, _ = orc.sqrt_inv_vjp(S, Wbar, 20, 0.0, 0.0)
    lam, Q = np.linalg.eigh(Sd)
    sl = np.sqrt(lam)
    Gam = -1.0 / (sl[:, None] * sl[None, :] * (sl[:, None] + sl[None, :]))
    ref = Q @ (Gam * (Q.T @ Wbar @ Q)) @ Q.T
    assert np.max(np.abs(dS - ref)) < 1e-9 * np.max(np.abs(ref))


# ---------------------------------------------------------------------------
# Planted mistakes: a plausible error in the oracle must fail at least one pin.
# ---------------------------------------------------------------------------

def _mutant(patch):
    """A copy of the oracle module with one function replaced."""
    mod = types.ModuleType("oracle_mutant")
    mod.__dict__.update({k: v for k, v in clr_oracle.__dict__.items()})
    patch(mod)
    # functions look up globals in their own module: rebind them to the mutant's namespace
    for name, obj in list(mod.__dict__.items()):
        if isinstance(obj, types.FunctionType) and obj.__module__ == clr_oracle.__name__:
            mod.__dict__[name] = types.FunctionType(obj.__code__, mod.__dict__, obj.__name__,
                                                   obj.__defaults__, obj.__closure__)
    return mod


def _wrong_ld(mod):
    orig = mod.block_product

    def bp(a, b, alpha=1.0):
        if a.kind == "L" and b.kind == "D":
            return ("L", alpha * a.U, b.D @ a.V[: b.D.shape[1]] if b.D.shape[0] == b.D.shape[1]
                    else b.D.T @ a.V[::-1])
        return orig(a, b, alpha)
    mod.block_product = bp


def _wrong_absorb(mod):
    orig = mod.block_product

    def bp(a, b, alpha=1.0):
        if a.kind == "L" and b.kind == "L":
            Z = a.V.T @ b.U
            return ("L", alpha * a.U, b.V @ Z)  # missing transpose of the core
        return orig(a, b, alpha)
    mod.block_product = bp


def _wrong_tail(mod):
    def tr(sigma, tol, normc):
        n = len(sigma)
        for r in range(n + 1):
            if math.sqrt(float(np.sum(np.asarray(sigma[r + 1:]) ** 2))) <= tol * normc:  # off by one
                return r
        return n
    mod.truncation_rank = tr


def _wrong_ns_sign(mod):
    orig = mod.ns_T

    def ns(X, Q, tol, eps_sp, screen="abs"):
        return orig(X, mod.scale(Q, -1.0), tol, eps_sp, screen)  # sign of the X^2 term
    mod.ns_T = ns


def _wrong_screen(mod):
    orig = mod.block_tau
    mod.block_tau = lambda eps, m, n, screen: orig(eps, m, n, screen) * 1e3


def _dropped_term(mod):
    orig = mod.combine

    def comb(m, n, contribs, tol, tau, force_dense):
        return orig(m, n, contribs[:-1] if len(contribs) > 2 else contribs, tol, tau, force_dense)
    mod.combine = comb


def _alpha_column_sums(mod):
    def da(S):
        cols = np.zeros(S.ncb)
        for (_i, j), b in S.blocks.items():
            cols[j] += b.norm
        return 1.0 / float(np.max(cols))
    mod.default_alpha = da


def _alpha_smaller(mod):
    orig = mod.default_alpha
    mod.default_alpha = lambda S: 0.5 * orig(S)


def _area_as_abs(mod):
    mod.block_tau = lambda eps, m, n, screen: eps   # per-area mode ignored


MUTANTS = {
    "ld-operand": _wrong_ld,
    "ll-core-transpose": _wrong_absorb,
    "tail-off-by-one": _wrong_tail,
    "ns-sign": _wrong_ns_sign,
    "screen-threshold": _wrong_screen,
    "dropped-term": _dropped_term,
    "alpha-column-sums": _alpha_column_sums,
    "alpha-smaller": _alpha_smaller,
    "area-screen-as-abs": _area_as_abs,
}


def _pins_pass(mod):
    checks = [
        lambda: pins.pin_triple_loop_exact(mod) == 0.0,
        lambda: pins.pin_product_kinds(mod) < 1e-14,
        lambda: pins.pin_eckart_young(mod) < 1e-13,
        lambda: pins.pin_lowrank_recompression(mod) < 1e-12,
        lambda: pins.pin_screening(mod) < 1e-12,
        lambda: pins.pin_ns_coefficients(mod) < 1e-15,
        lambda: pins.pin_ns_diagonal(mod) < 1e-13,
        lambda: pins.pin_default_alpha(mod) == 0.0,
        lambda: pins.pin_screening_area(mod) < 1e-13,
    ]
    for c in checks:
        try:
            if not c():
                return False
        except Exception:
            return False
    return True


def test_unmutated_oracle_passes_fast_pins():
    assert _pins_pass(_mutant(lambda m: None))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    assert not _pins_pass(_mutant(MUTANTS[name]))


# ---------------------------------------------------------------------------
# Construction by rank-revealing QR (Sec. 4.1)
# ---------------------------------------------------------------------------

def test_rrqr_diagonal_example():
    # M = diag(1, 3, 2): greedy pivots take columns 1, 2, 0; R's rows have norms 3, 2, 1, so
    # the dropped parts are sqrt(14), sqrt(5), 1, 0 and tol ||M|| = 1.5 keeps rank 2: diag(0, 3, 2)
    M = np.diag([1.0, 3.0, 2.0])
    r, X, W, tails = orc.rrqr_truncate(M, 1.5 / math.sqrt(14.0))
    assert np.allclose(tails, [math.sqrt(14.0), math.sqrt(5.0), 1.0, 0.0], rtol=1e-15, atol=1e-15)
    assert r == 2
    assert np.allclose(X @ W.T, np.diag([0.0, 3.0, 2.0]), rtol=0, atol=1e-15)


def test_rrqr_exact_rank_error_identity_and_minimality():
    rng = rng_for(31)
    for (m, n, k) in ((40, 30, 7), (25, 60, 11), (50, 50, 1)):
        M = rng.standard_normal((m, k)) @ rng.standard_normal((k, n))
        r, X, W, tails = orc.rrqr_truncate(M, 1e-12)
        assert r == k
        assert np.allclose(X.T @ X, np.eye(r), atol=1e-13)
        # a smooth block: the kept error is exactly the dropped part of R, and r is minimal
        P = rng.standard_normal((m, 3))
        K = np.exp(-0.5 * (P[:, :1] - rng.standard_normal((1, n))) ** 2)
        for tol in (1e-3, 1e-6, 1e-9):
            r, X, W, tails = orc.rrqr_truncate(K, tol)
            nk = np.linalg.norm(K)
            err = np.linalg.norm(K - X @ W.T)
            assert abs(err - tails[r]) <= 1e-12 * nk
            assert tails[r] <= tol * nk and (r == 0 or tails[r - 1] > tol * nk)


def test_rrqr_rank_at_least_svd_rank():
    # Eckart-Young: no rank-r approximation beats the truncated SVD, so RRQR keeps at least as
    # many columns as the SVD for the same tolerance
    wl = line_n512()
    Sd = wl.dense()
    offs = wl.offsets()
    for (i, j) in ((0, 1), (2, 5), (3, 4), (1, 6)):
        D = Sd[offs[i]:offs[i + 1], offs[j]:offs[j + 1]]
        for tol in (1e-4, 1e-8, 1e-12):
            r, _X, _W, _t = orc.rrqr_truncate(D, tol)
            s = np.linalg.svd(D, compute_uv=False)
            assert r >= orc.truncation_rank(s, tol, float(np.linalg.norm(D)))


def test_compress_rrqr_rules_line_n512():
    wl = line_n512()
    Sd = wl.dense()
    O = orc.compress_rrqr(Sd, wl.sizes, wl.sizes, wl.tol, 1e-10)
    offs = wl.offsets()
    kinds = O.kinds()
    for i in range(len(wl.sizes)):
        assert kinds[i, i] == 1
        for j in range(len(wl.sizes)):
            D = Sd[offs[i]:offs[i + 1], offs[j]:offs[j + 1]]
            b = O.blocks.get((i, j))
            if b is None:
                assert np.linalg.norm(D) < 1e-10
                continue
            assert np.linalg.norm(D - b.dense()) <= wl.tol * np.linalg.norm(D) * (1 + 1e-12)
            if b.kind == "L":
                assert 2 * b.rank <= min(D.shape)
