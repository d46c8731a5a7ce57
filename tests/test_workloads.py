"""The seeded input generators (no arithmetic of the method): orderings and kernels."""
import numpy as np

from workloads import (coulomb_3d_morton, coulomb_matrix, lattice_3d, lattice_3d_morton, lattice_side,
                       morton_order, points_3d, rng_for, scaled_workload)


def _sites(n):
    ns = lattice_side(n)
    idx = np.arange(n)
    return np.stack([idx // (ns * ns), (idx // ns) % ns, idx % ns], axis=1)


def test_morton_order_is_a_permutation_of_nested_cubes():
    # on a full 8^3 lattice every aligned run of 8^k sites is a 2^k x 2^k x 2^k cube
    n = 512
    o = morton_order(n)
    assert sorted(o.tolist()) == list(range(n))
    sites = _sites(n)[o]
    for run in (8, 64, 512):
        edge = round(run ** (1 / 3))
        for start in range(0, n, run):
            box = sites[start:start + run]
            assert np.all(box.max(axis=0) - box.min(axis=0) == edge - 1)
            assert len({tuple(s) for s in box}) == run


def test_morton_order_partial_lattice():
    # n below a full cube: still a permutation, first sites in the origin octant
    n = 700
    o = morton_order(n)
    assert sorted(o.tolist()) == list(range(n))
    assert np.all(_sites(n)[o[:8]] <= 1)


def test_morton_workload_reuses_the_lattice_draws():
    a = lattice_3d(1000)
    b = lattice_3d_morton(1000)
    o = morton_order(1000)
    assert np.array_equal(b.points, a.points[o])
    assert b.sizes == a.sizes and (b.a, b.diag, b.tol) == (a.a, a.diag, a.tol)


def test_coulomb_kernel_matrix():
    pts = points_3d(rng_for(11), 40, 1.0, 0.3)
    S = coulomb_matrix(pts, 1.0, 0.1)
    assert np.array_equal(S, S.T)
    assert np.allclose(np.diag(S), 1.1, rtol=0, atol=1e-15)
    i, j = 3, 17
    r2 = float(np.sum((pts[i] - pts[j]) ** 2))
    assert S[i, j] == 1.0 / np.sqrt(r2 + 1.0)
    # positive entries that decay with distance but never vanish
    far = np.argmax(np.sum((pts - pts[0]) ** 2, axis=1))
    assert 0 < S[0, far] < S[0, 1]


def test_coulomb_workload_dense_uses_the_coulomb_kernel():
    wl = scaled_workload("coulomb", 200, seed=5)
    assert wl.extra.get("kernel") == "coulomb"
    assert np.array_equal(wl.dense(), coulomb_matrix(wl.points, wl.a, wl.diag))
    big = coulomb_3d_morton(1000)
    assert big.extra.get("kernel") == "coulomb" and sum(big.sizes) == 1000
