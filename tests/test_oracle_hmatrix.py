"""Pins of the oracle's H-matrix representation (Section 3)."""
import numpy as np
import pytest

import oracle
import pins
import workloads as W


def test_cluster_tree_leaves_partition_indices():
    for M in (128, 100, 33, 4096):
        root = oracle.cluster_tree(0, M, 16)
        leaves = []

        def walk(c):
            if c.is_leaf():
                leaves.append((c.lo, c.hi))
            for ch in c.children:
                walk(ch)
        walk(root)
        assert leaves[0][0] == 0 and leaves[-1][1] == M
        assert all(a[1] == b[0] for a, b in zip(leaves, leaves[1:]))
        assert all(0 < hi - lo <= 16 for lo, hi in leaves)


@pytest.mark.parametrize("M,r", [(128, 3.0), (300, 5.0), (1024, 1.0)])
def test_blocks_tile_lower_triangle_once(M, r):
    t = W.graded_mesh(M, 1.0, r)
    cover = np.zeros((M, M), dtype=int)
    for kind, rows, cols in oracle.block_partition(t, 16):
        cover[rows.lo:rows.hi, cols.lo:cols.hi] += 1
        if kind == "rk":
            assert cols.hi < rows.lo          # strictly below the diagonal, separated
    assert np.all(np.tril(cover) == np.tril(np.ones_like(cover)))
    assert np.all(cover <= 1)


def test_uniform_mesh_three_admissible_blocks_at_second_level():
    """Text around Figure 2: on a uniform mesh nothing is admissible after the first
    split and three blocks are admissible after the second."""
    t = W.graded_mesh(64, 1.0, 1.0)
    rk = [(rows.lo, cols.lo, rows.size) for kind, rows, cols in oracle.block_partition(t, 16) if kind == "rk"]
    assert sorted(rk) == [(32, 0, 16), (48, 0, 16), (48, 16, 16)]


def test_full_blocks_copy_R():
    t = W.graded_mesh(256, 1.0, 3.0)
    R = oracle.l1_matrix(t, 0.5)
    Rt = oracle.hmatrix_dense(t, 0.5, 8, 16, R=R)
    for kind, rows, cols in oracle.block_partition(t, 16):
        if kind == "full":
            assert np.array_equal(Rt[rows.lo:rows.hi, cols.lo:cols.hi], R[rows.lo:rows.hi, cols.lo:cols.hi])


@pytest.mark.parametrize("alpha,r,k", [(0.5, 3.0, 4), (0.5, 3.0, 10), (0.3, 17 / 3, 8), (0.8, 1.25, 12), (0.2, 9.0, 6)])
def test_theorem_31_entrywise_bound(alpha, r, k):
    assert pins.theorem_bound_violation(512, alpha, r, k) <= 1.0


def test_error_decays_like_three_to_minus_k():
    t = W.graded_mesh(1024, 1.0, 3.0)
    R = oracle.l1_matrix(t, 0.5)
    scale = np.max(np.diag(R))
    errs = []
    for k in range(3, 12):
        errs.append(np.max(np.abs(oracle.hmatrix_dense(t, 0.5, k, 16, R=R) - R)) / scale)
    ratios = [a / b for a, b in zip(errs, errs[1:]) if b > 1e-15]
    assert len(ratios) >= 5
    assert all(q >= 2.5 for q in ratios), ratios


def test_solution_error_shrinks_with_k():
    """Remark after Theorem 3.1: ||u - u~||_inf = O(3^-k)."""
    p = W.manufactured(1, 31, 512, 0.5, r=3.0)
    R = oracle.l1_matrix(p.t, p.alpha)
    lam = oracle.mode_eigenvalue((1,), p.n, p.length)
    phi = p.modes[0][1]
    w_exact = oracle.single_mode_profile(R, lam, phi)
    diffs = []
    for k in (4, 6, 8, 10, 12, 14, 16):
        Rt = oracle.hmatrix_dense(p.t, p.alpha, k, 16, R=R)
        diffs.append(np.max(np.abs(oracle.single_mode_profile(Rt, lam, phi) - w_exact)) / np.max(np.abs(w_exact)))
    # two more Taylor terms gain at least a factor 6 (3^2 = 9 asymptotically)
    assert all(a / b > 6.0 for a, b in zip(diffs, diffs[1:])), diffs
    assert diffs[-1] < 1e-9
