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


# ---- admissibility parameter eta and the geometric cluster tree ------------
# (the remark after Definition 3.1 allows other conditions; neither variant is
# the default, so the plain construction pinned above is unchanged)

def _block_q(t, rows, cols):
    """Contraction ratio of the Taylor series on a block (proof of Theorem
    3.1): q = |a - t_c| / (|a - t_c| + |a - d|), I_t = [a, b], I_s = [c, d]."""
    a, b, d = t[rows.lo + 1], t[rows.hi], t[cols.hi + 1]
    half = 0.5 * (b - a)
    return half / (half + (a - d))


@pytest.mark.parametrize("eta", [0.5, 2.0, 4.0])
@pytest.mark.parametrize("cluster", ["index", "geometric"])
def test_eta_blocks_obey_the_contraction_bound(eta, cluster):
    """diam <= eta dist gives q <= eta / (eta + 2) on every low-rank block
    (closed form), and the entrywise bound of Theorem 3.1's proof holds."""
    t = W.graded_mesh(512, 1.0, 3.0)
    R = oracle.l1_matrix(t, 0.5)
    Rt = oracle.hmatrix_dense(t, 0.5, 8, 16, R=R, eta=eta, cluster=cluster)
    qs = []
    for kind, rows, cols in oracle.block_partition(t, 16, eta, cluster):
        if kind != "rk":
            continue
        qs.append(_block_q(t, rows, cols))
        err = np.abs(Rt[rows.lo:rows.hi, cols.lo:cols.hi] - R[rows.lo:rows.hi, cols.lo:cols.hi])
        bound = oracle.theorem_bound(t, 0.5, 8, rows, cols)
        assert np.all(err <= bound * (1 + 1e-9) + 1e-15 * np.max(np.diag(R))), (eta, rows.lo, cols.lo)
    assert qs and max(qs) <= eta / (eta + 2.0) * (1 + 1e-12)
    if eta > 1.0:
        # the looser condition is really used: some block lies beyond eta = 1's ratio 1/3
        assert max(qs) > 1.0 / 3.0


def test_eta_to_zero_keeps_every_block_full():
    """No block satisfies diam <= eta dist for eta -> 0: R~ = R exactly."""
    t = W.graded_mesh(200, 1.0, 2.5)
    R = oracle.l1_matrix(t, 0.6)
    Rt = oracle.hmatrix_dense(t, 0.6, 6, 16, R=R, eta=1e-12)
    assert np.array_equal(Rt, R)


def test_eta_one_is_definition_31():
    t = W.graded_mesh(300, 1.0, 3.0)
    a = [(k, r.lo, r.hi, c.lo, c.hi) for k, r, c in oracle.block_partition(t, 16)]
    b = [(k, r.lo, r.hi, c.lo, c.hi) for k, r, c in oracle.block_partition(t, 16, 1.0, "index")]
    assert a == b


@pytest.mark.parametrize("M", [64, 256, 1024])
def test_geometric_tree_equals_index_tree_on_uniform_power_of_two_mesh(M):
    """Halving the time interval of a uniform mesh halves the index range when
    every cluster has an even size."""
    t = W.graded_mesh(M, 1.0, 1.0)
    a = [(k, r.lo, r.hi, c.lo, c.hi) for k, r, c in oracle.block_partition(t, 16, 1.0, "index")]
    b = [(k, r.lo, r.hi, c.lo, c.hi) for k, r, c in oracle.block_partition(t, 16, 1.0, "geometric")]
    assert a == b


@pytest.mark.parametrize("M,r", [(512, 3.0), (300, 17 / 3), (100, 1.5)])
def test_geometric_split_halves_time_intervals(M, r):
    """Brute force on every split: the first child holds exactly the levels
    not beyond the midpoint of the parent's time interval (unless that would
    leave a child empty), and the leaves partition 1..M with at most 16 levels."""
    t = W.graded_mesh(M, 1.0, r)
    root = oracle.cluster_tree(0, M, 16, "geometric", t)
    leaves = []

    def walk(c):
        if c.is_leaf():
            leaves.append((c.lo, c.hi))
            return
        a, b = c.children
        assert a.lo == c.lo and a.hi == b.lo and b.hi == c.hi and a.size >= 1 and b.size >= 1
        tm = 0.5 * (t[c.lo + 1] + t[c.hi])
        below = [m for m in range(c.lo + 1, c.hi + 1) if t[m] <= tm]
        want = min(max(len(below), 1), c.size - 1)
        assert a.size == want
        walk(a)
        walk(b)
    walk(root)
    assert leaves[0][0] == 0 and leaves[-1][1] == M
    assert all(x[1] == y[0] for x, y in zip(leaves, leaves[1:]))
    assert all(0 < hi - lo <= 16 for lo, hi in leaves)
