"""Pin checks for the oracle: each returns a number that must be small.

The mutation tests plant a mistake in the oracle and check that one of these
numbers becomes large, so the pins are known to bite.
"""
from __future__ import annotations

import math

import numpy as np

import oracle
import workloads as W
from conftest import read_golden


def linear_exactness(M=64, alpha=0.4, r=3.0):
    """L1 is exact on u(t) = t (u(0) = 0): R t = t_m^{1-alpha}/Gamma(2-alpha)
    (Caputo derivative of t).  Relative max error."""
    t = W.graded_mesh(M, 1.0, r)
    R = oracle.l1_matrix(t, alpha)
    want = t[1:] ** (1 - alpha) / math.gamma(2 - alpha)
    return float(np.max(np.abs(R @ t[1:] - want) / want))


def row_sums(M=64, alpha=0.6, r=2.0):
    """sum_j R_{m,j} = a_{m,1} = (t_m^{1-a} - (t_m - t_1)^{1-a}) / (Gamma(2-a) t_1):
    the discrete derivative of a constant (including u_0) vanishes."""
    t = W.graded_mesh(M, 1.0, r)
    R = oracle.l1_matrix(t, alpha)
    tm = t[1:]
    want = (tm ** (1 - alpha) - (tm - t[1]) ** (1 - alpha)) / (math.gamma(2 - alpha) * t[1])
    return float(np.max(np.abs(R.sum(axis=1) - want) / np.abs(want)))


def uniform_toeplitz(M=40, alpha=0.3):
    """Uniform mesh: R_{m,m} = dt^{-a}/G(2-a), R_{m,m-k} = ((k+1)^{1-a} - 2k^{1-a} + (k-1)^{1-a}) dt^{-a}/G(2-a),
    the textbook L1 coefficients."""
    t = W.graded_mesh(M, 1.0, 1.0)
    dt = 1.0 / M
    R = oracle.l1_matrix(t, alpha)
    c = dt ** (-alpha) / math.gamma(2 - alpha)
    want = np.zeros((M, M))
    for m in range(M):
        want[m, m] = c
        for kk in range(1, m + 1):
            want[m, m - kk] = c * ((kk + 1) ** (1 - alpha) - 2 * kk ** (1 - alpha) + (kk - 1) ** (1 - alpha))
    return float(np.max(np.abs(R - want)) / c)


def theorem_bound_violation(M=512, alpha=0.5, r=3.0, k=6, leaf=16):
    """max over admissible blocks of |R - A B^T| / bound (must be <= 1)."""
    t = W.graded_mesh(M, 1.0, r)
    R = oracle.l1_matrix(t, alpha)
    worst = 0.0
    for kind, rows, cols in oracle.block_partition(t, leaf):
        if kind != "rk":
            continue
        A, B = oracle.rk_factors(t, alpha, k, rows, cols)
        err = np.abs(R[rows.lo:rows.hi, cols.lo:cols.hi] - A @ B.T)
        bnd = oracle.theorem_bound(t, alpha, k, rows, cols)
        # allowance for the rounding of R itself (far entries lose relative accuracy)
        tol = 1e-15 * np.abs(np.diag(R)[rows.lo:rows.hi])[:, None]
        worst = max(worst, float(np.max(err / (bnd + tol))))
    return worst


def min_decay_ratio(M=256, alpha=0.5, r=3.0, ks=range(3, 9), leaf=16):
    """Smallest factor by which max|R - R~_k| shrinks per extra Taylor term
    (Theorem 3.1: about 3)."""
    t = W.graded_mesh(M, 1.0, r)
    R = oracle.l1_matrix(t, alpha)
    errs = [float(np.max(np.abs(oracle.hmatrix_dense(t, alpha, k, leaf, R=R) - R))) for k in ks]
    return min(a / b for a, b in zip(errs, errs[1:]))


def kron_mismatch(dim=1, n=7, M=32, alpha=0.5, r=3.0, k=4, leaf=4, seed=5):
    """Time marching vs dense Kronecker LU on a tiny grid with a random right-hand side
    and random initial value."""
    rng = np.random.default_rng(seed)
    t = W.graded_mesh(M, 1.0, r)
    Rt = oracle.hmatrix_dense(t, alpha, k, leaf)
    N = n ** dim
    F = rng.standard_normal((M, N))
    g = rng.standard_normal(N)
    B = oracle.rhs(F, t, alpha, g)
    U1 = oracle.timestep_solve(Rt, B, dim, n, 1.0)
    U2 = oracle.kron_solve(Rt, B, dim, n, 1.0)
    return float(np.max(np.abs(U1 - U2)) / np.max(np.abs(U2)))


def single_mode_mismatch(dim=1, n=31, M=64, alpha=0.5, kvec=None, length=1.0, k=8):
    """Time marching vs the single-sine-mode reduction."""
    if kvec is None:
        kvec = (3,) * dim
    t = W.graded_mesh(M, 1.0, W.default_grading(alpha))
    Rt = oracle.hmatrix_dense(t, alpha, k, 16)
    s = W.sine_mode(n, dim, length, kvec)
    phi = 1.0 + t[1:] ** alpha
    B = np.outer(phi, s)
    U = oracle.timestep_solve(Rt, B, dim, n, length)
    w = oracle.single_mode_profile(Rt, oracle.mode_eigenvalue(kvec, n, length), phi)
    return float(np.max(np.abs(U - np.outer(w, s))) / np.max(np.abs(U)))


def table1_ratio(alphas=(0.4, 0.6, 0.8), Ms=(32, 64, 128, 256, 512)):
    """max over the printed entries of |E_oracle / E_paper - 1| (first experiment,
    max error over all nodes, exact L1 matrix)."""
    printed = {(a, int(m)): e for a, m, e in read_golden("table1_max_errors.txt")}
    worst = 0.0
    got = {}
    for a in alphas:
        for m in Ms:
            p = W.paper_1d_mittag_leffler(1024, m, a)
            U = oracle.solve(p, k=None)
            ex = oracle.mittag_leffler(a, -p.t[1:] ** a)[:, None] * p.g[None, :]
            e = float(np.max(np.abs(U - ex)))
            got[(a, m)] = e
            worst = max(worst, abs(e / printed[(a, m)] - 1.0))
    return worst, got
