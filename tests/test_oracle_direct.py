"""Pins of the oracle's direct time marching and of the whole oracle chain."""
import math

import numpy as np
import pytest

import oracle
import pins
import workloads as W
from conftest import read_golden


@pytest.mark.parametrize("dim,n", [(1, 7), (1, 8), (2, 3), (2, 5)])
def test_time_marching_matches_dense_kronecker_lu(dim, n):
    assert pins.kron_mismatch(dim=dim, n=n) < 1e-12


@pytest.mark.parametrize("dim,n,kvec", [(1, 31, (3,)), (1, 63, (1,)), (2, 15, (2, 5)), (2, 31, (1, 1))])
def test_time_marching_matches_single_mode_reduction(dim, n, kvec):
    assert pins.single_mode_mismatch(dim=dim, n=n, kvec=kvec) < 1e-12


def test_residual_of_direct_solution_is_rounding():
    p = W.manufactured(2, 15, 64, 0.5, r=3.0, k=8)
    Rt = oracle.hmatrix_dense(p.t, p.alpha, p.k, 16)
    B = oracle.rhs(p.f, p.t, p.alpha, p.g)
    U = oracle.timestep_solve(Rt, B, 2, p.n, p.length)
    r = oracle.residual(Rt, U, B, 2, p.n, p.length)
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(B))
    cols = np.array([0, 5, 17, 100, 224])
    rc = oracle.residual_columns(Rt, U + 1e-3, B, 2, p.n, p.length, cols)
    rf = oracle.residual(Rt, U + 1e-3, B, 2, p.n, p.length)[:, cols]
    assert np.max(np.abs(rc - rf)) < 1e-12 * np.max(np.abs(rf))


def test_table1_max_errors_and_orders():
    """Values printed in Table 1 (two significant digits): within 8%."""
    worst, got = pins.table1_ratio()
    assert worst < 0.08, got
    for a, m, order in read_golden("table1_orders.txt"):
        mine = math.log2(got[(a, int(m))] / got[(a, int(m) * 2)])
        assert abs(mine - order) < 0.08, (a, m, mine, order)


@pytest.mark.parametrize("alpha,r", [(0.5, 3.0), (0.3, 17 / 3), (0.7, 3.0), (0.5, None)])
def test_graded_mesh_convergence_order(alpha, r):
    """Section 2: order min(r alpha, 2 - alpha) in time on the graded mesh for the
    typical solution t^alpha; approached from below."""
    if r is None:
        r = W.default_grading(alpha)
    expect = min(r * alpha, 2 - alpha)
    lam = math.pi ** 2      # time discretisation alone: D^a w + pi^2 w = G(1+a) + pi^2 t^a, w = t^a
    errs = []
    Ms = (128, 256, 512, 1024, 2048)
    for M in Ms:
        t = W.graded_mesh(M, 1.0, r)
        R = oracle.l1_matrix(t, alpha)
        phi = math.gamma(1 + alpha) + lam * t[1:] ** alpha
        w = oracle.single_mode_profile(R, lam, phi)
        errs.append(np.max(np.abs(w - t[1:] ** alpha)))
    orders = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(b >= a - 0.01 for a, b in zip(orders, orders[1:])), orders
    assert expect - 0.12 < orders[-1] < expect + 0.05, (orders, expect)


def test_uniform_mesh_order_is_alpha():
    """Section 2: order alpha on the uniform mesh (slowly approached)."""
    alpha = 0.5
    lam = math.pi ** 2
    errs = []
    for M in (256, 512, 1024, 2048):
        t = W.graded_mesh(M, 1.0, 1.0)
        R = oracle.l1_matrix(t, alpha)
        phi = math.gamma(1 + alpha) + lam * t[1:] ** alpha
        errs.append(np.max(np.abs(oracle.single_mode_profile(R, lam, phi) - t[1:] ** alpha)))
    order = math.log2(errs[-2] / errs[-1])
    assert alpha - 0.2 < order < alpha + 0.05


def test_mittag_leffler_special_values():
    # E_1(z) = exp(z); E_{1/2}(-x) = exp(x^2) erfc(x)
    z = np.linspace(-1, 0, 7)
    assert np.max(np.abs(oracle.mittag_leffler(1.0, z) - np.exp(z))) < 1e-14
    x = np.linspace(0, 1, 5)
    ref = np.array([math.exp(v * v) * math.erfc(v) for v in x])
    assert np.max(np.abs(oracle.mittag_leffler(0.5, -x) - ref)) < 1e-13


def test_sampled_residual_equals_full_residual_on_those_points():
    """The residual from gathered time lines equals the full residual at the
    same points (1D and 2D, boundary points included)."""
    rng = np.random.default_rng(5)
    for dim, n in ((1, 15), (2, 7)):
        M = 40
        t = W.graded_mesh(M, 1.0, 3.0)
        Rt = oracle.hmatrix_dense(t, 0.4, 6)
        N = n ** dim
        U = rng.standard_normal((M, N))
        B = rng.standard_normal((M, N))
        h = 1.0 / (n + 1)
        full = oracle.residual(Rt, U, B, dim, n, 1.0)
        cols = np.array([0, 1, N // 2, N - 1])
        nb = []
        if dim == 1:
            pairs = [(cols - 1, cols >= 1), (cols + 1, cols + 1 < n)]
        else:
            ix, iy = cols % n, cols // n
            pairs = [(cols - 1, ix > 0), (cols + 1, ix < n - 1), (cols - n, iy > 0), (cols + n, iy < n - 1)]
        for q, ok in pairs:
            nb.append(np.where(ok[None, :], U[:, np.where(ok, q, 0)], 0.0))
        r = oracle.residual_sampled(Rt, B[:, cols], U[:, cols], nb, h)
        assert np.max(np.abs(r - full[:, cols])) <= 1e-12 * np.max(np.abs(full))
