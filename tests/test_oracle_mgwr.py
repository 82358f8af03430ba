"""Pins of the oracle's multigrid cycle (oracle/mgwr.py), on the CPU.

The semi-algebraic mode analysis (oracle/sama.py, pinned to Table 2's printed
factors) gives, for every sine-mode pair (1D) or quadruple (2D), the exact
action of the two-grid error propagation of Algorithm 2 with homogeneous
Dirichlet values.  With a zero right-hand side the oracle's cycle maps the
error, so on a two-grid hierarchy (coarse grid solved directly) it must
reproduce those blocks element by element: this fixes the smoother's colour
order and line solves, the defect, the restriction and interpolation
weights and the coarse operator.  A cycle with any of them changed (planted
below) misses the blocks by orders of magnitude more than rounding.
"""
import math

import numpy as np
import pytest

import oracle
import oracle.mgwr as omg
import oracle.sama as sama
import workloads as W


def _R(M, alpha, r):
    return oracle.l1_matrix(W.graded_mesh(M, 1.0, r), alpha)


def _modes_1d(n, k):
    i = np.arange(1, n + 1)
    s = np.sin(k * math.pi * i / (n + 1))
    red = (i % 2 == 0)
    return np.where(red, s, 0.0), np.where(red, 0.0, s)


def _two_grid_mismatch_1d(R, n, nu1, nu2, rng, cyc=omg.cycle):
    """Largest relative mismatch over the frequencies between the oracle's
    two-grid cycle on e_R a + e_B b and the SAMA block applied to (a, b)."""
    h = 1.0 / (n + 1)
    M = R.shape[0]
    nc = (n - 1) // 2
    worst = 0.0
    for k in range(1, nc + 1):
        eR, eB = _modes_1d(n, k)
        a, b = rng.standard_normal(M), rng.standard_normal(M)
        U0 = np.outer(a, eR) + np.outer(b, eB)
        U1 = cyc(R, U0, np.zeros_like(U0), 1, n, 1.0, nu1=nu1, nu2=nu2, gamma=1, coarsest=nc)
        ab = sama.two_grid_block(R, h, k * math.pi / (n + 1), nu1, nu2) @ np.concatenate([a, b])
        want = np.outer(ab[:M], eR) + np.outer(ab[M:], eB)
        scale = max(np.max(np.abs(want)), np.max(np.abs(U0)))
        worst = max(worst, np.max(np.abs(U1 - want)) / scale)
    return worst


def _modes_2d(n, k1, k2):
    """e = s, f = (-1)^(i+1) s with s(i, j) = sin(k1 pi i/(n+1)) sin(k2 pi j/(n+1)),
    i the 1-based x index, j the y index; split into the red ((i + j) even) and
    black parts; flattened with y major (flat index y n + x)."""
    j, i = np.meshgrid(np.arange(1, n + 1), np.arange(1, n + 1), indexing="ij")
    s = np.sin(k1 * math.pi * i / (n + 1)) * np.sin(k2 * math.pi * j / (n + 1))
    f = (-1.0) ** (i + 1) * s
    red = (i + j) % 2 == 0
    parts = [np.where(red, s, 0.0), np.where(red, 0.0, s), np.where(red, f, 0.0), np.where(red, 0.0, f)]
    return [p.reshape(-1) for p in parts]


def _two_grid_mismatch_2d(R, n, nu1, nu2, rng, cyc=omg.cycle):
    h = 1.0 / (n + 1)
    M = R.shape[0]
    nc = (n - 1) // 2
    worst = 0.0
    zero = None
    for k1 in range(1, nc + 1):
        for k2 in range(1, nc + 1):
            parts = _modes_2d(n, k1, k2)
            coef = [rng.standard_normal(M) for _ in range(4)]
            U0 = sum(np.outer(c, p) for c, p in zip(coef, parts))
            zero = np.zeros_like(U0)
            U1 = cyc(R, U0, zero, 2, n, 1.0, nu1=nu1, nu2=nu2, gamma=1, coarsest=nc)
            T = sama.two_grid_block_2d(R, h, k1 * math.pi / (n + 1), k2 * math.pi / (n + 1), nu1, nu2)
            out = T @ np.concatenate(coef)
            want = sum(np.outer(out[q * M:(q + 1) * M], p) for q, p in enumerate(parts))
            scale = max(np.max(np.abs(want)), np.max(np.abs(U0)))
            worst = max(worst, np.max(np.abs(U1 - want)) / scale)
    # one index (n + 1)/2: no coarse-grid correction reaches the mode, only the smoother acts
    kh = (n + 1) // 2
    for k in range(1, nc + 1):
        e = _modes_2d(n, kh, k)
        sR, sB = e[0], e[1]
        a, b = rng.standard_normal(M), rng.standard_normal(M)
        U0 = np.outer(a, sR) + np.outer(b, sB)
        U1 = cyc(R, U0, np.zeros_like(U0), 2, n, 1.0, nu1=nu1, nu2=nu2, gamma=1, coarsest=nc)
        ab = sama.smoother_block_2d(R, h, k * math.pi / (n + 1), nu1 + nu2) @ np.concatenate([a, b])
        want = np.outer(ab[:M], sR) + np.outer(ab[M:], sB)
        scale = max(np.max(np.abs(want)), np.max(np.abs(U0)))
        worst = max(worst, np.max(np.abs(U1 - want)) / scale)
    return worst


@pytest.mark.parametrize("nu1,nu2", [(1, 0), (1, 1), (0, 1), (2, 1)])
def test_two_grid_cycle_matches_sama_blocks_1d(nu1, nu2):
    rng = np.random.default_rng(3 + nu1 + 5 * nu2)
    R = _R(12, 0.4, 2.0 / 0.4 - 0.5)
    assert _two_grid_mismatch_1d(R, 15, nu1, nu2, rng) < 1e-11


@pytest.mark.parametrize("nu1,nu2", [(1, 0), (1, 1), (0, 1)])
def test_two_grid_cycle_matches_sama_blocks_2d(nu1, nu2):
    rng = np.random.default_rng(11 + nu1 + 5 * nu2)
    R = _R(8, 0.6, 3.0)
    assert _two_grid_mismatch_2d(R, 7, nu1, nu2, rng) < 1e-11


def _mutant(monkeypatch, what):
    """Plants one mistake in the oracle's cycle (module attributes the cycle
    looks up at call time)."""
    if what == "colour order":
        first, second = omg._first_colour, omg._second_colour
        monkeypatch.setattr(omg, "_first_colour", second)
        monkeypatch.setattr(omg, "_second_colour", first)
    elif what == "restriction weights":
        orig = omg._restrict_axis
        monkeypatch.setattr(omg, "_restrict_axis", lambda a, axis: 2.0 * orig(a, axis))
    elif what == "interpolation weights":
        orig = omg._prolong_axis

        def half_between(e, axis):
            out = np.moveaxis(orig(e, axis), axis, -1).copy()
            out[..., 0::2] *= 0.5
            return np.moveaxis(out, -1, axis)
        monkeypatch.setattr(omg, "_prolong_axis", half_between)
    elif what == "coarse spacing":
        orig = omg.timestep_solve     # the coarse grid solved with the fine grid's h
        monkeypatch.setattr(omg, "timestep_solve", lambda Rt, B, dim, n, length: orig(Rt, B, dim, n, 0.5 * length))
    elif what == "defect sign":
        orig = omg.laplacian_apply
        monkeypatch.setattr(omg, "laplacian_apply", lambda U, dim, n, h: -orig(U, dim, n, h))
    return omg.cycle


@pytest.mark.parametrize("what", ["colour order", "restriction weights", "interpolation weights",
                                  "coarse spacing", "defect sign"])
def test_sama_pin_catches_planted_mistakes(monkeypatch, what):
    """Each planted mistake in the oracle's cycle misses the SAMA blocks."""
    R = _R(8, 0.5, 3.0)
    rng = np.random.default_rng(1)
    cyc = _mutant(monkeypatch, what)
    bad1 = _two_grid_mismatch_1d(R, 15, 1, 1, rng, cyc=cyc)
    bad2 = _two_grid_mismatch_2d(R, 7, 1, 1, rng, cyc=cyc)
    assert bad1 > 1e-4 and bad2 > 1e-4, (what, bad1, bad2)


@pytest.mark.parametrize("dim,n,M,gamma", [(1, 31, 24, 1), (1, 15, 16, 2), (2, 15, 12, 1), (2, 7, 10, 2)])
def test_direct_solution_is_a_fixed_point_and_cycles_converge_to_it(dim, n, M, gamma):
    rng = np.random.default_rng(dim * 100 + n)
    alpha = 0.5
    t = W.graded_mesh(M, 1.0, 3.0)
    Rt = oracle.hmatrix_dense(t, alpha, 6, 4)
    B = rng.standard_normal((M, n ** dim))
    ref = oracle.timestep_solve(Rt, B, dim, n, 1.0)
    fixed = omg.cycle(Rt, ref, B, dim, n, 1.0, gamma=gamma)
    assert np.max(np.abs(fixed - ref)) <= 1e-12 * np.max(np.abs(ref))
    its = omg.cycles(Rt, B, dim, n, 1.0, 14, gamma=gamma)
    res = [np.max(np.abs(oracle.residual(Rt, U, B, dim, n, 1.0))) / np.max(np.abs(B)) for U in its]
    assert res[-1] < 1e-10, res
    assert all(b < 0.5 * a for a, b in zip(res[:6], res[1:7])), res
    assert np.max(np.abs(its[-1] - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_restriction_and_interpolation_on_small_grids():
    """The transfers written out on a 1D grid of 7 points and a 2D grid of
    3 x 3: full weighting is a quarter of the transpose of linear
    interpolation per direction, and interpolation is exact on grid functions
    linear between the coarse points."""
    e = np.array([[1.0, 2.0, 3.0]])
    assert np.allclose(omg.prolong(e, 1, 3), [[0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 1.5]])
    r = np.array([[1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0]])
    assert np.allclose(omg.restrict(r, 1, 7), [[2.0, 4.0, 6.0]])
    P = np.stack([omg.prolong(np.eye(3)[i][None, :], 1, 3)[0] for i in range(3)], axis=1)   # 7 x 3
    Rw = np.stack([omg.restrict(np.eye(7)[i][None, :], 1, 7)[0] for i in range(7)], axis=1)  # 3 x 7
    assert np.allclose(Rw, 0.5 * P.T)
    g = np.zeros((1, 9))
    g[0, 4] = 16.0                       # the middle fine point of a 3 x 3 grid
    assert np.allclose(omg.restrict(g, 2, 3), [[4.0]])
    c = omg.prolong(np.array([[8.0]]), 2, 1).reshape(3, 3)
    assert np.allclose(c, [[2.0, 4.0, 2.0], [4.0, 8.0, 4.0], [2.0, 4.0, 2.0]])
