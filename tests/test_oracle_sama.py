"""Pins of the semi-algebraic mode analysis (oracle/sama.py): the exact
block decomposition against the brute-force spectral radius of the assembled
two-grid matrix on tiny grids, a closed-form special case, and the values
Table 2 prints."""
import math

import numpy as np
import pytest

import oracle
import oracle.sama as S
import workloads as W
from conftest import read_golden


def _two_grid_matrix(R, n, h, nu1, nu2):
    """The two-grid error propagation of Algorithm 2 (one space dimension)
    assembled from its definitions on an [n][M] error array: zebra
    half-sweeps (even 1-based points first), full weighting, linear
    interpolation, exact solve with R + A_{2h} on the coarse grid."""
    M = R.shape[0]
    nc = (n - 1) // 2
    D = R + (2.0 / h ** 2) * np.eye(M)

    def A(E):   # E [n][M]
        out = E @ R.T + (2.0 / h ** 2) * E
        out[1:] -= E[:-1] / h ** 2
        out[:-1] -= E[1:] / h ** 2
        return out

    def smooth(E):
        E = E.copy()
        for parity in (1, 0):          # 0-based odd = 1-based even first
            for i in range(parity, n, 2):
                nb = (E[i - 1] if i > 0 else 0.0) + (E[i + 1] if i + 1 < n else 0.0)
                E[i] = np.linalg.solve(D, nb / h ** 2)
        return E

    Hc = 2.0 * h
    Ac = np.kron(np.eye(nc), R) + np.kron((2 * np.eye(nc) - np.eye(nc, k=1) - np.eye(nc, k=-1)) / Hc ** 2,
                                          np.eye(M))

    def cgc(E):
        r = -A(E)
        rc = np.array([(r[2 * j] + 2 * r[2 * j + 1] + r[2 * j + 2]) / 4.0 for j in range(nc)])
        ec = np.linalg.solve(Ac, rc.reshape(-1)).reshape(nc, M)
        corr = np.zeros_like(E)
        for j in range(nc):
            corr[2 * j + 1] += ec[j]
            corr[2 * j] += 0.5 * ec[j]
            corr[2 * j + 2] += 0.5 * ec[j]
        return E + corr

    cols = []
    for col in range(n * M):
        E = np.zeros(n * M)
        E[col] = 1.0
        E = E.reshape(n, M)
        for _ in range(nu1):
            E = smooth(E)
        E = cgc(E)
        for _ in range(nu2):
            E = smooth(E)
        cols.append(E.reshape(-1))
    return np.array(cols).T


@pytest.mark.parametrize("n,M,alpha,r,nu1,nu2", [(7, 8, 0.5, 3.0, 1, 0), (15, 6, 0.3, 17 / 3, 0, 1),
                                                 (7, 10, 0.8, 1.25, 1, 1), (3, 12, 0.6, 1.0, 2, 0)])
def test_blocks_equal_brute_force_two_grid_matrix(n, M, alpha, r, nu1, nu2):
    """The assembled two-grid matrix maps e_R (x) a + e_B (x) b of every
    frequency pair to e_R (x) a' + e_B (x) b' with (a'; b') the block formula
    applied to (a; b) (the decomposition is exact with Dirichlet sine modes),
    and removes the mode k = (n+1)/2."""
    t = W.graded_mesh(M, 1.0, r)
    R = oracle.l1_matrix(t, alpha)
    h = math.pi / (n + 1)
    Tbf = _two_grid_matrix(R, n, h, nu1, nu2)
    rng = np.random.default_rng([n, M])
    i = np.arange(1, n + 1)
    scale = np.abs(Tbf).max()
    for k in range(1, (n - 1) // 2 + 1):
        s = np.sin(k * math.pi * i / (n + 1))
        eR, eB = np.where(i % 2 == 0, s, 0.0), np.where(i % 2 == 1, s, 0.0)
        a, b = rng.standard_normal(M), rng.standard_normal(M)
        out = (Tbf @ (np.outer(eR, a) + np.outer(eB, b)).reshape(-1)).reshape(n, M)
        ab = S.two_grid_block(R, h, k * math.pi / (n + 1), nu1, nu2) @ np.concatenate([a, b])
        want = np.outer(eR, ab[:M]) + np.outer(eB, ab[M:])
        assert np.max(np.abs(out - want)) <= 1e-10 * max(scale, 1.0), k
    s = np.sin(math.pi * i / 2.0)
    out = (Tbf @ np.outer(s, rng.standard_normal(M)).reshape(-1)).reshape(n, M)
    if nu1 + nu2 >= 1:
        assert np.max(np.abs(out)) <= 1e-10 * max(scale, 1.0)


def test_blocks_are_lower_triangular_in_time_with_scalar_diagonal_blocks():
    """Causality: the block of a frequency is block lower triangular in time,
    its 2 x 2 diagonal blocks are the formula with R_{m,m}, so the factor is
    the largest of their spectral radii."""
    M = 9
    t = W.graded_mesh(M, 1.0, 3.0)
    R = oracle.l1_matrix(t, 0.4)
    h = math.pi / 16
    for k in (1, 3, 7):
        B = S.two_grid_block(R, h, k * math.pi / 16)
        idx = np.concatenate([np.arange(M), np.arange(M)])          # time level of each row / column
        upper = idx[None, :] > idx[:, None]
        assert np.max(np.abs(B[upper])) <= 1e-12 * np.max(np.abs(B))
        for m in range(M):
            sub = B[np.ix_([m, M + m], [m, M + m])]
            ref = S.two_grid_block(np.array([[R[m, m]]]), h, k * math.pi / 16)
            assert np.max(np.abs(sub - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_no_time_term_gives_an_exact_two_grid_step():
    """R = 0 leaves the 1D Laplacian, for which red-black relaxation, full
    weighting and linear interpolation make the two-grid method exact."""
    assert S.two_grid_factor(31, 5, 0.5, 1.0, R=np.zeros((5, 5))) < 1e-12


def test_table2_sama_column():
    """The factors Table 2 prints (outside the brackets) within 0.003."""
    worst = 0.0
    for delta, M, printed in read_golden("table2_sama.txt"):
        M = int(M)
        got = S.two_grid_factor(M - 1, M, delta, (2 - delta) / delta)
        worst = max(worst, abs(got - printed))
        assert abs(got - printed) <= 0.003, (delta, M, got, printed)
    print("worst deviation from Table 2", worst)


@pytest.mark.parametrize("mutant", ["black_first", "interp_sign", "coarse_shift"])
def test_planted_mistake_fails_the_brute_force_identity(monkeypatch, mutant):
    """A plausible slip in the block formulas breaks the identity with the
    assembled two-grid matrix."""
    true = S.two_grid_block

    def wrong(R, h, theta, nu1=1, nu2=0):
        M = R.shape[0]
        I = np.eye(M)
        c = math.cos(theta)
        D = R + (2.0 / (h * h)) * I
        Dinv = np.linalg.inv(D)
        g = 2.0 * c / (h * h)
        A = np.block([[D, -g * I], [-g * I, D]])
        if mutant == "black_first":
            Sm = np.block([[g * g * Dinv @ Dinv, np.zeros((M, M))], [g * Dinv, np.zeros((M, M))]])
        else:
            Sm = np.block([[np.zeros((M, M)), g * Dinv], [np.zeros((M, M)), g * g * Dinv @ Dinv]])
        P = np.vstack([I, (-c if mutant == "interp_sign" else c) * I])
        lam = math.sin(theta) ** 2 / (h * h) if mutant != "coarse_shift" else 4 * math.sin(theta / 2) ** 2 / (h * h)
        K = np.eye(2 * M) - P @ np.linalg.solve(R + lam * I, np.hstack([0.5 * I, 0.5 * c * I]) @ A)
        T = K
        for _ in range(nu1):
            T = T @ Sm
        for _ in range(nu2):
            T = Sm @ T
        return T

    monkeypatch.setattr(S, "two_grid_block", wrong)
    with pytest.raises(AssertionError):
        test_blocks_equal_brute_force_two_grid_matrix(7, 8, 0.5, 3.0, 1, 0)
    monkeypatch.setattr(S, "two_grid_block", true)


def _two_grid_matrix_2d(R, n, h, nu1, nu2):
    """The 2D two-grid error propagation assembled from its definitions on an
    [n][n][M] error array (checkerboard zebra half-sweeps, (i + j) even
    first, 1-based; 9-point full weighting; bilinear interpolation; exact
    solve with R + A_{2h} on the coarse grid)."""
    M = R.shape[0]
    nc = (n - 1) // 2
    D = R + (4.0 / h ** 2) * np.eye(M)

    def nbsum(E, i, j):
        s = 0.0
        for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
            if 0 <= i + di < n and 0 <= j + dj < n:
                s = s + E[i + di, j + dj]
        return s

    def A(E):
        out = np.einsum("ijm,km->ijk", E, R) + (4.0 / h ** 2) * E
        for i in range(n):
            for j in range(n):
                out[i, j] = out[i, j] - nbsum(E, i, j) / h ** 2
        return out

    def smooth(E):
        E = E.copy()
        for parity in (0, 1):      # (i + j) even (1-based) = (i0 + j0) even (0-based) first
            for i in range(n):
                for j in range(n):
                    if (i + j) % 2 == parity:
                        E[i, j] = np.linalg.solve(D, nbsum(E, i, j) / h ** 2)
        return E

    H = 2.0 * h
    T1 = (2 * np.eye(nc) - np.eye(nc, k=1) - np.eye(nc, k=-1)) / H ** 2
    Ac = np.kron(np.eye(nc * nc), R) + np.kron(np.kron(np.eye(nc), T1) + np.kron(T1, np.eye(nc)), np.eye(M))

    def cgc(E):
        r = -A(E)
        rc = np.zeros((nc, nc, M))
        for I in range(nc):
            for J in range(nc):
                fi, fj = 2 * I + 1, 2 * J + 1
                for di in (-1, 0, 1):
                    for dj in (-1, 0, 1):
                        rc[I, J] += (2 - abs(di)) * (2 - abs(dj)) / 16.0 * r[fi + di, fj + dj]
        ec = np.linalg.solve(Ac, rc.reshape(-1)).reshape(nc, nc, M)
        corr = np.zeros_like(E)
        for I in range(nc):
            for J in range(nc):
                fi, fj = 2 * I + 1, 2 * J + 1
                for di in (-1, 0, 1):
                    for dj in (-1, 0, 1):
                        corr[fi + di, fj + dj] += (1 - 0.5 * abs(di)) * (1 - 0.5 * abs(dj)) * ec[I, J]
        return E + corr

    cols = []
    for col in range(n * n * M):
        E = np.zeros(n * n * M)
        E[col] = 1.0
        E = E.reshape(n, n, M)
        for _ in range(nu1):
            E = smooth(E)
        E = cgc(E)
        for _ in range(nu2):
            E = smooth(E)
        cols.append(E.reshape(-1))
    return np.array(cols).T


@pytest.mark.parametrize("nu1,nu2", [(1, 0), (0, 1)])
def test_2d_blocks_equal_brute_force_two_grid_matrix(nu1, nu2):
    """2D: the assembled two-grid matrix maps the four harmonics of every
    low-frequency pair as the 4M x 4M block says, the frequencies with an
    index (n+1)/2 as the smoother alone says."""
    n, M = 7, 3
    t = W.graded_mesh(M, 1.0, 3.0)
    R = oracle.l1_matrix(t, 0.4)
    h = math.pi / (n + 1)
    Tbf = _two_grid_matrix_2d(R, n, h, nu1, nu2)
    scale = max(1.0, np.abs(Tbf).max())
    i = np.arange(1, n + 1)[:, None]
    j = np.arange(1, n + 1)[None, :]
    red = (i + j) % 2 == 0
    rng = np.random.default_rng(3)

    def apply(field_coeffs):
        v = sum(np.einsum("ij,m->ijm", fld, cf) for fld, cf in field_coeffs)
        return (Tbf @ v.reshape(-1)).reshape(n, n, M)

    nc = (n - 1) // 2
    for k1 in range(1, nc + 1):
        for k2 in range(1, nc + 1):
            s = np.sin(k1 * math.pi * i / (n + 1)) * np.sin(k2 * math.pi * j / (n + 1))
            f = (-1.0) ** (i + 1) * s
            parts = [np.where(red, s, 0.0), np.where(~red, s, 0.0), np.where(red, f, 0.0), np.where(~red, f, 0.0)]
            coef = [rng.standard_normal(M) for _ in range(4)]
            out = apply(zip(parts, coef))
            new = S.two_grid_block_2d(R, h, k1 * math.pi / (n + 1), k2 * math.pi / (n + 1), nu1, nu2) @ \
                np.concatenate(coef)
            want = sum(np.einsum("ij,m->ijm", fld, new[q * M:(q + 1) * M]) for q, fld in enumerate(parts))
            assert np.max(np.abs(out - want)) <= 1e-10 * scale, (k1, k2)
        # one index (n + 1)/2: the smoother alone
        kh = (n + 1) // 2
        for s in (np.sin(kh * math.pi * i / (n + 1)) * np.sin(k1 * math.pi * j / (n + 1)),
                  np.sin(k1 * math.pi * i / (n + 1)) * np.sin(kh * math.pi * j / (n + 1))):
            parts = [np.where(red, s, 0.0), np.where(~red, s, 0.0)]
            coef = [rng.standard_normal(M) for _ in range(2)]
            out = apply(zip(parts, coef))
            new = S.smoother_block_2d(R, h, k1 * math.pi / (n + 1), nu1 + nu2) @ np.concatenate(coef)
            want = sum(np.einsum("ij,m->ijm", fld, new[q * M:(q + 1) * M]) for q, fld in enumerate(parts))
            assert np.max(np.abs(out - want)) <= 1e-10 * scale, k1


def test_2d_no_time_term_is_the_red_black_poisson_factor():
    """R = 0 leaves the 2D Poisson problem, whose two-grid factor with one
    red-black smoothing step, full weighting and bilinear interpolation tends
    to 1/4 as h -> 0 (and stays below it)."""
    vals = [S.two_grid_factor_2d(2 ** l - 1, 3, 0.5, 1.0, R=np.zeros((3, 3))) for l in (4, 6, 8)]
    assert all(v < 0.25 for v in vals) and vals[-1] > 0.249 and vals[0] < vals[1] < vals[2], vals
