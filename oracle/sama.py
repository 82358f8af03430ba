"""Semi-algebraic mode analysis (SAMA) of the two-grid method of Algorithm 2
in one space dimension: Fourier (sine) modes in space, the exact time matrix
in time.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The method analysed (Section 4, Algorithm 2, one space dimension): zebra line
relaxation in red-black order (first the even points, 1-based, which are the
coarse-grid points; each half-sweep solves (R + (2/h^2) I) u_i = b_i +
(u_{i-1} + u_{i+1})/h^2 for every line of its colour), full-weighting
restriction (1/4)[1 2 1], linear interpolation, and an exact solve with the
rediscretised operator R + A_{2h} on the coarse grid.  Section 5 applies the
analysis to the exact L1 matrix R (not to its H-matrix representation).

Derivation.  With homogeneous Dirichlet values on n = 2^l - 1 interior points
the sine modes s_k(i) = sin(k pi i/(n+1)) diagonalise A_h, and the mode k and
its complement k' = n + 1 - k agree on the odd points and differ in sign on
the even ones.  Writing a grid function of span{s_k, s_k'} as e_R a(t) +
e_B b(t), e_R / e_B the part of s_k on the even / odd points, and
c = cos(k pi/(n+1)), D = R + (2/h^2) I, gamma = 2c/h^2:
  A_k = [[D, -gamma I], [-gamma I, D]]       (the 3-point stencil couples
                                              the two colours through
                                              s_k(i-1) + s_k(i+1) = 2c s_k(i));
  smoothing step (red, then black):
      a' = gamma D^{-1} b,  b' = gamma D^{-1} a';
  restriction: (rho_R, rho_B) -> (rho_R + c rho_B)/2 (coefficient of the
      coarse mode s_k(2j));
  coarse operator: R + (sin^2(k pi/(n+1))/h^2) I (the coarse mode's
      eigenvalue of A_{2h});
  interpolation: e -> (e, c e).
The two-grid error propagation S^nu2 (I - P A_c^{-1} Rfw A_k) S^nu1 acts on
each 2M-dimensional block independently; the mode k = (n+1)/2 (c = 0) is
removed by one smoothing step.  With Dirichlet sine modes this block
decomposition is exact.

Exact evaluation in time.  R is lower triangular (Section 2), and so are D,
A_c and their inverses: every block is block lower triangular in time with
2 x 2 diagonal blocks, the same formulas with R replaced by the scalar
R_{m,m}.  Its spectrum is therefore the union of those 2 x 2 spectra, and the
two-grid factor is their largest modulus over the frequencies and the time
levels.  (Computing the eigenvalues of the full, strongly non-normal blocks
instead loses digits.)
"""
from __future__ import annotations

import math

import numpy as np

from .l1 import l1_matrix


def two_grid_block(R: np.ndarray, h: float, theta: float, nu1: int = 1, nu2: int = 0) -> np.ndarray:
    """2M x 2M two-grid error propagation on the harmonic pair of frequency
    theta = k pi/(n+1), k = 1..(n-1)/2."""
    M = R.shape[0]
    I = np.eye(M)
    c = math.cos(theta)
    D = R + (2.0 / (h * h)) * I
    Dinv = np.linalg.inv(D)
    gamma = 2.0 * c / (h * h)
    A = np.block([[D, -gamma * I], [-gamma * I, D]])
    S = np.block([[np.zeros((M, M)), gamma * Dinv], [np.zeros((M, M)), gamma * gamma * Dinv @ Dinv]])
    Rfw = np.hstack([0.5 * I, 0.5 * c * I])
    P = np.vstack([I, c * I])
    Ac = R + (math.sin(theta) ** 2 / (h * h)) * I
    K = np.eye(2 * M) - P @ np.linalg.solve(Ac, Rfw @ A)
    T = K
    for _ in range(nu1):
        T = T @ S
    for _ in range(nu2):
        T = S @ T
    return T


def spectral_radius(T: np.ndarray) -> float:
    return float(np.max(np.abs(np.linalg.eigvals(T))))


def two_grid_factor(n: int, M: int, alpha: float, r: float, length: float = math.pi, T: float = 1.0,
                    nu1: int = 1, nu2: int = 0, R: np.ndarray | None = None) -> float:
    """SAMA two-grid convergence factor on the graded mesh t_j = T (j/M)^r:
    the largest spectral radius over the frequencies k = 1..(n-1)/2 (the mode
    k = (n+1)/2 is removed by a smoothing step) and the time levels m of the
    2 x 2 diagonal blocks (R_{m,m} in place of R)."""
    if R is None:
        t = T * (np.arange(M + 1) / M) ** r
        t[-1] = T
        R = l1_matrix(t, alpha)
    h = length / (n + 1)
    rho = 0.0
    for sigma in np.unique(np.diag(R)):
        Rm = np.array([[sigma]])
        for k in range(1, (n - 1) // 2 + 1):
            rho = max(rho, spectral_radius(two_grid_block(Rm, h, k * math.pi / (n + 1), nu1, nu2)))
    return rho


# ---- two space dimensions ------------------------------------------------------
#
# Section 5.2's method on n x n points: checkerboard zebra relaxation ((i + j)
# even, 1-based, first: the coarse points (both indices even) are among
# them), 9-point full weighting, bilinear interpolation, R + A_{2h} on the
# coarse grid.  For a frequency pair k1, k2 <= (n-1)/2 with
# s(i, j) = sin(k1 pi i/(n+1)) sin(k2 pi j/(n+1)), the four harmonics
# (k1 or n+1-k1, k2 or n+1-k2) span the same space as the red and black
# parts of e = s and of f = (-1)^(i+1) s.  With c_d = cos(k_d pi/(n+1)),
# D = R + (4/h^2) I, gamma_e = 2 (c1 + c2)/h^2, gamma_f = 2 (c2 - c1)/h^2
# (the 5-point stencil sums the neighbours of s to 2 (c1 + c2) s and those of
# f to 2 (c2 - c1) f, each neighbour lying in the other colour):
#   A = diag([[D, -g_e I], [-g_e I, D]], [[D, -g_f I], [-g_f I, D]]) on
#       (a, b, p, q) = coefficients of (e_R, e_B, f_R, f_B);
#   smoothing step: a' = g_e D^-1 b, p' = g_f D^-1 q, then b' = g_e D^-1 a',
#       q' = g_f D^-1 p';
#   interpolation: e_c -> e_c ((1 + c1 c2)/2, (c1 + c2)/2, (c1 c2 - 1)/2, (c1 - c2)/2)
#       (coarse points carry e_c s, the other points the bilinear averages
#       c1 e_c s, c2 e_c s, c1 c2 e_c s);
#   restriction: half the transpose of the interpolation (9-point weights
#       (1/16)[1 2 1; 2 4 2; 1 2 1] applied to the four parts);
#   coarse operator: R + ((sin^2(k1 pi/(n+1)) + sin^2(k2 pi/(n+1)))/h^2) I.
# Frequencies with k1 or k2 = (n+1)/2 have no coarse representation (the
# restriction of their residual vanishes): one of them with the other index
# k <= (n-1)/2 spans the red and black parts of s, coupled through
# gamma = 2 cos(k pi/(n+1))/h^2 alone, and only the smoother acts on it; both
# indices (n+1)/2 leave a red-only mode that one half-sweep removes.

def two_grid_block_2d(R: np.ndarray, h: float, theta1: float, theta2: float, nu1: int = 1,
                      nu2: int = 0) -> np.ndarray:
    """4M x 4M two-grid error propagation on the harmonics of (theta1,
    theta2), theta_d = k_d pi/(n+1), k_d = 1..(n-1)/2."""
    M = R.shape[0]
    I = np.eye(M)
    Z = np.zeros((M, M))
    c1, c2 = math.cos(theta1), math.cos(theta2)
    D = R + (4.0 / (h * h)) * I
    Dinv = np.linalg.inv(D)
    ge, gf = 2.0 * (c1 + c2) / (h * h), 2.0 * (c2 - c1) / (h * h)
    A = np.block([[D, -ge * I, Z, Z], [-ge * I, D, Z, Z], [Z, Z, D, -gf * I], [Z, Z, -gf * I, D]])
    S = np.block([[Z, ge * Dinv, Z, Z], [Z, ge * ge * Dinv @ Dinv, Z, Z],
                  [Z, Z, Z, gf * Dinv], [Z, Z, Z, gf * gf * Dinv @ Dinv]])
    w = np.array([(1 + c1 * c2) / 2, (c1 + c2) / 2, (c1 * c2 - 1) / 2, (c1 - c2) / 2])
    P = np.vstack([wi * I for wi in w])
    Rfw = 0.5 * P.T
    Ac = R + ((math.sin(theta1) ** 2 + math.sin(theta2) ** 2) / (h * h)) * I
    K = np.eye(4 * M) - P @ np.linalg.solve(Ac, Rfw @ A)
    T = K
    for _ in range(nu1):
        T = T @ S
    for _ in range(nu2):
        T = S @ T
    return T


def smoother_block_2d(R: np.ndarray, h: float, theta: float, nu: int) -> np.ndarray:
    """2M x 2M error propagation of nu smoothing steps on a frequency with
    one index (n+1)/2 (no coarse-grid correction reaches it)."""
    M = R.shape[0]
    I = np.eye(M)
    Z = np.zeros((M, M))
    D = R + (4.0 / (h * h)) * I
    Dinv = np.linalg.inv(D)
    g = 2.0 * math.cos(theta) / (h * h)
    S = np.block([[Z, g * Dinv], [Z, g * g * Dinv @ Dinv]])
    return np.linalg.matrix_power(S, nu)


def two_grid_factor_2d(n: int, M: int, alpha: float, r: float, length: float = math.pi, T: float = 1.0,
                       nu1: int = 1, nu2: int = 0, R: np.ndarray | None = None) -> float:
    """SAMA two-grid factor in two space dimensions (exact in time through
    the 2 x 2 / 4 x 4 diagonal blocks, as in one dimension)."""
    if R is None:
        t = T * (np.arange(M + 1) / M) ** r
        t[-1] = T
        R = l1_matrix(t, alpha)
    h = length / (n + 1)
    nc = (n - 1) // 2
    th = [k * math.pi / (n + 1) for k in range(1, nc + 1)]
    rho = 0.0
    for sigma in np.unique(np.diag(R)):
        Rm = np.array([[sigma]])
        for t1 in th:
            for t2 in th:
                rho = max(rho, spectral_radius(two_grid_block_2d(Rm, h, t1, t2, nu1, nu2)))
            if nu1 + nu2 >= 1:
                rho = max(rho, spectral_radius(smoother_block_2d(Rm, h, t1, nu1 + nu2)))
    return rho
