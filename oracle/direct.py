"""Oracle: the fully discrete system and its direct solution, plain numpy/scipy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The system (Section 2 discrete problem; Section 3 last paragraph; Algorithm 2
applied to A_{h,tau}): for every interior point q and time level m = 1..M

    sum_j Rt_{m,j} u_{q,j} + (A_h u_{.,m})_q = f_{q,m} + a_{m,1} g_q

with A_h the 3-point (1D) or 5-point (2D) negative Laplacian / h^2 with
homogeneous Dirichlet values.  Grid functions are arrays [M][N], row m-1 holds
level t_m.

Because Rt is lower triangular, the plain solution marches in time: at level m
solve (Rt_{m,m} I + A_h) u_m = b_m - sum_{j<m} Rt_{m,j} u_j.  In 1D the
tridiagonal system is solved with a banded solver; in 2D the shifted Laplacian
is diagonalised by the orthonormal type-I sine transform in each direction.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft
import scipy.linalg

from .l1 import initial_value_weights


def laplacian_apply(U: np.ndarray, dim: int, n: int, h: float) -> np.ndarray:
    """(A_h U) for every row of U ([M][N]); Dirichlet zero outside."""
    M = U.shape[0]
    if dim == 1:
        P = np.zeros((M, n + 2))
        P[:, 1:-1] = U
        return (2.0 * P[:, 1:-1] - P[:, :-2] - P[:, 2:]) / (h * h)
    V = U.reshape(M, n, n)
    P = np.zeros((M, n + 2, n + 2))
    P[:, 1:-1, 1:-1] = V
    out = (4.0 * P[:, 1:-1, 1:-1] - P[:, :-2, 1:-1] - P[:, 2:, 1:-1]
           - P[:, 1:-1, :-2] - P[:, 1:-1, 2:]) / (h * h)
    return out.reshape(M, n * n)


def laplacian_dense(dim: int, n: int, h: float) -> np.ndarray:
    T = (np.diag(np.full(n, 2.0)) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)) / (h * h)
    if dim == 1:
        return T
    I = np.eye(n)
    return np.kron(I, T) + np.kron(T, I)


def laplacian_eigs(n: int, h: float, length: float) -> np.ndarray:
    """Eigenvalues (4/h^2) sin^2(p pi h / (2 length)), p = 1..n, of the 1D operator."""
    p = np.arange(1, n + 1)
    return 4.0 / (h * h) * np.sin(p * math.pi * h / (2.0 * length)) ** 2


def rhs(F: np.ndarray, t: np.ndarray, alpha: float, g: np.ndarray | None) -> np.ndarray:
    """b = f + a_{.,1} g (initial value moved to the right-hand side)."""
    if g is None:
        return np.array(F, dtype=np.float64, copy=True)
    return F + np.outer(initial_value_weights(t, alpha), g)


def solve_shifted_spatial(shift: float, b: np.ndarray, dim: int, n: int, h: float,
                          length: float) -> np.ndarray:
    """Solve (shift I + A_h) u = b for one time level b [N]."""
    if dim == 1:
        ab = np.empty((3, n))
        ab[0, :] = -1.0 / (h * h)
        ab[1, :] = shift + 2.0 / (h * h)
        ab[2, :] = -1.0 / (h * h)
        return scipy.linalg.solve_banded((1, 1), ab, b)
    lam = laplacian_eigs(n, h, length)
    B = b.reshape(n, n)
    Bh = scipy.fft.dstn(B, type=1, norm="ortho")
    Uh = Bh / (shift + lam[:, None] + lam[None, :])
    return scipy.fft.idstn(Uh, type=1, norm="ortho").reshape(-1)


def timestep_solve(Rt: np.ndarray, B: np.ndarray, dim: int, n: int, length: float,
                   m_stop: int | None = None) -> np.ndarray:
    """Direct solution of sum_j Rt_{m,j} u_j + A_h u_m = b_m, m = 1..M (or the
    first m_stop levels)."""
    M = Rt.shape[0] if m_stop is None else m_stop
    h = length / (n + 1)
    U = np.zeros((M, B.shape[1]))
    for m in range(M):
        hist = Rt[m, :m] @ U[:m] if m > 0 else 0.0
        U[m] = solve_shifted_spatial(Rt[m, m], B[m] - hist, dim, n, h, length)
    return U


def residual(Rt: np.ndarray, U: np.ndarray, B: np.ndarray, dim: int, n: int, length: float) -> np.ndarray:
    """r = b - (Rt (x) I) u - (I (x) A_h) u."""
    h = length / (n + 1)
    return B - Rt @ U - laplacian_apply(U, dim, n, h)


def residual_columns(Rt: np.ndarray, U: np.ndarray, B: np.ndarray, dim: int, n: int,
                     length: float, cols: np.ndarray) -> np.ndarray:
    """Residual restricted to the spatial points `cols` (flat indices)."""
    h = length / (n + 1)
    cols = np.asarray(cols)
    out = B[:, cols] - Rt @ U[:, cols]
    if dim == 1:
        nb = [cols - 1, cols + 1]
        valid = [cols - 1 >= 0, cols + 1 < n]
    else:
        ix, iy = cols % n, cols // n
        nb = [cols - 1, cols + 1, cols - n, cols + n]
        valid = [ix > 0, ix < n - 1, iy > 0, iy < n - 1]
    lap = 2.0 * dim * U[:, cols]
    for q, ok in zip(nb, valid):
        qq = np.where(ok, q, 0)
        lap = lap - np.where(ok[None, :], U[:, qq], 0.0)
    return out - lap / (h * h)


def residual_sampled(Rt: np.ndarray, b_cols: np.ndarray, u_cols: np.ndarray, u_nbrs, h: float) -> np.ndarray:
    """Residual at a few spatial points from their time lines alone:
    r = b - Rt u - (2 dim u - sum of the 2 dim neighbour lines) / h^2, with
    u_nbrs the neighbour lines [M][len(cols)] (zero where a neighbour is a
    Dirichlet boundary point); for arrays too large to hold on the host."""
    dim = len(u_nbrs) // 2
    lap = 2.0 * dim * u_cols
    for v in u_nbrs:
        lap = lap - v
    return b_cols - Rt @ u_cols - lap / (h * h)


def single_mode_profile(Rt: np.ndarray, lam: float, phi: np.ndarray) -> np.ndarray:
    """If b = phi(t) s with A_h s = lam s, then u = w(t) s with (Rt + lam I) w = phi."""
    M = Rt.shape[0]
    return scipy.linalg.solve_triangular(Rt + lam * np.eye(M), phi, lower=True)


def mode_eigenvalue(kvec, n: int, length: float) -> float:
    """Eigenvalue of A_h for the sine mode with wave numbers kvec."""
    h = length / (n + 1)
    return float(sum(4.0 / (h * h) * math.sin(kk * math.pi * h / (2.0 * length)) ** 2 for kk in kvec))


def kron_solve(Rt: np.ndarray, B: np.ndarray, dim: int, n: int, length: float) -> np.ndarray:
    """Dense LU solve of (Rt (x) I_N + I_M (x) A_h) vec(U) = vec(B) (time-major
    vec); for tiny grids only."""
    h = length / (n + 1)
    M = Rt.shape[0]
    N = B.shape[1]
    A = np.kron(Rt, np.eye(N)) + np.kron(np.eye(M), laplacian_dense(dim, n, h))
    lu = scipy.linalg.lu_factor(A)
    return scipy.linalg.lu_solve(lu, B.reshape(-1)).reshape(M, N)
