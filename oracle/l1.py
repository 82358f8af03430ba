"""Oracle: time mesh and L1 (Petrov-Galerkin) matrix R, plain float64 numpy.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py; never by the product library.

Paper passages followed
-----------------------
* Section 2, graded mesh t_m = T (m/M)^r.
* Section 2, equation (elements_matrix_R): R_{m,j} is the Caputo operator
  applied to the hat function phi_j and tested with the Dirac delta at t_m.
  For j <= m this integral is a_{m,j} - a_{m,j+1} (a_{m,m+1} := 0) with
  a_{m,j} = [(t_m - t_{j-1})^{1-alpha} - (t_m - t_j)^{1-alpha}] / (Gamma(2-alpha) dt_j),
  dt_j = t_j - t_{j-1}; R_{m,j} = 0 for j > m (the d_{m,k} of Section 2 with
  the step of the interval each difference quotient spans).
* The initial value u_0 = g enters the discrete Caputo sum as -a_{m,1} g and is
  moved to the right-hand side (Section 2, discrete problem with u_{n,0} = g).

Floating point: the difference of powers is evaluated as
x^p * expm1(p * log1p(d/x)), which avoids the cancellation of the plain
formula when the step d is small against x (near the origin of a graded mesh).
"""
from __future__ import annotations

import math

import numpy as np


def steps(t: np.ndarray) -> np.ndarray:
    """dt[j] = t_j - t_{j-1} for j = 1..M, returned with dt[0] unused (= nan)."""
    dt = np.empty_like(t)
    dt[0] = np.nan
    dt[1:] = t[1:] - t[:-1]
    return dt


def pow_diff(x, d, p):
    """(x + d)^p - x^p for x >= 0, d > 0 (elementwise)."""
    x = np.asarray(x, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    x, d = np.broadcast_arrays(x, d)
    out = np.empty(x.shape)
    pos = x > 0
    out[pos] = x[pos] ** p * np.expm1(p * np.log1p(d[pos] / x[pos]))
    out[~pos] = d[~pos] ** p
    return out


def l1_weights(t: np.ndarray, alpha: float) -> np.ndarray:
    """a[m-1, j-1] = a_{m,j} for 1 <= j <= m <= M, zero above the diagonal."""
    M = len(t) - 1
    dt = steps(t)
    g2 = math.gamma(2.0 - alpha)
    a = np.zeros((M, M))
    for m in range(1, M + 1):
        j = np.arange(1, m + 1)
        x = t[m] - t[j]                 # t_m - t_j  (>= 0)
        a[m - 1, :m] = pow_diff(x, dt[j], 1.0 - alpha) / (g2 * dt[j])
    return a


def l1_matrix(t: np.ndarray, alpha: float) -> np.ndarray:
    """Dense lower-triangular R (M x M): R_{m,m} = a_{m,m},
    R_{m,j} = a_{m,j} - a_{m,j+1} for j < m."""
    a = l1_weights(t, alpha)
    R = a.copy()
    R[:, :-1] -= a[:, 1:]
    return np.tril(R)


def initial_value_weights(t: np.ndarray, alpha: float) -> np.ndarray:
    """a_{m,1}, m = 1..M: weight with which g enters the right-hand side."""
    g2 = math.gamma(2.0 - alpha)
    t1 = t[1]
    x = t[1:] - t1
    return pow_diff(x, np.full_like(x, t1), 1.0 - alpha) / (g2 * t1)
