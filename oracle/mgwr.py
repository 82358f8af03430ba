"""Oracle: the multigrid waveform relaxation cycle itself, plain numpy/scipy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The rest of the oracle defines the result the cycles converge to (the direct
solution of the discrete system).  This module takes the steps of one cycle
(Algorithm 2, Section 4) in the paper's order, so that the iterate after a
fixed number of cycles can be compared as well:

* zebra-in-time line relaxation S: red-black order in space (the first colour
  is the set of coarse-grid points: 1-based even points in 1D, (i + j) even
  in 2D); each half-sweep solves, for every point q of its colour, the lower
  triangular system (Rt + (2 dim/h^2) I) u_q = b_q + (1/h^2) sum of the
  neighbour lines (those of the other colour; Dirichlet values are zero);
* the defect f - A u of the whole space-time system;
* full-weighting restriction in space only ((1/4)[1 2 1] per direction,
  coarse point p on fine point 2p + 1, 0-based);
* gamma cycles on the coarse grid (n_c = (n - 1)/2 points per direction, the
  same domain, so h_c = 2h, and the same time matrix Rt), from zero;
* linear (bilinear) interpolation of the correction in space only;
* nu2 post-smoothing steps;
* on the coarsest grid, the direct solve of the whole system there.

Pins (tests/test_oracle_mgwr.py): with a zero right-hand side the cycle maps
the error, and on a two-grid hierarchy it must act on each sine-mode pair
(quadruple in 2D) exactly as the blocks of the semi-algebraic mode analysis
(oracle/sama.py, itself pinned to Table 2's printed factors); the direct
solution is a fixed point of the cycle; cycles converge to it.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .direct import laplacian_apply, timestep_solve


def _first_colour(dim: int, n: int) -> np.ndarray:
    """Flat indices of the first colour (the coarse-grid points' colour)."""
    q = np.arange(n ** dim)
    if dim == 1:
        return q[q % 2 == 1]                 # 1-based even points
    y, x = np.divmod(q, n)
    return q[(x + y) % 2 == 0]               # (i + j) even, 1-based


def _second_colour(dim: int, n: int) -> np.ndarray:
    """Flat indices of the second colour."""
    q = np.arange(n ** dim)
    if dim == 1:
        return q[q % 2 == 0]                 # 1-based odd points
    y, x = np.divmod(q, n)
    return q[(x + y) % 2 == 1]


def half_sweep(Rt: np.ndarray, U: np.ndarray, B: np.ndarray, dim: int, n: int, length: float,
               points: np.ndarray) -> None:
    """Zebra-in-time line relaxation of the lines `points` (one colour; no two
    of them are neighbours), in place."""
    h = length / (n + 1)
    diag = 2.0 * dim / (h * h)
    # (1/h^2) sum of neighbour lines = diag u - A_h u
    nb = diag * U - laplacian_apply(U, dim, n, h)
    D = Rt + diag * np.eye(Rt.shape[0])
    U[:, points] = scipy.linalg.solve_triangular(D, B[:, points] + nb[:, points], lower=True)


def smooth(Rt, U, B, dim, n, length) -> None:
    """One red-black step S: the first colour, then the second."""
    half_sweep(Rt, U, B, dim, n, length, _first_colour(dim, n))
    half_sweep(Rt, U, B, dim, n, length, _second_colour(dim, n))


def _restrict_axis(a: np.ndarray, axis: int) -> np.ndarray:
    """(1/4)[1 2 1] along `axis` (length n = 2 nc + 1) onto the nc coarse points."""
    a = np.moveaxis(a, axis, -1)
    out = 0.25 * (a[..., 0:-2:2] + 2.0 * a[..., 1:-1:2] + a[..., 2::2])
    return np.moveaxis(out, -1, axis)


def _prolong_axis(e: np.ndarray, axis: int) -> np.ndarray:
    """Linear interpolation along `axis` from nc coarse points to n = 2 nc + 1
    fine points (zero Dirichlet values beyond both ends)."""
    e = np.moveaxis(e, axis, -1)
    nc = e.shape[-1]
    pad = np.zeros(e.shape[:-1] + (nc + 2,))
    pad[..., 1:-1] = e
    out = np.zeros(e.shape[:-1] + (2 * nc + 1,))
    out[..., 1::2] = e                                   # fine 2p + 1 is coarse p
    out[..., 0::2] = 0.5 * (pad[..., :-1] + pad[..., 1:])  # fine 2p between coarse p - 1 and p
    return np.moveaxis(out, -1, axis)


def restrict(R: np.ndarray, dim: int, n: int) -> np.ndarray:
    """Full weighting in space of a grid function [M][n^dim]."""
    M = R.shape[0]
    if dim == 1:
        return _restrict_axis(R, 1)
    G = R.reshape(M, n, n)
    return _restrict_axis(_restrict_axis(G, 1), 2).reshape(M, -1)


def prolong(E: np.ndarray, dim: int, nc: int) -> np.ndarray:
    """Linear (bilinear) interpolation in space of a coarse grid function."""
    M = E.shape[0]
    if dim == 1:
        return _prolong_axis(E, 1)
    G = E.reshape(M, nc, nc)
    return _prolong_axis(_prolong_axis(G, 1), 2).reshape(M, -1)


def cycle(Rt: np.ndarray, U: np.ndarray, B: np.ndarray, dim: int, n: int, length: float,
          nu1: int = 1, nu2: int = 1, gamma: int = 1, coarsest: int = 1) -> np.ndarray:
    """One cycle of Algorithm 2 on the grid with n points per direction; the
    grids with at most `coarsest` points per direction are solved directly.
    Returns the new iterate (U is not modified)."""
    if n <= coarsest:
        return timestep_solve(Rt, B, dim, n, length)
    U = np.array(U, dtype=np.float64, copy=True)
    for _ in range(nu1):
        smooth(Rt, U, B, dim, n, length)
    h = length / (n + 1)
    r = B - Rt @ U - laplacian_apply(U, dim, n, h)
    nc = (n - 1) // 2
    rc = restrict(r, dim, n)
    E = np.zeros_like(rc)
    for _ in range(gamma):
        E = cycle(Rt, E, rc, dim, nc, length, nu1, nu2, gamma, coarsest)
    U += prolong(E, dim, nc)
    for _ in range(nu2):
        smooth(Rt, U, B, dim, n, length)
    return U


def cycles(Rt, B, dim, n, length, count: int, U0=None, **kw) -> list:
    """The iterates after 1..count cycles from U0 (zero by default)."""
    U = np.zeros_like(B) if U0 is None else np.array(U0, dtype=np.float64, copy=True)
    out = []
    for _ in range(count):
        U = cycle(Rt, U, B, dim, n, length, **kw)
        out.append(U)
    return out
