"""The identity behind the library's zebra defects, on the CPU.

After a zebra sweep (each line of the first colour solved with the time
operator R~ + (2 dim / h^2) I against the second colour's values, then each
line of the second colour), the defect b - A u is zero on the second colour
and, at a first-colour point, 1/h^2 times the sum over its neighbours of the
changes d that the second-colour half-sweep made.  The full-weighting
restriction of that defect (first-colour taps only: the coarse point and, in
2D, its diagonal neighbours) can therefore be formed from d alone; the
kernels use two equivalent forms of it (five defects from their four
neighbours each, and twelve taps on d with weights 6/16 and 1/16), both
checked here against the defect of the oracle's residual.  The line solves
are dense numpy solves here, so the identity holds to rounding.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def _grid_neighbours(q, dim, n):
    if dim == 1:
        return [p for p in (q - 1, q + 1) if 0 <= p < n]
    y, x = divmod(q, n)
    out = []
    if y >= 1:
        out.append(q - n)
    if y + 1 < n:
        out.append(q + n)
    if x >= 1:
        out.append(q - 1)
    if x + 1 < n:
        out.append(q + 1)
    return out


def _zebra_sweep(Rt, B, U, dim, n, h):
    """One zebra sweep (first colour, then second) with exact line solves;
    returns the changes of the second-colour half-sweep."""
    N = n ** dim
    first = 1 if dim == 1 else 0   # 1D: odd flat indices (the coarse points); 2D: even (x + y even)
    D = Rt + (2 * dim / h ** 2) * np.eye(Rt.shape[0])
    d = np.zeros_like(U)
    for colour in (first, 1 - first):
        old = U.copy()
        for q in range(N):
            if q % 2 != colour:
                continue
            rhs = B[:, q] + sum(U[:, p] for p in _grid_neighbours(q, dim, n)) / h ** 2
            U[:, q] = np.linalg.solve(D, rhs)
        if colour == 1 - first:
            d = U - old
    return d


@pytest.mark.parametrize("dim,n,M,alpha", [(1, 15, 48, 0.5), (1, 31, 32, 0.3), (2, 7, 40, 0.5), (2, 15, 32, 0.7)])
def test_zebra_defect_identity_and_restrictions(dim, n, M, alpha):
    rng = np.random.default_rng(11 + 7 * dim + n)
    t = W.graded_mesh(M, 1.0, (2 - alpha) / alpha)
    Rt = oracle.hmatrix_dense(t, alpha, 8, 16)
    N = n ** dim
    h = 1.0 / (n + 1)
    B = rng.standard_normal((M, N))
    U = rng.standard_normal((M, N))
    d = _zebra_sweep(Rt, B, U, dim, n, h)
    r = oracle.residual(Rt, U, B, dim, n, 1.0)
    scale = np.max(np.abs(B)) + np.max(np.abs(U)) / h ** 2
    first = 1 if dim == 1 else 0
    ih2 = 1.0 / h ** 2
    for q in range(N):
        want = ih2 * sum(d[:, p] for p in _grid_neighbours(q, dim, n)) if q % 2 == first else 0.0
        assert np.max(np.abs(r[:, q] - want)) <= 1e-11 * scale, q

    nc = (n - 1) // 2
    if dim == 1:
        for p in range(nc):
            direct = 0.25 * (r[:, 2 * p] + 2 * r[:, 2 * p + 1] + r[:, 2 * p + 2])   # full weighting
            zebra = 0.5 * ih2 * (d[:, 2 * p] + d[:, 2 * p + 2])
            assert np.max(np.abs(direct - zebra)) <= 1e-11 * scale, p
        return

    def D(y, x):
        return d[:, y * n + x] if (0 <= y < n and 0 <= x < n) else 0.0

    def R(y, x):
        return r[:, y * n + x] if (0 <= y < n and 0 <= x < n) else 0.0

    taps12 = [(-1, 0), (1, 0), (0, -1), (0, 1), (-2, -1), (-2, 1), (2, -1), (2, 1), (-1, -2), (1, -2), (-1, 2), (1, 2)]
    for J in range(nc):
        for I in range(nc):
            y, x = 2 * J + 1, 2 * I + 1
            direct = sum((2 if dy == 0 else 1) * (2 if dx == 0 else 1) / 16.0 * R(y + dy, x + dx)
                         for dy in (-1, 0, 1) for dx in (-1, 0, 1))
            def rz(yy, xx):
                return ih2 * (D(yy - 1, xx) + D(yy + 1, xx) + D(yy, xx - 1) + D(yy, xx + 1))
            five = (rz(y - 1, x - 1) + rz(y - 1, x + 1) + rz(y + 1, x - 1) + rz(y + 1, x + 1) + 4 * rz(y, x)) / 16.0
            twelve = sum(((6.0 if k < 4 else 1.0) / 16.0) * ih2 * D(y + dy, x + dx)
                         for k, (dy, dx) in enumerate(taps12))
            assert np.max(np.abs(direct - five)) <= 1e-11 * scale, (J, I)
            assert np.max(np.abs(direct - twelve)) <= 1e-11 * scale, (J, I)


def test_zebra_identity_fails_without_the_exact_first_colour_solve():
    """The identity needs the first colour solved against the values the
    second colour had before its half-sweep: perturbing one first-colour
    line after the sweep breaks it at that line (a planted mistake)."""
    dim, n, M, alpha = 1, 15, 32, 0.5
    rng = np.random.default_rng(5)
    t = W.graded_mesh(M, 1.0, 3.0)
    Rt = oracle.hmatrix_dense(t, alpha, 8, 16)
    h = 1.0 / (n + 1)
    B = rng.standard_normal((M, n))
    U = rng.standard_normal((M, n))
    d = _zebra_sweep(Rt, B, U, dim, n, h)
    U[:, 7] += 1e-3   # flat index 7 is a first-colour point in 1D
    r = oracle.residual(Rt, U, B, dim, n, 1.0)
    want = (d[:, 6] + d[:, 8]) / h ** 2
    assert np.max(np.abs(r[:, 7] - want)) > 1e-6
