"""Pins of the oracle's mesh and L1 matrix against closed forms and the defining integral."""
import math

import mpmath
import numpy as np
import pytest

import oracle
import pins
import workloads as W


def test_sign_pattern_and_triangularity():
    t = W.graded_mesh(96, 1.0, 3.0)
    R = oracle.l1_matrix(t, 0.5)
    assert np.all(np.triu(R, 1) == 0.0)
    assert np.all(np.diag(R) > 0)
    low = R[np.tril_indices(96, -1)]
    assert np.all(low < 0)          # M-matrix sign pattern of the L1 scheme


def test_linear_functions_are_exact():
    for alpha, r in [(0.4, 3.0), (0.2, 9.0), (0.8, 1.0)]:
        assert pins.linear_exactness(64, alpha, r) < 1e-12


def test_row_sums_annihilate_constants():
    assert pins.row_sums() < 1e-12


def test_uniform_mesh_gives_textbook_l1():
    assert pins.uniform_toeplitz() < 1e-13


def _integral_entry(t, alpha, m, j):
    """R_{m,j} by quadrature of (1/Gamma(1-a)) int_0^{t_m} (t_m - s)^{-a} phi_j'(s) ds
    at 30 digits (Section 2, equation for the entries of R)."""
    mpmath.mp.dps = 30
    a = mpmath.mpf(alpha)
    tm = mpmath.mpf(t[m])
    tj0, tj, = mpmath.mpf(t[j - 1]), mpmath.mpf(t[j])
    # integrate over v = t_m - s > 0 so the integrand stays real at the endpoint;
    # the interval touching v = 0 is split geometrically for the singularity
    f = lambda v: v ** (-a)

    def q(lo, hi):
        if lo == 0:
            return mpmath.quad(f, [0, hi * mpmath.mpf("1e-20"), hi * mpmath.mpf("1e-10"), hi])
        return mpmath.quad(f, [lo, hi])
    val = q(tm - tj, tm - tj0) / (tj - tj0)
    if j < m:
        tj1 = mpmath.mpf(t[j + 1])
        val -= q(tm - tj1, tm - tj) / (tj1 - tj)
    return float(val / mpmath.gamma(1 - a))


@pytest.mark.parametrize("alpha,r,M", [(0.5, 3.0, 48), (0.2, 9.0, 40), (0.7, 1.857142857142857, 64)])
def test_entries_match_defining_integral(alpha, r, M):
    t = W.graded_mesh(M, 1.0, r)
    R = oracle.l1_matrix(t, alpha)
    rng = np.random.default_rng(11)
    rows = sorted(set([1, 2, 3, M // 2, M] + list(rng.integers(1, M + 1, 4))))
    worst = 0.0
    for m in rows:
        for j in sorted(set(j for j in (1, 2, m - 1, m, m // 2) if 1 <= j <= m)):
            ref = _integral_entry(t, alpha, m, j)
            worst = max(worst, abs(R[m - 1, j - 1] - ref) / R[m - 1, m - 1])
    assert worst < 1e-13


def test_initial_value_weights():
    t = W.graded_mesh(50, 1.0, 3.0)
    a1 = oracle.initial_value_weights(t, 0.4)
    R = oracle.l1_matrix(t, 0.4)
    # a_{m,1} equals the row sum of R (telescoping of a_{m,j} - a_{m,j+1})
    assert np.max(np.abs(a1 - R.sum(axis=1)) / a1) < 1e-12
    # and equals the L1 weight of the first interval (t_m^{1-a} - (t_m-t_1)^{1-a})/(G(2-a) t_1),
    # evaluated here at 40 digits (in float64 this plain difference cancels for large m)
    mpmath.mp.dps = 40
    t1 = mpmath.mpf(t[1])
    want = np.array([float((mpmath.mpf(tm) ** mpmath.mpf(0.6) - (mpmath.mpf(tm) - t1) ** mpmath.mpf(0.6))
                           / (mpmath.gamma(mpmath.mpf(1.6)) * t1)) for tm in t[1:]])
    assert np.max(np.abs(a1 - want) / want) < 1e-14
