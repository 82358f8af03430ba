"""Plant plausible mistakes in the oracle (on the CPU) and check that a pin fails.

Each case monkeypatches one oracle function with a wrong variant and asserts
that at least one pin number leaves its tolerance.
"""
import math

import numpy as np
import pytest

import oracle
import oracle.direct as od
import oracle.hmatrix as oh
import oracle.l1 as ol
import pins


def _b_literal_tau(t, alpha, k, rows, cols):
    """B with the step indices of the printed formula taken literally under
    dt_j = t_j - t_{j-1} (divides the left difference by dt_{j-1})."""
    dt = ol.steps(t)
    j = np.arange(cols.lo + 1, cols.hi + 1)
    m = np.arange(rows.lo + 1, rows.hi + 1)
    tc = 0.5 * (t[rows.lo + 1] + t[rows.hi])
    cnu = oh.taylor_coeffs(alpha, k)
    A = np.empty((len(m), k))
    B = np.empty((len(j), k))
    dprev = np.where(j - 1 >= 1, dt[np.maximum(j - 1, 1)], dt[1])
    for nu in range(k):
        A[:, nu] = (t[m] - tc) ** nu / math.gamma(1 - alpha)
        q = 1 - alpha - nu
        left = ol.pow_diff(tc - t[j], dt[j], q) / dprev
        right = ol.pow_diff(tc - t[j + 1], dt[j + 1], q) / dt[j]
        B[:, nu] = cnu[nu] / q * (left - right)
    return A, B


def _coeff_sign_flip(alpha, k):
    c = np.empty(k)
    c[0] = 1.0
    for nu in range(1, k):
        c[nu] = c[nu - 1] * (1.0 + alpha - nu) / nu
    return c


def _rhs_drop_initial(F, t, alpha, g):
    return np.array(F, dtype=np.float64, copy=True)


def _timestep_history_off_by_one(Rt, B, dim, n, length, m_stop=None):
    M = Rt.shape[0]
    h = length / (n + 1)
    U = np.zeros((M, B.shape[1]))
    for m in range(M):
        hist = Rt[m, :m - 1] @ U[:m - 1] if m > 1 else 0.0
        U[m] = od.solve_shifted_spatial(Rt[m, m], B[m] - hist, dim, n, h, length)
    return U


def _timestep_transposed(Rt, B, dim, n, length, m_stop=None):
    M = Rt.shape[0]
    h = length / (n + 1)
    U = np.zeros((M, B.shape[1]))
    for m in range(M):
        hist = Rt[:m, m] @ U[:m] if m > 0 else 0.0
        U[m] = od.solve_shifted_spatial(Rt[m, m], B[m] - hist, dim, n, h, length)
    return U


def _admissible_column_diameter(t, rows, cols, eta=1.0):
    """Definition 3.1 with the diameter of the column interval I_s instead of I_t."""
    M = len(t) - 1
    m1 = rows.lo + 1
    j1, j2 = cols.lo + 1, cols.hi
    if j2 + 1 > M:
        return False
    a, d = t[m1], t[j2 + 1]
    return d < a and (t[j2 + 1] - t[j1 - 1]) <= (a - d)


def _all_pins():
    vals = {
        "linear": pins.linear_exactness(),
        "rowsum": pins.row_sums(),
        "bound": pins.theorem_bound_violation(M=256, k=6),
        "decay": pins.min_decay_ratio(M=256),
        "kron1": pins.kron_mismatch(1, 7),
        "kron2": pins.kron_mismatch(2, 3),
        "mode1": pins.single_mode_mismatch(1, 31),
        "mode2": pins.single_mode_mismatch(2, 15, kvec=(2, 5)),
    }
    ok = (vals["linear"] < 1e-12 and vals["rowsum"] < 1e-12 and vals["bound"] <= 1.0 and vals["decay"] >= 2.5
          and vals["kron1"] < 1e-12 and vals["kron2"] < 1e-12 and vals["mode1"] < 1e-12
          and vals["mode2"] < 1e-12)
    return ok, vals


def test_unmutated_oracle_passes_all_pins():
    ok, vals = _all_pins()
    assert ok, vals


MUTANTS = [
    ("B literal step indices", oh, "rk_factors", _b_literal_tau),
    ("Taylor coefficient sign", oh, "taylor_coeffs", _coeff_sign_flip),
    ("admissibility on the column diameter", oh, "admissible", _admissible_column_diameter),
    ("history sum off by one", od, "timestep_solve", _timestep_history_off_by_one),
    ("transposed operator in history", od, "timestep_solve", _timestep_transposed),
]


@pytest.mark.parametrize("name,mod,attr,fn", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(monkeypatch, name, mod, attr, fn):
    monkeypatch.setattr(mod, attr, fn)
    # the package namespace re-exports these names
    if hasattr(oracle, attr):
        monkeypatch.setattr(oracle, attr, fn)
    ok, vals = _all_pins()
    assert not ok, (name, vals)


def test_planted_double_gamma_fails_linear_exactness(monkeypatch):
    true = ol.l1_weights
    monkeypatch.setattr(ol, "l1_weights", lambda t, a: true(t, a) / math.gamma(2 - a))
    assert pins.linear_exactness() > 1e-3


def test_planted_dropped_initial_value_fails_table1(monkeypatch):
    monkeypatch.setattr(od, "rhs", _rhs_drop_initial)
    monkeypatch.setattr(oracle, "rhs", _rhs_drop_initial)
    worst, _ = pins.table1_ratio(alphas=(0.4,), Ms=(32,))
    assert worst > 1.0


def test_planted_wrong_mesh_width_fails_single_mode(monkeypatch):
    true = od.solve_shifted_spatial

    def wrong(shift, b, dim, n, h, length):
        return true(shift, b, dim, n, h * 1.01, length)
    monkeypatch.setattr(od, "solve_shifted_spatial", wrong)
    assert pins.single_mode_mismatch(1, 31) > 1e-6


def _admissible_eta_ignored(t, rows, cols, eta=1.0):
    """The general condition with eta dropped (Definition 3.1 always)."""
    M = len(t) - 1
    m1, m2, j2 = rows.lo + 1, rows.hi, cols.hi
    if j2 + 1 > M:
        return False
    a, d = t[m1], t[j2 + 1]
    return d < a and (t[m2] - t[m1]) <= (a - d)


def _admissible_eta_wrong_side(t, rows, cols, eta=1.0):
    """eta multiplying the diameter instead of the distance."""
    M = len(t) - 1
    m1, m2, j2 = rows.lo + 1, rows.hi, cols.hi
    if j2 + 1 > M:
        return False
    a, d = t[m1], t[j2 + 1]
    return d < a and eta * (t[m2] - t[m1]) <= (a - d)


def _eta_pins():
    """eta -> 0 keeps R exactly; eta = 2 reaches beyond eta = 1's ratio 1/3
    while staying within eta / (eta + 2)."""
    t = pins.W.graded_mesh(200, 1.0, 2.5)
    R = oracle.l1_matrix(t, 0.6)
    exact = np.array_equal(oracle.hmatrix_dense(t, 0.6, 6, 16, R=R, eta=1e-12), R)
    qs = []
    for kind, rows, cols in oracle.block_partition(t, 16, 2.0):
        if kind == "rk":
            a, b, d = t[rows.lo + 1], t[rows.hi], t[cols.hi + 1]
            qs.append(0.5 * (b - a) / (0.5 * (b - a) + (a - d)))
    return exact and bool(qs) and 1.0 / 3.0 < max(qs) <= 0.5 * (1 + 1e-12)


def test_unmutated_oracle_passes_eta_pins():
    assert _eta_pins()


@pytest.mark.parametrize("fn", [_admissible_eta_ignored, _admissible_eta_wrong_side])
def test_planted_eta_mistake_fails_a_pin(monkeypatch, fn):
    monkeypatch.setattr(oh, "admissible", fn)
    monkeypatch.setattr(oracle, "admissible", fn)
    assert not _eta_pins()
