"""Oracle: H-matrix representation R~ of the L1 matrix (Section 3), plain numpy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 3 passages followed
---------------------------
* Definition 3.1 (admissibility): row block rows m1..m2 has I_t = [t_{m1}, t_{m2}]
  (supports of the Dirac tests), column block j1..j2 has
  I_s = [t_{j1-1}, t_{j2+1}] (supports of the hats); the block is admissible
  iff t_{j2+1} < t_{m1} and t_{m2} - t_{m1} <= t_{m1} - t_{j2+1}.
* Construction (Figure 2 and the text around it): start from the whole matrix,
  split 2x2 recursively; blocks strictly above the diagonal are zero,
  admissible blocks are stored in low-rank form, the others are split again
  until they are small, where they are kept full.
* Truncated Taylor expansion of (t - s)^{-alpha} in t about the midpoint t_c of
  I_t with k terms, giving the rank-k factors
  A_{m,nu} = (t_m - t_c)^nu / Gamma(1 - alpha)                (equation A_elements)
  B_{j,nu} = c_nu/(1-alpha-nu) [ (mu_{j-1} - mu_j)/dt_j - (mu_j - mu_{j+1})/dt_{j+1} ],
  mu_i = (t_c - t_i)^{1-alpha-nu}, c_nu = prod_{l=1}^{nu} (1-alpha-l) / nu!
                                                              (equation B_elements)
  where each divided difference is divided by the length of the interval it
  spans.

Readings where the paper leaves a choice:
* cluster tree: index bisection, a cluster of size s > leaf has children of
  sizes s//2 and s - s//2; leaves have size <= leaf (16 by default);
* the block recursion pairs clusters of the same depth; if exactly one of the
  two clusters is a leaf, only the other one is split.

Variants the remark after Definition 3.1 leaves open (off by default, so the
plain construction above is unchanged):
* admissibility with a parameter eta > 0: diam(I_t) <= eta dist(I_s, I_t)
  (still with d < a); eta = 1 is Definition 3.1;
* geometric cluster tree: a cluster of the levels t_{lo+1}..t_hi splits
  after the last level that does not exceed the midpoint of its time
  interval, each child keeping at least one level.
"""
from __future__ import annotations

import math

import numpy as np

from .l1 import l1_matrix, pow_diff, steps


class Cluster:
    __slots__ = ("lo", "hi", "children")

    def __init__(self, lo, hi):
        self.lo, self.hi, self.children = lo, hi, []

    @property
    def size(self):
        return self.hi - self.lo

    def is_leaf(self):
        return not self.children


def cluster_tree(lo: int, hi: int, leaf: int, rule: str = "index", t: np.ndarray | None = None) -> Cluster:
    """0-based index range [lo, hi) of the time levels t_{lo+1}..t_{hi}.
    rule "index": halve the index range; "geometric": halve the time
    interval [t_{lo+1}, t_hi] (needs the mesh t)."""
    c = Cluster(lo, hi)
    if hi - lo > leaf:
        if rule == "index":
            mid = lo + (hi - lo) // 2
        elif rule == "geometric":
            tm = 0.5 * (t[lo + 1] + t[hi])
            count = int(np.sum(t[lo + 1:hi + 1] <= tm))      # levels at or before the midpoint
            mid = min(max(lo + count, lo + 1), hi - 1)
        else:
            raise ValueError(rule)
        c.children = [cluster_tree(lo, mid, leaf, rule, t), cluster_tree(mid, hi, leaf, rule, t)]
    return c


def admissible(t: np.ndarray, rows: Cluster, cols: Cluster, eta: float = 1.0) -> bool:
    M = len(t) - 1
    m1, m2 = rows.lo + 1, rows.hi          # 1-based rows
    j2 = cols.hi                            # 1-based last column
    if j2 + 1 > M:
        return False
    a, d = t[m1], t[j2 + 1]
    return d < a and (t[m2] - t[m1]) <= eta * (a - d)


def block_partition(t: np.ndarray, leaf: int = 16, eta: float = 1.0, cluster: str = "index"):
    """List of (kind, rows, cols) with kind in {'rk', 'full'}; zero blocks are omitted."""
    M = len(t) - 1
    root = cluster_tree(0, M, leaf, cluster, t)
    out = []

    def rec(r: Cluster, c: Cluster):
        if c.lo >= r.hi:                   # columns entirely after the rows: zero block
            return
        if admissible(t, r, c, eta):
            out.append(("rk", r, c))
            return
        if r.is_leaf() and c.is_leaf():
            out.append(("full", r, c))
            return
        rs = [r] if r.is_leaf() else r.children
        cs = [c] if c.is_leaf() else c.children
        for rr in rs:
            for cc in cs:
                rec(rr, cc)

    rec(root, root)
    return out


def taylor_coeffs(alpha: float, k: int) -> np.ndarray:
    """c_nu = prod_{l=1}^{nu} (1 - alpha - l) / nu!, nu = 0..k-1."""
    c = np.empty(k)
    c[0] = 1.0
    for nu in range(1, k):
        c[nu] = c[nu - 1] * (1.0 - alpha - nu) / nu
    return c


def rk_factors(t: np.ndarray, alpha: float, k: int, rows: Cluster, cols: Cluster):
    """A (|rows| x k) and B (|cols| x k) with R~ = A B^T on the block."""
    dt = steps(t)
    m = np.arange(rows.lo + 1, rows.hi + 1)          # 1-based rows
    j = np.arange(cols.lo + 1, cols.hi + 1)          # 1-based columns
    tc = 0.5 * (t[rows.lo + 1] + t[rows.hi])
    cnu = taylor_coeffs(alpha, k)
    A = np.empty((len(m), k))
    B = np.empty((len(j), k))
    ginv = 1.0 / math.gamma(1.0 - alpha)
    for nu in range(k):
        A[:, nu] = (t[m] - tc) ** nu * ginv
        q = 1.0 - alpha - nu
        # mu_{j-1} - mu_j = (tc - t_j + dt_j)^q - (tc - t_j)^q
        left = pow_diff(tc - t[j], dt[j], q) / dt[j]
        # mu_j - mu_{j+1} = (tc - t_{j+1} + dt_{j+1})^q - (tc - t_{j+1})^q
        right = pow_diff(tc - t[j + 1], dt[j + 1], q) / dt[j + 1]
        B[:, nu] = cnu[nu] / q * (left - right)
    return A, B


def hmatrix_dense(t: np.ndarray, alpha: float, k: int, leaf: int = 16, R: np.ndarray | None = None,
                  eta: float = 1.0, cluster: str = "index"):
    """R~ expanded to a dense M x M array: full blocks copy R, admissible blocks are A B^T."""
    if R is None:
        R = l1_matrix(t, alpha)
    Rt = np.zeros_like(R)
    for kind, r, c in block_partition(t, leaf, eta, cluster):
        if kind == "full":
            Rt[r.lo:r.hi, c.lo:c.hi] = R[r.lo:r.hi, c.lo:c.hi]
        else:
            A, B = rk_factors(t, alpha, k, r, c)
            Rt[r.lo:r.hi, c.lo:c.hi] = A @ B.T
    return Rt


def theorem_bound(t: np.ndarray, alpha: float, k: int, rows: Cluster, cols: Cluster) -> np.ndarray:
    """Entrywise error bound from the proof of Theorem 3.1 on an admissible block:
    (dt_j + dt_{j+1}) / (2 Gamma(1-alpha) rho^{1+alpha}) * q^k (alpha/(1-q) + k/(1-q) + q/(1-q)^2),
    rho = |a - t_c| + |a - d|, q = |a - t_c| / rho, I_t = [a, b], I_s = [c, d]."""
    dt = steps(t)
    a = t[rows.lo + 1]
    b = t[rows.hi]
    d = t[cols.hi + 1]
    tc = 0.5 * (a + b)
    rho = abs(a - tc) + abs(a - d)
    q = abs(a - tc) / rho
    s = q ** k * (alpha / (1 - q) + k / (1 - q) + q / (1 - q) ** 2)
    j = np.arange(cols.lo + 1, cols.hi + 1)
    colfac = (dt[j] + dt[j + 1]) / (2.0 * math.gamma(1.0 - alpha) * rho ** (1.0 + alpha)) * s
    return np.broadcast_to(colfac[None, :], (rows.size, cols.size))
