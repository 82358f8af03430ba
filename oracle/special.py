"""Oracle: Mittag-Leffler function for the exact solution of the first
experiment of Section 5.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

E_alpha(z) = sum_{k>=0} z^k / Gamma(alpha k + 1) (Section 5.1).  For z in
[-1, 0] the terms decrease in size after the first few, so the partial sums
are summed until the term drops below 1e-18 of the sum.
"""
from __future__ import annotations

import math

import numpy as np


def mittag_leffler(alpha: float, z) -> np.ndarray:
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    out = np.empty_like(z)
    for i, zi in enumerate(z):
        s = 0.0
        for kk in range(0, 400):
            term = zi ** kk / math.gamma(alpha * kk + 1.0)
            s += term
            if kk > 5 and abs(term) < 1e-18 * max(abs(s), 1e-300):
                break
        out[i] = s
    return out
