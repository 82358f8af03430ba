"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds no arithmetic of the solution method: it only produces the
data of the continuous problem (the time mesh points, source samples f(x, t_m),
initial data g(x), closed-form exact solutions) on which both sides run.

Conventions
-----------
* Time mesh: ``t[0..M]`` with ``t[0] = 0`` and ``t[j] = T (j/M)^r`` (graded
  mesh of Section 2; r = 1 is the uniform mesh).
* Space: ``n`` interior points per side of (0, length)^dim, ``h = length/(n+1)``,
  ``x_i = (i+1) h`` for 0-based ``i``.  A grid function is stored as an array
  ``[M][N]`` with ``N = n**dim``; row ``m`` holds time level ``t[m+1]``; in 2D
  the flat spatial index is ``q = iy*n + ix`` (x fastest).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem",
    "graded_mesh",
    "default_grading",
    "grid_points",
    "sine_mode",
    "manufactured",
    "paper_1d_mittag_leffler",
    "paper_2d_polynomial",
    "random_fourier_2d",
    "batched_instances",
    "warm_start_family",
    "config",
]


def default_grading(alpha: float) -> float:
    """Grading exponent r = (2 - alpha)/alpha (Section 2, choice after the
    graded-mesh accuracy statement)."""
    return (2.0 - alpha) / alpha


def graded_mesh(M: int, T: float = 1.0, r: float = 1.0) -> np.ndarray:
    """t_j = T (j/M)^r, j = 0..M, as float64 (Section 2)."""
    j = np.arange(M + 1, dtype=np.float64)
    t = T * (j / M) ** r
    t[0] = 0.0
    t[M] = T
    return t


def grid_points(n: int, length: float) -> np.ndarray:
    """Interior points x_i = (i+1) h, h = length/(n+1)."""
    h = length / (n + 1)
    return (np.arange(n, dtype=np.float64) + 1.0) * h


def sine_mode(n: int, dim: int, length: float, kvec) -> np.ndarray:
    """Product of sines prod_d sin(k_d pi x_d / length) on the interior grid,
    flattened as [N] (x fastest)."""
    x = grid_points(n, length)
    if dim == 1:
        (kx,) = kvec
        return np.sin(kx * math.pi * x / length)
    kx, ky = kvec
    sx = np.sin(kx * math.pi * x / length)
    sy = np.sin(ky * math.pi * x / length)
    return np.outer(sy, sx).reshape(-1)


@dataclass
class Problem:
    """One synthetic instance of the time-fractional heat equation."""

    dim: int
    n: int
    M: int
    alpha: float
    r: float
    k: int
    length: float = 1.0
    T: float = 1.0
    leaf: int = 16
    t: np.ndarray = None           # [M+1]
    f: np.ndarray = None           # [M][N]
    g: np.ndarray = None           # [N] or None (zero initial data)
    exact: object = None           # callable -> [M][N] continuous solution at nodes, or None
    modes: list = field(default_factory=list)   # [(kvec, time profile [M]), ...] if f is a sum of sine modes
    g_modes: list = field(default_factory=list)  # [(kvec, amplitude)] if g is a sum of sine modes
    name: str = ""

    @property
    def N(self) -> int:
        return self.n ** self.dim

    @property
    def h(self) -> float:
        return self.length / (self.n + 1)


def manufactured(dim: int, n: int, M: int, alpha: float, r: float | None = None,
                 k: int = 10, length: float = 1.0, T: float = 1.0, leaf: int = 16,
                 dtype=np.float64) -> Problem:
    """u = t^alpha prod sin(pi x_d/length): source f = (Gamma(1+alpha) +
    dim (pi/length)^2 t^alpha) prod sin(pi x_d/length), zero initial data."""
    if r is None:
        r = default_grading(alpha)
    t = graded_mesh(M, T, r)
    s = sine_mode(n, dim, length, (1,) * dim)
    lam = dim * (math.pi / length) ** 2
    prof = math.gamma(1.0 + alpha) + lam * t[1:] ** alpha
    f = np.outer(prof, s).astype(dtype)

    def exact():
        return np.outer(t[1:] ** alpha, s)

    return Problem(dim=dim, n=n, M=M, alpha=alpha, r=r, k=k, length=length, T=T, leaf=leaf,
                   t=t, f=f, g=None, exact=exact, modes=[((1,) * dim, prof)],
                   name=f"manufactured{dim}d_n{n}_M{M}_a{alpha}")


def paper_1d_mittag_leffler(n: int, M: int, alpha: float, k: int = 20,
                            r: float | None = None) -> Problem:
    """First experiment of Section 5: x in (0, pi), T = 1, f = 0, g = sin x.
    The exact solution E_alpha(-t^alpha) sin x needs the Mittag-Leffler
    function, which the caller evaluates."""
    if r is None:
        r = default_grading(alpha)
    length = math.pi
    t = graded_mesh(M, 1.0, r)
    s = sine_mode(n, 1, length, (1,))
    f = np.zeros((M, n))
    return Problem(dim=1, n=n, M=M, alpha=alpha, r=r, k=k, length=length, T=1.0, t=t, f=f,
                   g=s.copy(), modes=[((1,), np.zeros(M))], g_modes=[((1,), 1.0)],
                   name=f"paper1d_n{n}_M{M}_a{alpha}")


def paper_2d_polynomial(n: int, M: int, alpha: float, k: int = 20,
                        r: float | None = None) -> Problem:
    """Second experiment of Section 5 on (0, pi)^2: u = (t^3 + t^alpha) sin x sin y."""
    if r is None:
        r = default_grading(alpha)
    length = math.pi
    t = graded_mesh(M, 1.0, r)
    s = sine_mode(n, 2, length, (1, 1))
    tt = t[1:]
    prof = 2.0 * (tt ** 3 + tt ** alpha) + (math.gamma(alpha + 1.0)
                                           + math.gamma(4.0) / math.gamma(4.0 - alpha) * tt ** (3.0 - alpha))
    f = np.outer(prof, s)

    def exact():
        return np.outer(tt ** 3 + tt ** alpha, s)

    return Problem(dim=2, n=n, M=M, alpha=alpha, r=r, k=k, length=length, T=1.0, t=t, f=f,
                   exact=exact, modes=[((1, 1), prof)], name=f"paper2d_n{n}_M{M}_a{alpha}")


def random_fourier_2d(n: int, M: int, alpha: float, rng: np.random.Generator, k: int = 10,
                      r: float | None = None, nmodes: int = 8, kmax: int = 16, build_f: bool = True) -> Problem:
    """Source made of `nmodes` distinct sine modes (kx, ky) in {1..kmax}^2 with
    amplitudes z/(1 + kx^2 + ky^2), z ~ N(0, 1), times t^alpha; zero initial data,
    unit square, T = 1.  With build_f False only the modes are kept (f None):
    f = sum over modes of outer(profile, sine_mode(n, 2, 1, kvec))."""
    if r is None:
        r = default_grading(alpha)
    t = graded_mesh(M, 1.0, r)
    flat = rng.choice(kmax * kmax, size=nmodes, replace=False)
    z = rng.standard_normal(nmodes)
    tt = t[1:] ** alpha
    f = np.zeros((M, n * n)) if build_f else None
    modes = []
    for idx, zi in zip(flat, z):
        kx, ky = int(idx % kmax) + 1, int(idx // kmax) + 1
        amp = zi / (1.0 + kx * kx + ky * ky)
        if build_f:
            f += np.outer(amp * tt, sine_mode(n, 2, 1.0, (kx, ky)))
        modes.append(((kx, ky), amp * tt))
    return Problem(dim=2, n=n, M=M, alpha=alpha, r=r, k=k, t=t, f=f, modes=modes,
                   name=f"fourier2d_n{n}_M{M}_a{alpha:.3f}")


def batched_instances(count: int = 64, seed: int = 20261203, sides=(63, 127, 255),
                      Ms=(256, 512, 1024, 2048), alpha_range=(0.2, 0.9), k: int = 10,
                      build_f: bool = True):
    """Uneven instances of the batched workload: side, M and alpha drawn per
    instance from numpy's PCG64 seeded with [seed, i]."""
    out = []
    for i in range(count):
        rng = np.random.default_rng([seed, i])
        n = int(rng.choice(sides))
        M = int(rng.choice(Ms))
        alpha = float(rng.uniform(*alpha_range))
        if build_f == "modes":
            out.append(random_fourier_2d(n, M, alpha, rng, k=k, build_f=False))
        elif build_f:
            out.append(random_fourier_2d(n, M, alpha, rng, k=k))
        else:
            out.append((n, M, alpha))
    return out


def warm_start_family(dim: int, n: int, M: int, rng: np.random.Generator, alpha_range=(0.2, 0.9),
                      nmodes: int = 6, kmax: int = 16, k: int = 10, build_f: bool = True) -> Problem:
    """Training and evaluation family of the learned initial guess: alpha ~
    U(alpha_range), r = (2 - alpha)/alpha, zero initial data on (0, 1)^dim,
    T = 1, and a source made of `nmodes` distinct sine modes (wave numbers in
    {1..kmax}^dim, mode 1 always present) with time profiles
    a * Gamma(1 + alpha) + c * t^alpha, a ~ U(0, 1), c ~ N(0, 1), both divided by
    1 + |kvec|^2.  The manufactured sources of the benchmark workloads (one mode,
    a = 1, c = pi^2 dim) lie in its span.  With build_f False only the modes are
    kept (f None; the same random draws)."""
    alpha = float(rng.uniform(*alpha_range))
    r = default_grading(alpha)
    t = graded_mesh(M, 1.0, r)
    total = kmax ** dim
    flat = np.concatenate([[0], 1 + rng.choice(total - 1, size=nmodes - 1, replace=False)])
    a = rng.uniform(0.0, 1.0, nmodes)
    c = rng.standard_normal(nmodes)
    tt = t[1:] ** alpha
    f = np.zeros((M, n ** dim)) if build_f else None
    modes = []
    for idx, ai, ci in zip(flat, a, c):
        kvec = tuple(int(idx // kmax ** d % kmax) + 1 for d in range(dim))
        w = 1.0 + sum(kk * kk for kk in kvec)
        prof = (ai * math.gamma(1 + alpha) + ci * tt) / w
        if build_f:
            f += np.outer(prof, sine_mode(n, dim, 1.0, kvec))
        modes.append((kvec, prof))
    return Problem(dim=dim, n=n, M=M, alpha=alpha, r=r, k=k, t=t, f=f, modes=modes,
                   name=f"warm{dim}d_n{n}_M{M}_a{alpha:.3f}")


def config(name: str, alpha: float | None = None) -> Problem:
    """The named workloads.

    small1d : 1D, n=63, M=128, r=3, alpha=0.5, k=8 (manufactured)
    large1d : 1D, n=1023, M=4096, r=(2-a)/a, a in {0.3,0.5,0.7}, k=10
    large2d : 2D, n=255, M=1024, r=3, alpha=0.5, k=10
    """
    if name == "small1d":
        return manufactured(1, 63, 128, 0.5 if alpha is None else alpha, r=3.0, k=8)
    if name == "large1d":
        a = 0.5 if alpha is None else alpha
        return manufactured(1, 1023, 4096, a, r=default_grading(a), k=10)
    if name == "large2d":
        return manufactured(2, 255, 1024, 0.5 if alpha is None else alpha, r=3.0, k=10)
    raise KeyError(name)
