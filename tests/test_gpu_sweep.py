"""Seeded sweep over the solver's parameter space on the GPU, each case
against the float64 oracle with the same R~: dimension, grid, time mesh
(graded and uniform, ragged leaf counts), leaf size, Taylor rank, smoothing
counts, V- and W-cycles, both schedules, float64 and mixed precision, with
and without an initial value."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1706_07632_amd as mg  # noqa: E402


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _cases(count=48, seed=20261203):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        dim = int(rng.integers(1, 3))
        n = int(rng.choice([7, 15, 31, 63] if dim == 1 else [7, 15, 31]))
        M = int(rng.integers(16, 301))
        alpha = float(rng.uniform(0.2, 0.9))
        r = 1.0 if rng.random() < 0.25 else (2 - alpha) / alpha
        k = int(rng.integers(4, 11))
        leaf = int(rng.choice([8, 12, 16]))
        nu1, nu2 = [(1, 1), (2, 1), (1, 2), (0, 1), (1, 0)][int(rng.integers(0, 5))]
        gamma = int(rng.choice([1, 1, 2]))
        schedule = str(rng.choice(["staged", "pipelined"]))
        precision = str(rng.choice(["fp64", "fp64", "mixed"]))
        with_g = bool(rng.random() < 0.5)
        out.append((i, dim, n, M, alpha, r, k, leaf, nu1, nu2, gamma, schedule, precision, with_g))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"c{c[0]}")
def test_sweep_against_oracle(dev, case):
    i, dim, n, M, alpha, r, k, leaf, nu1, nu2, gamma, schedule, precision, with_g = case
    print("case", case, flush=True)
    rng = np.random.default_rng([7, i])
    N = n ** dim
    t = W.graded_mesh(M, 1.0, r)
    f = rng.standard_normal((M, N))
    g = rng.standard_normal(N) if with_g else None
    plan = mg.Plan(dim, n, M, alpha, k=k, t=t, leaf=leaf, nu1=nu1, nu2=nu2, gamma=gamma, schedule=schedule,
                   precision=precision, max_cycles=160).bind()
    fd = torch.as_tensor(f, dtype=torch.float64, device=dev)
    gd = None if g is None else torch.as_tensor(g, dtype=torch.float64, device=dev)
    # float64 plans solve to 1e-12 (every grid here has h >= 1/64, whose float64
    # residual floor lies below 1e-12) and must match the oracle to 1e-10;
    # mixed plans stop at 1e-10 and match to 1e-8
    tol = 1e-12 if precision == "fp64" else 1e-10
    u, st = plan.solve(fd, gd, tol=tol)
    U = u.cpu().numpy()
    Rt = oracle.hmatrix_dense(t, alpha, k, leaf)
    B = oracle.rhs(f, t, alpha, g)
    ref = oracle.timestep_solve(Rt, B, dim, n, 1.0)
    err = np.max(np.abs(U - ref)) / np.max(np.abs(ref))
    res = np.max(np.abs(oracle.residual(Rt, U, B, dim, n, 1.0))) / np.max(np.abs(B))
    bound = 1e-10 if precision == "fp64" else 1e-8
    assert res <= 1.2 * tol + 1e-13 and err < bound, (case, err, res, st["cycles"])
    plan.close()


@pytest.mark.parametrize("case", [c for c in _cases() if c[12] == "fp64"], ids=lambda c: f"z{c[0]}")
def test_sweep_zebra_tolerance(dev, case):
    """The float64 cases of the sweep at a tolerance of 1e-10, where the
    cycles form their restriction's defect (and, staged in 2D, the stopping
    test's norm) from the changes of the last half-sweep wherever the
    smoothing counts allow it: the oracle's residual of the returned iterate
    meets the tolerance and the error matches the mixed cases' bound."""
    i, dim, n, M, alpha, r, k, leaf, nu1, nu2, gamma, schedule, precision, with_g = case
    print("case", case, flush=True)
    rng = np.random.default_rng([7, i])
    N = n ** dim
    t = W.graded_mesh(M, 1.0, r)
    f = rng.standard_normal((M, N))
    g = rng.standard_normal(N) if with_g else None
    plan = mg.Plan(dim, n, M, alpha, k=k, t=t, leaf=leaf, nu1=nu1, nu2=nu2, gamma=gamma, schedule=schedule,
                   max_cycles=160).bind()
    fd = torch.as_tensor(f, dtype=torch.float64, device=dev)
    gd = None if g is None else torch.as_tensor(g, dtype=torch.float64, device=dev)
    u, st = plan.solve(fd, gd, tol=1e-10)
    U = u.cpu().numpy()
    Rt = oracle.hmatrix_dense(t, alpha, k, leaf)
    B = oracle.rhs(f, t, alpha, g)
    ref = oracle.timestep_solve(Rt, B, dim, n, 1.0)
    err = np.max(np.abs(U - ref)) / np.max(np.abs(ref))
    res = np.max(np.abs(oracle.residual(Rt, U, B, dim, n, 1.0))) / np.max(np.abs(B))
    assert res <= 1.2e-10 + 1e-13 and err < 1e-8, (case, err, res, st["cycles"])
    plan.close()
