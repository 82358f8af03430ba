"""Parity at the benchmark's full sizes, in the launch configurations the
benchmark times:

* the three 1D instances (n = 1023, M = 4096) in one batch, i.e. one merged
  pipelined launch (float64);
* the 2D instance n = 255, M = 1024 in float64 and with float32 inner cycles;
* the 64 uneven 2D instances of the batched workload in one graph-replayed
  batch, with float64 cycles and with float32 inner cycles.

Outputs are compared on sampled columns with the oracle's solution for the
same H-matrix (each source is a sum of separable sine modes, so the exact
discrete solution is a sum of one triangular solve per mode), and the oracle
evaluates the float64 residual at the sampled points from their time lines
and those of their neighbours."""
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


def _sampled_reference(p, cols, Rt=None):
    """Oracle solution and right-hand side at the sampled columns."""
    Rt = oracle.hmatrix_dense(p.t, p.alpha, p.k, p.leaf) if Rt is None else Rt
    ref = np.zeros((p.M, len(cols)))
    b = np.zeros((p.M, len(cols)))
    for kvec, prof in p.modes:
        w = oracle.single_mode_profile(Rt, oracle.mode_eigenvalue(kvec, p.n, p.length), prof)
        s = W.sine_mode(p.n, p.dim, p.length, kvec)
        ref += np.outer(w, s[cols])
        b += np.outer(prof, s[cols])
    return ref, b, Rt


def _columns(N, rng, count=48):
    return np.unique(np.concatenate([[0, 1, N // 2, N - 2, N - 1], rng.integers(0, N, count)]))


def _sampled_check(p, u, cols, dev, Rt=None):
    """(relative error, relative oracle residual) of u at the sampled columns;
    the residual uses the time lines of the columns and their neighbours."""
    ref, b, Rt = _sampled_reference(p, cols, Rt)
    idx = torch.as_tensor(cols, device=dev)
    U = u[:, idx].cpu().numpy()
    if p.dim == 1:
        pairs = [(cols - 1, cols >= 1), (cols + 1, cols + 1 < p.n)]
    else:
        ix, iy = cols % p.n, cols // p.n
        pairs = [(cols - 1, ix > 0), (cols + 1, ix < p.n - 1), (cols - p.n, iy > 0), (cols + p.n, iy < p.n - 1)]
    nb = []
    for q, ok in pairs:
        v = u[:, torch.as_tensor(np.where(ok, q, 0), device=dev)].cpu().numpy()
        nb.append(np.where(ok[None, :], v, 0.0))
    r = oracle.residual_sampled(Rt, b, U, nb, p.h)
    return np.max(np.abs(U - ref)) / np.max(np.abs(ref)), np.abs(r).max() / _bnorm(p)


def _bnorm(p, rows=256):
    """||b||_inf of a sum of separable sine modes (g = 0), in blocks of time rows."""
    P = np.stack([prof for _, prof in p.modes], axis=1)                          # [M][modes]
    S = np.stack([W.sine_mode(p.n, p.dim, p.length, kv) for kv, _ in p.modes])   # [modes][N]
    return max(np.abs(P[m:m + rows] @ S).max() for m in range(0, p.M, rows))


def _batched_sources(probs, dev):
    fs = []
    for p in probs:
        f = torch.zeros((p.M, p.N), dtype=torch.float64, device=dev)
        for kvec, prof in p.modes:
            f.add_(torch.outer(torch.as_tensor(prof, dtype=torch.float64, device=dev),
                               torch.as_tensor(W.sine_mode(p.n, 2, 1.0, kvec), dtype=torch.float64, device=dev)))
        fs.append(f)
    return fs


def test_large1d_batch_as_benchmarked(dev):
    probs = [W.config("large1d", a) for a in (0.3, 0.5, 0.7)]
    plans = [mg.Plan(p.dim, p.n, p.M, p.alpha, k=p.k, r=p.r, t=p.t, length=p.length, leaf=p.leaf).bind()
             for p in probs]
    batch = mg.Batch(plans).bind()
    fs = [torch.as_tensor(p.f, dtype=torch.float64, device=dev) for p in probs]
    us = [torch.empty_like(f) for f in fs]
    rng = np.random.default_rng(11)
    cols = _columns(probs[0].N, rng)
    # the float64 residual of any iterate stalls near 2e-10 at h = 1/1024
    for rep in range(2):
        _, sts = batch.solve(fs, tol=5e-10, us=us)
        for p, u, st in zip(probs, us, sts):
            err, res = _sampled_check(p, u, cols, dev)
            print(f"large1d alpha={p.alpha} rep={rep}: error {err:.2e}, sampled residual {res:.2e}", flush=True)
            assert err < 1e-10, (rep, p.alpha, st)
            assert res <= 6e-10 and st["res"] <= 5e-10 * st["bnorm"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_large2d_as_benchmarked(dev, precision):
    """2D n = 255, M = 1024 (float64, or float32 inner cycles with a float64
    residual), to the benchmark's 1e-8 and, in float64, to 5e-11 as well."""
    p = W.config("large2d")
    plan = mg.Plan(p.dim, p.n, p.M, p.alpha, k=p.k, r=p.r, t=p.t, length=p.length, leaf=p.leaf,
                   precision=precision).bind()
    f = torch.as_tensor(p.f, dtype=torch.float64, device=dev)
    u = torch.empty_like(f)
    cols = _columns(p.N, np.random.default_rng(13))
    ref, _, Rt = _sampled_reference(p, cols)
    for tol in ((1e-8, 5e-11) if precision == "fp64" else (1e-8,)):
        _, st = plan.solve(f, tol=tol, u=u)
        err, res = _sampled_check(p, u, cols, dev, Rt)
        print(f"large2d {precision} tol={tol:g}: {st['cycles']} cycles, error {err:.2e}, sampled residual "
              f"{res:.2e}", flush=True)
        assert st["res"] <= tol * st["bnorm"] and res <= 1.2 * tol
        assert err < (1e-10 if tol < 1e-9 else 1e-7), (precision, tol, err)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_workload_as_benchmarked(dev, precision):
    """All 64 instances in one graph-replayed batch: float64 cycles to 5e-11
    (error 1e-10), or float32 inner cycles with the float64 residual to the
    benchmark's 1e-8."""
    probs = W.batched_instances(count=64, build_f="modes")
    fs = _batched_sources(probs, dev)
    us = [torch.empty_like(f) for f in fs]
    plans = [mg.Plan(2, p.n, p.M, p.alpha, k=p.k, r=p.r, t=p.t, precision=precision).bind() for p in probs]
    batch = mg.Batch(plans, graph=True).bind()
    tol = 5e-11 if precision == "fp64" else 1e-8
    for rep in range(2):
        _, sts = batch.solve(fs, tol=tol, us=us)
    print(f"{precision}: solved", sum(p.M * p.N for p in probs), "unknowns; staged",
          sum(pl.tuned()["schedule"] == "staged" for pl in plans), "graph replays", batch.graph_replays(), flush=True)
    rng = np.random.default_rng(12)
    worst_err = worst_res = 0.0
    for i, (p, u, st) in enumerate(zip(probs, us, sts)):
        cols = _columns(p.N, rng, count=24)
        err, res = _sampled_check(p, u, cols, dev)
        worst_err, worst_res = max(worst_err, err), max(worst_res, res)
        assert err < (1e-10 if precision == "fp64" else 1e-7), (i, p.n, p.M, p.alpha, err, st)
        assert res <= 1.2 * tol and st["res"] <= tol * st["bnorm"], (i, res, st)
    print(f"{precision}: worst sampled error {worst_err:.2e}, worst sampled residual {worst_res:.2e}", flush=True)
