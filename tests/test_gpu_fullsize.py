"""Parity at the benchmark's full sizes, in the launch configurations the
benchmark times: the three 1D instances (n = 1023, M = 4096) in one batch,
i.e. one merged pipelined launch, and the 64 uneven 2D instances of the
batched workload in one graph-replayed batch (pipelined instances merged,
staged ones side by side).  Outputs are compared on sampled columns with the
oracle's solution for the same H-matrix: each source is a sum of separable
sine modes, so the exact discrete solution is a sum of one triangular solve
per mode."""
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


def _sampled_reference(p, cols):
    Rt = oracle.hmatrix_dense(p.t, p.alpha, p.k, p.leaf)
    ref = np.zeros((p.M, len(cols)))
    scale = 0.0
    for kvec, prof in p.modes:
        w = oracle.single_mode_profile(Rt, oracle.mode_eigenvalue(kvec, p.n, p.length), prof)
        s = W.sine_mode(p.n, p.dim, p.length, kvec)
        ref += np.outer(w, s[cols])
        scale += np.max(np.abs(w)) * np.max(np.abs(s))
    return ref, scale


def _columns(N, rng, count=48):
    return np.unique(np.concatenate([[0, 1, N // 2, N - 2, N - 1], rng.integers(0, N, count)]))


def test_large1d_batch_as_benchmarked(dev):
    probs = [W.config("large1d", a) for a in (0.3, 0.5, 0.7)]
    plans = [mg.Plan(p.dim, p.n, p.M, p.alpha, k=p.k, r=p.r, t=p.t, length=p.length, leaf=p.leaf).bind()
             for p in probs]
    batch = mg.Batch(plans).bind()
    fs = [torch.as_tensor(p.f, dtype=torch.float64, device=dev) for p in probs]
    us = [torch.empty_like(f) for f in fs]
    rng = np.random.default_rng(11)
    cols = _columns(probs[0].N, rng)
    refs = [_sampled_reference(p, cols) for p in probs]
    # the float64 residual of any iterate stalls near 2e-10 at h = 1/1024
    for rep in range(2):
        _, sts = batch.solve(fs, tol=5e-10, us=us)
        for p, u, st, (ref, scale) in zip(probs, us, sts, refs):
            U = u[:, torch.as_tensor(cols, device=dev)].cpu().numpy()
            assert np.max(np.abs(U - ref)) / np.max(np.abs(ref)) < 1e-10, (rep, p.alpha, st)
            assert st["res"] <= 5e-10 * st["bnorm"]


def test_batched_workload_as_benchmarked(dev):
    probs = W.batched_instances(count=64, build_f="modes")
    fs = []
    for p in probs:
        f = torch.zeros((p.M, p.N), dtype=torch.float64, device=dev)
        for kvec, prof in p.modes:
            f.add_(torch.outer(torch.as_tensor(prof, dtype=torch.float64, device=dev),
                               torch.as_tensor(W.sine_mode(p.n, 2, 1.0, kvec), dtype=torch.float64, device=dev)))
        fs.append(f)
    us = [torch.empty_like(f) for f in fs]
    plans = [mg.Plan(2, p.n, p.M, p.alpha, k=p.k, r=p.r, t=p.t).bind() for p in probs]
    batch = mg.Batch(plans, graph=True).bind()
    for rep in range(2):
        _, sts = batch.solve(fs, tol=1e-10, us=us)
    print("solved", sum(p.M * p.N for p in probs), "unknowns; schedules",
          sum(pl.tuned()["schedule"] == "staged" for pl in plans), "staged", flush=True)
    rng = np.random.default_rng(12)
    worst = 0.0
    for i, (p, u, st) in enumerate(zip(probs, us, sts)):
        cols = _columns(p.N, rng, count=24)
        ref, scale = _sampled_reference(p, cols)
        U = u[:, torch.as_tensor(cols, device=dev)].cpu().numpy()
        err = np.max(np.abs(U - ref)) / scale
        worst = max(worst, err)
        assert err < 1e-8, (i, p.n, p.M, p.alpha, err, st)
        assert st["res"] <= 1e-10 * st["bnorm"], (i, st)
    print("worst sampled error", worst, flush=True)
