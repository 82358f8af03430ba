"""GPU parity of the HIP path (through the C ABI) against the float64 oracle."""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1706_07632_amd as mg  # noqa: E402  (fails loudly if the library is missing)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _plan(p, dev, **kw):
    return mg.Plan(p.dim, p.n, p.M, p.alpha, k=p.k, t=p.t, length=p.length, leaf=p.leaf, **kw).bind()


def _cuda(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


@pytest.mark.parametrize("M,alpha,r,k,ncols", [(128, 0.5, 3.0, 8, 16), (256, 0.3, 17 / 3, 10, 37),
                                               (1024, 0.5, 3.0, 10, 5), (300, 0.7, 1.857142857142857, 6, 70),
                                               (2048, 0.4, 4.0, 10, 24)])
def test_hmatvec_matches_oracle(dev, M, alpha, r, k, ncols):
    t = W.graded_mesh(M, 1.0, r)
    plan = mg.Plan(1, 15, M, alpha, k=k, t=t).bind()
    rng = np.random.default_rng(1)
    X = rng.standard_normal((M, ncols))
    Y = plan.hmatvec(_cuda(X, dev)).cpu().numpy()
    ref = oracle.hmatrix_dense(t, alpha, k) @ X
    assert np.max(np.abs(Y - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("M,alpha,r,k,ncols,level", [(128, 0.5, 3.0, 8, 16, 0), (512, 0.3, 17 / 3, 10, 33, 1),
                                                     (2048, 0.2, 9.0, 10, 20, 0), (100, 0.5, 1.0, 6, 3, 2)])
def test_htrsm_matches_oracle(dev, M, alpha, r, k, ncols, level):
    t = W.graded_mesh(M, 1.0, r)
    plan = mg.Plan(1, 31, M, alpha, k=k, t=t).bind()
    rng = np.random.default_rng(2)
    B = rng.standard_normal((M, ncols))
    X = plan.htrsm(_cuda(B, dev), level=level).cpu().numpy()
    n_l = (31 + 1) // (2 ** level) - 1
    c = 2.0 / (1.0 / (n_l + 1)) ** 2
    Rt = oracle.hmatrix_dense(t, alpha, k)
    ref = scipy.linalg.solve_triangular(Rt + c * np.eye(M), B, lower=True)
    assert np.max(np.abs(X - ref)) <= 1e-12 * np.max(np.abs(ref))


def _solve_and_compare(p, dev, tol=1e-12, parity=1e-10, g=None, **kw):
    plan = _plan(p, dev, **kw)
    f = _cuda(p.f, dev)
    gd = None if g is None else _cuda(g, dev)
    u, st = plan.solve(f, gd, tol=tol)
    U = u.cpu().numpy()
    Rt = oracle.hmatrix_dense(p.t, p.alpha, p.k, p.leaf)
    B = oracle.rhs(p.f, p.t, p.alpha, g)
    ref = oracle.timestep_solve(Rt, B, p.dim, p.n, p.length)
    err = np.max(np.abs(U - ref)) / np.max(np.abs(ref))
    res = np.max(np.abs(oracle.residual(Rt, U, B, p.dim, p.n, p.length))) / np.max(np.abs(B))
    return err, res, st


def test_small1d_manufactured_parity(dev):
    p = W.config("small1d")
    err, res, st = _solve_and_compare(p, dev)
    assert err < 1e-10, (err, st)
    assert res < 1e-12, (res, st)
    assert 4 <= st["cycles"] <= 15


def test_small1d_mesh_from_formula(dev):
    p = W.config("small1d")
    plan = mg.Plan(1, p.n, p.M, p.alpha, k=p.k, r=p.r).bind()
    u, st = plan.solve(_cuda(p.f, dev), tol=1e-12)
    Rt = oracle.hmatrix_dense(p.t, p.alpha, p.k)
    ref = oracle.timestep_solve(Rt, oracle.rhs(p.f, p.t, p.alpha, None), 1, p.n, 1.0)
    assert np.max(np.abs(u.cpu().numpy() - ref)) / np.max(np.abs(ref)) < 1e-10


@pytest.mark.parametrize("dim,n,M,alpha,r,k", [(1, 31, 96, 0.3, 17 / 3, 6), (2, 15, 64, 0.5, 3.0, 8),
                                               (2, 7, 40, 0.8, 1.25, 10), (1, 1, 32, 0.5, 2.0, 4),
                                               (2, 3, 17, 0.6, 2.0, 5)])
def test_random_source_and_initial_value_parity(dev, dim, n, M, alpha, r, k):
    rng = np.random.default_rng(3)
    N = n ** dim
    t = W.graded_mesh(M, 1.0, r)
    p = W.Problem(dim=dim, n=n, M=M, alpha=alpha, r=r, k=k, t=t, f=rng.standard_normal((M, N)))
    g = rng.standard_normal(N)
    err, res, st = _solve_and_compare(p, dev, g=g)
    assert err < 1e-10, (err, st)
    assert res < 1e-12


@pytest.mark.parametrize("schedule", ["staged", "pipelined"])
@pytest.mark.parametrize("dim,n,M,precision", [(1, 15, 16, "fp64"), (1, 31, 17, "fp64"), (2, 7, 33, "fp64"),
                                               (2, 15, 16, "mixed"), (1, 63, 33, "mixed"),
                                               (2, 15, 16, "mixed_bf16"), (1, 63, 33, "mixed_bf16")])
def test_one_to_three_leaves(dev, schedule, dim, n, M, precision):
    """Time meshes of one leaf (M = 16) and of two or three ragged leaves
    (M = 17: 8 + 9; M = 33: 16 + 8 + 9): the first and last leaf steps of the
    marches, the input loads one leaf ahead and the progress reads near the
    end all meet their edge cases."""
    rng = np.random.default_rng(M + n)
    N = n ** dim
    t = W.graded_mesh(M, 1.0, 2.5)
    p = W.Problem(dim=dim, n=n, M=M, alpha=0.45, r=2.5, k=6, t=t, f=rng.standard_normal((M, N)))
    print("case", schedule, dim, n, M, precision, flush=True)
    err, res, st = _solve_and_compare(p, dev, g=rng.standard_normal(N), schedule=schedule, precision=precision,
                                      tol=1e-11)
    assert err < 1e-9 and res < 1e-10, (err, res, st)


def test_paper_1d_problem_small(dev):
    p = W.paper_1d_mittag_leffler(63, 64, 0.6, k=20)
    err, res, st = _solve_and_compare(p, dev, g=p.g)
    assert err < 1e-10
    ex = oracle.mittag_leffler(0.6, -p.t[1:] ** 0.6)[:, None] * p.g[None, :]
    plan = _plan(p, dev)
    u, _ = plan.solve(_cuda(p.f, dev), _cuda(p.g, dev), tol=1e-10)
    assert np.max(np.abs(u.cpu().numpy() - ex)) < 2e-2   # discretisation error at this size


def test_residual_entry_point(dev):
    rng = np.random.default_rng(4)
    p = W.manufactured(2, 15, 64, 0.4, r=3.0, k=8)
    plan = _plan(p, dev)
    U = rng.standard_normal((p.M, p.N))
    g = rng.standard_normal(p.N)
    out = torch.empty((p.M, p.N), dtype=torch.float64, device=dev)
    _, nrm = plan.residual(_cuda(p.f, dev), _cuda(U, dev), g=_cuda(g, dev), out=out)
    Rt = oracle.hmatrix_dense(p.t, p.alpha, p.k)
    ref = oracle.residual(Rt, U, oracle.rhs(p.f, p.t, p.alpha, g), 2, p.n, 1.0)
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert abs(nrm - np.max(np.abs(ref))) <= 1e-13 * np.max(np.abs(ref))


def test_w_cycle_and_v01_converge(dev):
    p = W.config("small1d")
    e1, _, st1 = _solve_and_compare(p, dev, gamma=2)
    e2, _, st2 = _solve_and_compare(p, dev, nu1=0, nu2=1)
    assert e1 < 1e-10 and e2 < 1e-10
    assert st1["cycles"] <= st2["cycles"] + 2


@pytest.mark.parametrize("schedule", ["staged", "pipelined"])
@pytest.mark.parametrize("dim,nu1,nu2", [(1, 1, 0), (1, 0, 1), (1, 2, 2), (2, 0, 1), (2, 1, 0)])
def test_smoothing_counts_with_and_without_fused_transfers(dev, schedule, dim, nu1, nu2):
    """Cycles whose grid transfers are fused into the marches (1D, nu1 >= 1
    restriction, nu2 >= 1 prolongation) and those that keep separate stencil
    stages (the others, and 2D) reach the oracle's solution."""
    p = W.manufactured(dim, 31 if dim == 1 else 15, 128, 0.5, r=3.0, k=8)
    print("case", schedule, dim, nu1, nu2, flush=True)
    err, res, st = _solve_and_compare(p, dev, nu1=nu1, nu2=nu2, schedule=schedule, tol=1e-11, parity=1e-9)
    assert err < 1e-9 and res < 1e-10, (err, res, st)


def _single_mode_reference(p):
    Rt = oracle.hmatrix_dense(p.t, p.alpha, p.k, p.leaf)
    (kvec, prof), = p.modes
    w = oracle.single_mode_profile(Rt, oracle.mode_eigenvalue(kvec, p.n, p.length), prof)
    s = W.sine_mode(p.n, p.dim, p.length, kvec)
    return Rt, w, s


@pytest.mark.parametrize("dim,n,M,precision", [(1, 63, 2048, "fp64"), (2, 31, 2048, "fp64"),
                                               (2, 31, 2048, "mixed"), (1, 127, 4096, "mixed_bf16"),
                                               (2, 15, 1024, "fp64")])
def test_staged_solves_on_long_meshes(dev, dim, n, M, precision):
    """Marches launched one by one on meshes of 128 and 256 time leaves
    (which take the deeper operand prefetch) and of 64 leaves (the shallower
    one), against the single-mode oracle."""
    p = W.manufactured(dim, n, M, 0.4, r=4.0, k=10)
    print("case", dim, n, M, precision, flush=True)
    plan = _plan(p, dev, schedule="staged", precision=precision)
    u, st = plan.solve(_cuda(p.f, dev), tol=1e-10)
    Rt, w, s = _single_mode_reference(p)
    ref = np.outer(w, s)
    assert np.max(np.abs(u.cpu().numpy() - ref)) / np.max(np.abs(ref)) < 1e-9, st


@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.7])
def test_large1d_parity_full_size(dev, alpha):
    """n = 1023, M = 4096: the source is one sine mode, so the exact discrete
    solution is w(t) s(x) with (R~ + lambda_h I) w = phi (one triangular solve)."""
    p = W.config("large1d", alpha)
    plan = _plan(p, dev)
    # the float64 relative residual of any iterate stalls near 2e-10 at h = 1/1024
    # (rounding of A u with ||A|| ~ 4/h^2), so stop at 5e-10
    u, st = plan.solve(_cuda(p.f, dev), tol=5e-10)
    Rt, w, s = _single_mode_reference(p)
    ref = np.outer(w, s)
    U = u.cpu().numpy()
    assert np.max(np.abs(U - ref)) / np.max(np.abs(ref)) < 1e-10, st
    cols = np.array([0, 1, 511, 512, 1000, 1022])
    r = oracle.residual_columns(Rt, U, p.f, 1, p.n, 1.0, cols)
    assert np.max(np.abs(r)) <= 5e-10 * st["bnorm"] * 1.01


def test_large2d_parity_full_size(dev):
    p = W.config("large2d")
    plan = _plan(p, dev)
    u, st = plan.solve(_cuda(p.f, dev), tol=1e-10)   # residual floor here is about 1.5e-11
    Rt, w, s = _single_mode_reference(p)
    rng = np.random.default_rng(5)
    cols = np.unique(np.concatenate([[0, 1, 254, 255, 32512, 65024], rng.integers(0, p.N, 200)]))
    U = u[:, torch.as_tensor(cols, device=dev)].cpu().numpy()
    ref = np.outer(w, s[cols])
    assert np.max(np.abs(U - ref)) / np.max(np.abs(np.outer(w, s))) < 1e-10, st


@pytest.mark.parametrize("precision", ["mixed", "mixed_bf16"])
@pytest.mark.parametrize("schedule,inner", [("staged", 1), ("pipelined", 1), ("pipelined", 2)])
def test_mixed_precision_reaches_tolerance(dev, schedule, inner, precision):
    p = W.manufactured(1, 255, 1024, 0.5, r=3.0, k=10)
    plan = _plan(p, dev, precision=precision, inner_cycles=inner, schedule=schedule)
    u, st = plan.solve(_cuda(p.f, dev), tol=1e-8)
    Rt, w, s = _single_mode_reference(p)
    U = u.cpu().numpy()
    res = np.max(np.abs(oracle.residual(Rt, U, p.f, 1, p.n, 1.0)))
    assert res <= 1e-8 * st["bnorm"] * 1.01, st
    assert st["refinements"] >= 1
    err = np.max(np.abs(U - np.outer(w, s))) / np.max(np.abs(w))
    assert err < 1e-7, err


def test_not_converged_status_and_nonfinite(dev):
    p = W.config("small1d")
    plan = _plan(p, dev, max_cycles=1)
    u, st = plan.solve(_cuda(p.f, dev), tol=1e-14, allow_unconverged=True)
    assert st["cycles"] == 1 and st["res"] > 1e-14 * st["bnorm"]
    with pytest.raises(mg.MgwrError) as ei:
        plan.solve(_cuda(p.f, dev), tol=1e-14)
    assert ei.value.code == mg.MGWR_ERR_NOT_CONVERGED
    f = p.f.copy()
    f[3, 7] = np.nan
    with pytest.raises(mg.MgwrError) as ei:
        plan.solve(_cuda(f, dev), tol=1e-10)
    assert ei.value.code == mg.MGWR_ERR_NONFINITE


@pytest.mark.parametrize("precision", ["mixed", "mixed_bf16"])
def test_mixed_precision_on_strongly_graded_mesh(dev, precision):
    """alpha = 0.3, r = 17/3, M = 4096 puts t_1 near 3e-21: the float32 (and
    bfloat16) copies of the Taylor factors must stay in range (they are stored
    rescaled)."""
    p = W.config("large1d", 0.3)
    plan = _plan(p, dev, precision=precision, inner_cycles=1)
    u, st = plan.solve(_cuda(p.f, dev), tol=1e-8)
    Rt, w, s = _single_mode_reference(p)
    U = u.cpu().numpy()
    cols = np.array([0, 3, 511, 512, 1022])
    r = oracle.residual_columns(Rt, U, p.f, 1, p.n, 1.0, cols)
    assert np.max(np.abs(r)) <= 1e-8 * st["bnorm"] * 1.01, st
    err = np.max(np.abs(U - np.outer(w, s))) / np.max(np.abs(w))
    assert err < 1e-7, err


@pytest.mark.parametrize("dim,n,M,alpha,r,k,gamma", [(1, 63, 128, 0.5, 3.0, 8, 1), (2, 31, 256, 0.4, 3.0, 10, 1),
                                                     (1, 127, 512, 0.3, 17 / 3, 10, 2)])
def test_pipelined_schedule_matches_staged(dev, dim, n, M, alpha, r, k, gamma):
    """The time-pipelined launch of whole cycles computes the same iterates as one
    launch per stage (up to float64 rounding order)."""
    rng = np.random.default_rng(9)
    N = n ** dim
    t = W.graded_mesh(M, 1.0, r)
    f = _cuda(rng.standard_normal((M, N)), dev)
    g = _cuda(rng.standard_normal(N), dev)
    out = {}
    for sched in ("staged", "pipelined"):
        plan = mg.Plan(dim, n, M, alpha, k=k, t=t, gamma=gamma, schedule=sched, max_cycles=5).bind()
        u, st = plan.solve(f, g, tol=1e-30, allow_unconverged=True)
        out[sched] = (u.cpu().numpy(), st)
    (u1, s1), (u2, s2) = out["staged"], out["pipelined"]
    assert s1["cycles"] == s2["cycles"] == 5
    assert np.max(np.abs(u1 - u2)) <= 1e-12 * np.max(np.abs(u1))
    h1, h2 = np.array(s1["history"]), np.array(s2["history"])
    assert np.all(np.abs(h1 - h2) <= 1e-6 * h1 + 1e-14 * s1["bnorm"]), (h1, h2)


def test_batched_uneven_instances_match_oracle(dev):
    """Instances of different dimension, size, mesh and rank in one merged
    pipelined launch; each checked against the oracle."""
    rng = np.random.default_rng(21)
    cases = [(1, 63, 128, 0.5, 3.0, 8, True), (2, 15, 64, 0.3, 17 / 3, 10, False),
             (1, 127, 256, 0.7, 1.857142857142857, 6, True), (2, 31, 96, 0.6, 2.0, 8, False)]
    plans, fs, gs, probs = [], [], [], []
    for dim, n, M, alpha, r, k, with_g in cases:
        N = n ** dim
        t = W.graded_mesh(M, 1.0, r)
        p = W.Problem(dim=dim, n=n, M=M, alpha=alpha, r=r, k=k, t=t, f=rng.standard_normal((M, N)),
                      g=rng.standard_normal(N) if with_g else None)
        probs.append(p)
        plans.append(mg.Plan(dim, n, M, alpha, k=k, t=t).bind())
        fs.append(_cuda(p.f, dev))
        gs.append(None if p.g is None else _cuda(p.g, dev))
    batch = mg.Batch(plans).bind()
    for rep in range(2):    # the second solve reuses the learned cycle counts
        us, sts = batch.solve(fs, gs, tol=1e-11)
        for p, u, st in zip(probs, us, sts):
            Rt = oracle.hmatrix_dense(p.t, p.alpha, p.k)
            ref = oracle.timestep_solve(Rt, oracle.rhs(p.f, p.t, p.alpha, p.g), p.dim, p.n, 1.0)
            err = np.max(np.abs(u.cpu().numpy() - ref)) / np.max(np.abs(ref))
            assert err < 1e-10, (p.dim, p.n, p.M, err, st)
            assert st["res"] <= 1e-11 * st["bnorm"]


def test_repeated_solves_keep_cycle_count(dev):
    """After the first solve the cycle count is known and a pipelined launch
    evaluates the defect only after its last cycle: the second solve must run
    the same number of cycles and reach the same residual."""
    p = W.manufactured(1, 255, 1024, 0.5, r=3.0, k=10)
    plan = _plan(p, dev, schedule="pipelined")
    f = _cuda(p.f, dev)
    u1, s1 = plan.solve(f, tol=1e-8)
    u2, s2 = plan.solve(f, tol=1e-8)
    assert s1["cycles"] == s2["cycles"]
    assert s2["res"] <= 1e-8 * s2["bnorm"]
    assert torch.equal(u1, u2)
    batch = mg.Batch([plan]).bind()
    (u3,), (s3,) = batch.solve([f], tol=1e-8)
    assert s3["cycles"] == s1["cycles"] and torch.equal(u1, u3)


def test_batched_mixed_and_plain_instances(dev):
    """A batch holding float64, mixed-precision and bfloat16-factor plans (1D
    and 2D) in one launch."""
    probs = [W.manufactured(1, 127, 512, 0.4, k=10), W.manufactured(2, 31, 256, 0.6, r=3.0, k=8)]
    plans = [_plan(probs[0], dev, precision="mixed"), _plan(probs[1], dev),
             _plan(probs[1], dev, precision="mixed", inner_cycles=2),
             _plan(probs[0], dev, precision="mixed_bf16"), _plan(probs[1], dev, precision="mixed_bf16")]
    probs = [probs[0], probs[1], probs[1], probs[0], probs[1]]
    batch = mg.Batch(plans).bind()
    us, sts = batch.solve([_cuda(p.f, dev) for p in probs], tol=1e-8)
    for p, u, st in zip(probs, us, sts):
        Rt, w, s = _single_mode_reference(p)
        U = u.cpu().numpy()
        res = np.max(np.abs(oracle.residual(Rt, U, p.f, p.dim, p.n, 1.0)))
        assert res <= 1e-8 * st["bnorm"] * 1.01, st
        assert np.max(np.abs(U - np.outer(w, s))) / np.max(np.abs(w)) < 1e-7


@pytest.mark.parametrize("schedule", ["pipelined", "staged"])
def test_stalled_progress_wait_fails_and_the_plan_recovers(dev, schedule):
    """A progress bound of 0 polls makes the first wait that finds its
    producer behind give up: the pipelined launch (or, staged, the launch of
    the coarse levels) stops every work item, the solve reports the stall, and
    with the default bound restored the same plan solves correctly."""
    p = W.manufactured(1, 127, 512, 0.5, r=3.0, k=8)
    plan = _plan(p, dev, schedule=schedule)
    f = _cuda(p.f, dev)
    Rt, w, s = _single_mode_reference(p)
    plan.set_progress_limit(0)
    with pytest.raises(mg.MgwrError) as ei:
        plan.solve(f, tol=1e-10)
    assert ei.value.code == mg.MGWR_ERR_HIP and "stalled" in str(ei.value)
    plan.set_progress_limit(1 << 22)
    for rep in range(2):
        u, st = plan.solve(f, tol=1e-10)
        err = np.max(np.abs(u.cpu().numpy() - np.outer(w, s))) / np.max(np.abs(w))
        assert err < 1e-9, (rep, err, st)


@pytest.mark.parametrize("schedule", ["staged", "pipelined"])
def test_bfloat16_factors_change_the_inner_cycles_not_the_answer(dev, schedule):
    """The bfloat16 form runs different inner cycles from the float32 form (its
    low-rank factors carry about 3 significant digits), so after one
    refinement step the two iterates differ by more than float32 rounding
    explains; both converge to the float64 tolerance and to the oracle's
    solution."""
    p = W.manufactured(1, 255, 1024, 0.5, r=3.0, k=10)
    f = _cuda(p.f, dev)
    Rt, w, s = _single_mode_reference(p)
    ref = np.outer(w, s)
    one = {}
    for precision in ("mixed", "mixed_bf16"):
        plan = _plan(p, dev, precision=precision, schedule=schedule, max_cycles=1)
        u1, _ = plan.solve(f, tol=1e-14, allow_unconverged=True)
        one[precision] = u1.cpu().numpy()
        plan = _plan(p, dev, precision=precision, schedule=schedule)
        u, st = plan.solve(f, tol=1e-9)
        U = u.cpu().numpy()
        res = np.max(np.abs(oracle.residual(Rt, U, p.f, 1, p.n, 1.0)))
        assert res <= 1e-9 * st["bnorm"] * 1.01, (precision, st)
        assert np.max(np.abs(U - ref)) / np.max(np.abs(w)) < 1e-8, precision
    d = np.max(np.abs(one["mixed"] - one["mixed_bf16"])) / np.max(np.abs(ref))
    assert 1e-6 < d < 1e-1, d


@pytest.mark.parametrize("prefetch,coarse,precision", [(1, 1, "fp64"), (2, 1, "fp64"), (1, 2, "fp64"),
                                                       (2, 3, "fp64"), (1, 0, "fp64"), (2, 0, "mixed"),
                                                       (0, -1, "mixed")])
def test_staged_knobs_give_the_same_solution(dev, prefetch, coarse, precision):
    """Every march prefetch and coarse-launch level of the staged schedule
    (host-side choices of how the cycle's operators are launched) solves to
    the oracle's solution."""
    p = W.manufactured(2, 63, 256, 0.4, r=3.0, k=10)
    plan = _plan(p, dev, schedule="staged", precision=precision).set_staging(prefetch, coarse)
    print("case", prefetch, coarse, precision, plan.tuned(), flush=True)
    u, st = plan.solve(_cuda(p.f, dev), tol=1e-10)
    Rt, w, s = _single_mode_reference(p)
    ref = np.outer(w, s)
    assert np.max(np.abs(u.cpu().numpy() - ref)) / np.max(np.abs(ref)) < 1e-9, st


@pytest.mark.parametrize("schedule", ["staged", "pipelined"])
@pytest.mark.parametrize("dim,n,M,precision", [(1, 1, 1, "fp64"), (1, 7, 1, "fp64"), (2, 1, 3, "fp64"),
                                               (2, 3, 2, "fp64"), (1, 15, 5, "fp64"), (2, 7, 9, "mixed"),
                                               (1, 31, 1, "mixed")])
def test_degenerate_sizes(dev, schedule, dim, n, M, precision):
    """One time step, meshes shorter than one leaf, a one-point grid (the
    coarsest level is the finest): random source and initial value against
    the oracle's direct time stepping."""
    rng = np.random.default_rng([dim, n, M])
    N = n ** dim
    t = W.graded_mesh(M, 1.0, 2.0)
    p = W.Problem(dim=dim, n=n, M=M, alpha=0.55, r=2.0, k=6, t=t, f=rng.standard_normal((M, N)))
    print("case", schedule, dim, n, M, precision, flush=True)
    err, res, st = _solve_and_compare(p, dev, g=rng.standard_normal(N), schedule=schedule, precision=precision,
                                      tol=1e-11)
    assert err < 1e-9 and res < 1e-10, (err, res, st)


@pytest.mark.parametrize("dim,n,M,alpha,r,k", [(1, 63, 300, 0.4, 4.0, 8), (2, 31, 128, 0.6, 3.0, 10),
                                               (1, 1, 17, 0.5, 1.0, 4), (2, 15, 2048, 0.3, 17 / 3, 10)])
def test_apply_A_matches_oracle(dev, dim, n, M, alpha, r, k):
    """mgwr_apply_A: the float64 space-time operator (R~ in time plus the
    stencil) on a random iterate against the oracle's (Rt (x) I + I (x) A_h) U."""
    print(f"apply_A dim={dim} n={n} M={M}", flush=True)
    t = W.graded_mesh(M, 1.0, r)
    plan = mg.Plan(dim, n, M, alpha, k=k, t=t).bind()
    rng = np.random.default_rng([3, dim, n, M])
    U = rng.standard_normal((M, n ** dim))
    out = plan.apply_A(_cuda(U, dev)).cpu().numpy()
    Rt = oracle.hmatrix_dense(t, alpha, k)
    ref = -oracle.residual(Rt, U, np.zeros_like(U), dim, n, 1.0)
    assert np.max(np.abs(out - ref)) <= 1e-13 * np.max(np.abs(ref))
    x = _cuda(U, dev)
    rc = mg.lib().mgwr_apply_A(plan._h, mg.ctypes.c_void_p(x.data_ptr()), mg.ctypes.c_void_p(x.data_ptr()))
    assert rc == mg.MGWR_ERR_INVALID_ARG       # in place is refused


@pytest.mark.parametrize("schedule", ["staged", "pipelined"])
@pytest.mark.parametrize("dim,n,M,alpha,r,eta,cluster", [
    (1, 63, 512, 0.5, 3.0, 2.0, "index"), (1, 63, 300, 0.3, 17 / 3, 1.0, "geometric"),
    (2, 31, 256, 0.6, 3.0, 2.0, "geometric"), (2, 15, 128, 0.4, 4.0, 0.5, "index")])
def test_eta_and_geometric_clusters_solve_against_oracle(dev, schedule, dim, n, M, alpha, r, eta, cluster):
    """The general admissibility parameter and the geometric cluster tree
    change R~ (and with it the packed program: leaf sizes, far-field stacks,
    accumulator slots); the solve still matches the oracle built with the same
    choices to 1e-10."""
    print(f"eta={eta} cluster={cluster} dim={dim} n={n} M={M} {schedule}", flush=True)
    p = W.manufactured(dim, n, M, alpha, r=r, k=10)
    plan = mg.Plan(dim, n, M, alpha, k=10, t=p.t, eta=eta, cluster=cluster, schedule=schedule).bind()
    rng = np.random.default_rng([17, dim, n, M])
    F = rng.standard_normal((M, p.N))
    u, st = plan.solve(_cuda(F, dev), tol=1e-12)
    Rt = oracle.hmatrix_dense(p.t, alpha, 10, 16, eta=eta, cluster=cluster)
    ref = oracle.timestep_solve(Rt, F, dim, n, 1.0)
    U = u.cpu().numpy()
    assert np.max(np.abs(U - ref)) <= 1e-10 * np.max(np.abs(ref)), st
    res = np.max(np.abs(oracle.residual(Rt, U, F, dim, n, 1.0))) / np.max(np.abs(F))
    assert res <= 1.2e-12 + 1e-13


def test_stats_report_setup_and_solve_times(dev):
    p = W.config("small1d")
    plan = _plan(p, dev)
    u, st = plan.solve(_cuda(p.f, dev), tol=1e-10)
    assert st["setup_ms"] > 0.0 and st["solve_ms"] > 0.0
    assert st["solve_ms"] < 60e3 and np.isnan(st["warm_res0"])


@pytest.mark.parametrize("schedule,n", [("staged", 31), ("staged", 63), ("pipelined", 31)])
@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_bf16"])
def test_colour_split_storage_is_bit_identical_to_natural(dev, schedule, n, precision):
    """Colour-split storage moves points, not operations: in the pipelined
    schedule every point's arithmetic is the same in either storage, so the
    solutions (from zero and from a given iterate, with an initial value g)
    agree bit for bit.  The staged schedule in split storage forms its
    defects from the last half-sweep's changes (zebra defects), which equal
    the defect march's up to rounding: there the two solutions agree to the
    solve tolerance.  The float64 one matches the oracle either way."""
    rng = np.random.default_rng(77 + n)
    M, N = 80, n * n
    t = W.graded_mesh(M, 1.0, 3.0)
    p = W.Problem(dim=2, n=n, M=M, alpha=0.5, r=3.0, k=8, t=t, f=rng.standard_normal((M, N)))
    g = rng.standard_normal(N)
    u0 = rng.standard_normal((M, N))
    f, gd = _cuda(p.f, dev), _cuda(g, dev)
    tol = 1e-12 if precision == "fp64" else 1e-10
    out = {}
    for layout, code in (("natural", 0), ("split", 1)):
        print("case", schedule, n, precision, layout, flush=True)
        plan = _plan(p, dev, schedule=schedule, precision=precision).set_layout(layout)
        assert plan.info()["layout"] == code
        u, st = plan.solve(f, gd, tol=tol)
        ug = _cuda(u0, dev)
        _, st2 = plan.solve(f, gd, tol=tol, u=ug, guess=True)
        out[layout] = (u.cpu().numpy(), ug.cpu().numpy(), st["cycles"], st2["cycles"], st["res"])
    a, b = out["natural"], out["split"]
    if schedule == "pipelined":
        assert a[2:4] == b[2:4]
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    else:
        for x, y in ((a[0], b[0]), (a[1], b[1])):
            assert np.max(np.abs(x - y)) / np.max(np.abs(y)) < 100 * tol
        assert abs(a[2] - b[2]) <= 1 and abs(a[3] - b[3]) <= 1
    Rt = oracle.hmatrix_dense(p.t, p.alpha, p.k, p.leaf)
    B = oracle.rhs(p.f, p.t, p.alpha, g)
    ref = oracle.timestep_solve(Rt, B, p.dim, p.n, p.length)
    err = np.max(np.abs(b[0] - ref)) / np.max(np.abs(ref))
    res = np.max(np.abs(oracle.residual(Rt, b[1], B, p.dim, p.n, p.length))) / np.max(np.abs(B))
    assert err < (1e-10 if precision == "fp64" else 1e-8) and res <= 1.5 * tol, (err, res)
    if precision == "fp64":
        # the reported residual (a zebra stopping test in staged split
        # storage) is the oracle's residual of the returned iterate
        true_res = np.max(np.abs(oracle.residual(Rt, b[0], B, p.dim, p.n, p.length)))
        assert abs(b[4] - true_res) <= 0.1 * true_res + 1e-12 * np.max(np.abs(B)), (b[4], true_res)


def test_autotuner_times_both_storages(dev):
    """The autotuner's last candidate is its best schedule in the other
    storage; whatever it keeps, the plan reports it and still solves to the
    oracle's solution."""
    p = W.manufactured(2, 63, 128, 0.5, r=3.0, k=8)
    plan = _plan(p, dev)
    f = _cuda(p.f, dev)
    plan.autotune(f, tol=1e-10)
    assert plan.info()["layout"] in (0, 1)
    u, st = plan.solve(f, tol=1e-10)
    Rt, w, s = _single_mode_reference(p)
    ref = np.outer(w, s)
    assert np.max(np.abs(u.cpu().numpy() - ref)) / np.max(np.abs(ref)) < 1e-9, st


@pytest.mark.parametrize("dim,n,M,alpha", [(2, 31, 96, 0.5), (2, 63, 64, 0.3), (1, 127, 256, 0.7), (1, 63, 128, 0.5)])
def test_zebra_defects_match_defect_marches(dev, dim, n, M, alpha):
    """Zebra defects (the restriction's defect from the changes of the last
    second-colour half-sweep; 2D staged in colour-split storage, the
    pipelined cycles in either storage) against the defect marches of
    Algorithm 3 (the staged levels in natural storage, the 1D staged
    cycle): the same
    cycle counts within one, both solutions at the oracle's, and the
    reported residual (a zebra stopping test in 2D) equal to the oracle's
    residual of the returned iterate.  Below a tolerance of 1e-10 the
    library uses the defect marches, which the bit-identity of the two 2D
    storages at 1e-12 shows."""
    rng = np.random.default_rng(300 + n)
    N = n ** dim
    t = W.graded_mesh(M, 1.0, (2 - alpha) / alpha)
    p = W.Problem(dim=dim, n=n, M=M, alpha=alpha, r=(2 - alpha) / alpha, k=8, t=t, f=rng.standard_normal((M, N)))
    f = _cuda(p.f, dev)
    Rt = oracle.hmatrix_dense(p.t, p.alpha, p.k, p.leaf)
    B = oracle.rhs(p.f, p.t, p.alpha, None)
    ref = oracle.timestep_solve(Rt, B, p.dim, p.n, p.length)
    bn = np.max(np.abs(B))
    # zebra form, and the same cycle with defect marches
    if dim == 2:
        forms = {"zebra": dict(schedule="staged", layout="split"),
                 "zebra_pipelined": dict(schedule="pipelined", layout="split"),
                 "zebra_pipelined_natural": dict(schedule="pipelined", layout="natural"),
                 "march": dict(schedule="staged", layout="natural")}
    else:
        forms = {"zebra": dict(schedule="pipelined"), "march": dict(schedule="staged")}
    out = {}
    for name, kw in forms.items():
        print("case", dim, n, M, alpha, name, flush=True)
        plan = _plan(p, dev, schedule=kw["schedule"])
        if "layout" in kw:
            plan.set_layout(kw["layout"])
        u, st = plan.solve(f, tol=1e-10)
        un = u.cpu().numpy()
        true_res = np.max(np.abs(oracle.residual(Rt, un, B, p.dim, p.n, p.length)))
        err = np.max(np.abs(un - ref)) / np.max(np.abs(ref))
        assert true_res <= 1.5e-10 * bn and err < 1e-8, (name, true_res / bn, err)
        assert abs(st["res"] - true_res) <= 0.1 * true_res + 1e-13 * bn, (name, st["res"], true_res)
        out[name] = (un, st["cycles"])
    for name in out:
        assert abs(out[name][1] - out["march"][1]) <= 1, name
        diff = np.max(np.abs(out[name][0] - out["march"][0])) / np.max(np.abs(ref))
        assert diff < 1e-8, (name, diff)
