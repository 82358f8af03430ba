"""GPU tests of batching: merged launches of uneven instances, graph replay,
the schedule autotuner, and the batched random-Fourier family checked mode by
mode against the float64 oracle (the source is a sum of separable sine
modes, so the exact discrete solution is the sum of one triangular solve per
mode)."""
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


def _cuda(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def _plan(p, **kw):
    return mg.Plan(p.dim, p.n, p.M, p.alpha, k=p.k, r=p.r, t=p.t, length=p.length, leaf=p.leaf, **kw).bind()


def _modewise_reference(p):
    """Exact discrete solution of a multi-mode source with the same R~."""
    Rt = oracle.hmatrix_dense(p.t, p.alpha, p.k, p.leaf)
    U = np.zeros((p.M, p.N))
    for kvec, prof in p.modes:
        w = oracle.single_mode_profile(Rt, oracle.mode_eigenvalue(kvec, p.n, p.length), prof)
        U += np.outer(w, W.sine_mode(p.n, p.dim, p.length, kvec))
    return U


def _family(count, seed, sides, Ms):
    return W.batched_instances(count=count, seed=seed, sides=sides, Ms=Ms, k=10)


def _check(p, u, ref, tol, fp64=True):
    """Solution error against the oracle (float64 plans: 1e-10 relative;
    mixed plans: 1e-7) and the oracle's own float64 residual of the result."""
    U = u.cpu().numpy()
    err = np.abs(U - ref).max() / np.abs(ref).max()
    Rt = oracle.hmatrix_dense(p.t, p.alpha, p.k, p.leaf)
    B = oracle.rhs(p.f, p.t, p.alpha, p.g)
    res = np.abs(oracle.residual(Rt, U, B, p.dim, p.n, p.length)).max() / np.abs(B).max()
    assert err < (1e-10 if fp64 else 1e-7), (p.dim, p.n, p.M, p.alpha, err)
    # the library's stopping test and the oracle's residual agree up to rounding
    assert res <= 1.2 * tol + 1e-13, (p.dim, p.n, p.M, res)
    return err, res


def test_batched_random_fourier_family_matches_oracle(dev):
    """Uneven 2D instances of the batched family (sides 15/31/63, M 64..256)
    in one batch: every solution against the mode-by-mode oracle."""
    probs = _family(6, 20261203, sides=(15, 31, 63), Ms=(64, 128, 256))
    print("instances", [(p.n, p.M, round(p.alpha, 3)) for p in probs], flush=True)
    plans = [_plan(p) for p in probs]
    batch = mg.Batch(plans).bind()
    fs = [_cuda(p.f, dev) for p in probs]
    for rep in range(2):
        us, sts = batch.solve(fs, tol=1e-12)
        for p, u, st in zip(probs, us, sts):
            _check(p, u, _modewise_reference(p), 1e-12)
            assert st["res"] <= 1e-12 * st["bnorm"]


def test_graph_replay_matches_eager(dev):
    """The same batch solved repeatedly with graph replay on, other eager work
    in between: every replay equals the eager batch's result."""
    cases = [(1, 63, 128, 0.5), (2, 15, 64, 0.3), (1, 127, 256, 0.7)]
    probs = [W.manufactured(d, n, M, a, k=8) for d, n, M, a in cases]
    fs = [_cuda(p.f, dev) for p in probs]
    eager = mg.Batch([_plan(p) for p in probs]).bind()
    graph = mg.Batch([_plan(p) for p in probs], graph=True).bind()
    other_p = W.manufactured(1, 31, 64, 0.4, k=6)
    other = _plan(other_p)
    ref_us = None
    ue_arr = [torch.empty_like(f) for f in fs]
    ug_arr = [torch.empty_like(f) for f in fs]   # fixed arrays: an unchanged launch can be replayed
    for rep in range(5):
        us_e, st_e = eager.solve(fs, tol=1e-12, us=ue_arr)
        us_g, st_g = graph.solve(fs, tol=1e-12, us=ug_arr)
        other.solve(_cuda(other_p.f, dev), tol=1e-12)     # unrelated eager work between replays
        torch.cuda.synchronize()
        for ue, ug, se, sg in zip(us_e, us_g, st_e, st_g):
            assert torch.equal(ue, ug), rep
            assert se["cycles"] == sg["cycles"] and se["res"] == sg["res"]
        if ref_us is None:
            ref_us = [_modewise_reference(p) for p in probs]
        for p, u, r in zip(probs, us_g, ref_us):
            _check(p, u, r, 1e-12)
    assert graph.graph_replays() >= 2
    assert eager.graph_replays() == 0


def test_autotune_picks_a_schedule_and_later_plans_follow(dev):
    p = W.manufactured(1, 255, 512, 0.5, k=10)
    f = _cuda(p.f, dev)
    plan = _plan(p)
    chosen = plan.autotune(f, tol=5e-11)
    assert chosen in ("staged", "pipelined")
    # h = 1/256: the float64 residual floor is near 6e-12, so 5e-11 is reachable
    u, st = plan.solve(f, tol=5e-11)
    _check(p, u, _modewise_reference(p), 5e-11)
    # a new AUTO plan of the same shape uses the measured schedule
    plan2 = _plan(p)
    plan2.timing(True)
    plan2.solve(f, tol=5e-11)
    tm = plan2.timing()
    assert (tm["pipe64"]["launches"] > 0) == (chosen == "pipelined"), (chosen, tm)
    assert plan.tuned()["schedule"] == chosen and plan2.tuned() == plan.tuned()


def test_autotune_of_a_staged_shape_keeps_its_knobs(dev):
    """A 2D shape where the staged schedule wins: the tuned prefetch and
    coarse level are among the candidates, later AUTO plans of the shape take
    them, and their solutions match the oracle."""
    p = W.manufactured(2, 127, 256, 0.5, r=3.0, k=8)
    f = _cuda(p.f, dev)
    plan = _plan(p)
    # 2D h = 1/128: the float64 residual floor is near 1.5e-12, so 1e-11
    chosen = plan.autotune(f, tol=1e-11)
    t = plan.tuned()
    print("tuned", chosen, t, flush=True)
    assert t["schedule"] == chosen
    if chosen == "staged":
        assert t["prefetch"] in ("shallow", "deep") and t["coarse_level"] in (1, 2, 3)
    plan2 = _plan(p)
    assert plan2.tuned() == t
    ref = _modewise_reference(p)
    for pl in (plan, plan2):
        u, st = pl.solve(f, tol=1e-11)
        _check(p, u, ref, 1e-11)


def test_batch_runs_staged_and_pipelined_instances(dev):
    probs = [W.manufactured(1, 63, 128, 0.5, k=8), W.manufactured(2, 31, 128, 0.6, r=3.0, k=8),
             W.manufactured(1, 127, 256, 0.4, k=10)]
    plans = [_plan(probs[0], schedule="staged"), _plan(probs[1]), _plan(probs[2], schedule="staged")]
    batch = mg.Batch(plans).bind()
    us, sts = batch.solve([_cuda(p.f, dev) for p in probs], tol=1e-12)
    for p, u, st in zip(probs, us, sts):
        _check(p, u, _modewise_reference(p), 1e-12)
        assert st["res"] <= 1e-12 * st["bnorm"]


def test_batch_of_mixed_plans_with_several_inner_cycles(dev):
    """A pipelined batch whose refinement steps hold 3 float32 cycles each
    (the launch's stage table grows with the inner cycles)."""
    probs = [W.manufactured(1, 127, 512, a, k=10) for a in (0.4, 0.6)]
    plans = [_plan(p, precision="mixed", inner_cycles=3, schedule="pipelined") for p in probs]
    batch = mg.Batch(plans).bind()
    for rep in range(2):
        us, sts = batch.solve([_cuda(p.f, dev) for p in probs], tol=1e-9)
        for p, u, st in zip(probs, us, sts):
            _check(p, u, _modewise_reference(p), 1e-9, fp64=False)
            assert st["res"] <= 1e-9 * st["bnorm"] and st["cycles"] % 3 == 0


def test_staged_instances_solved_side_by_side(dev):
    """Five staged instances (1D and 2D, float64 and mixed precision, uneven
    sizes) and one pipelined one in a batch: the staged ones are solved by
    several host threads, each on a stream of its own; every solution against
    the oracle, twice in a row."""
    cases = [(2, 63, 128, 0.5, "fp64"), (1, 255, 256, 0.4, "fp64"), (2, 31, 64, 0.6, "mixed"),
             (1, 127, 512, 0.7, "fp64"), (2, 63, 256, 0.3, "mixed")]
    probs = [W.manufactured(d, n, M, a, r=3.0, k=8) for d, n, M, a, _ in cases]
    plans = [_plan(p, schedule="staged", precision=c[4]) for p, c in zip(probs, cases)]
    pp = W.manufactured(1, 63, 128, 0.5, k=8)
    probs.append(pp)
    plans.append(_plan(pp, schedule="pipelined"))
    batch = mg.Batch(plans).bind()
    fs = [_cuda(p.f, dev) for p in probs]
    refs = [_modewise_reference(p) for p in probs]
    kinds = [c[4] for c in cases] + ["fp64"]
    for rep in range(2):
        # 1D h = 1/256 has its float64 residual floor near 6e-12
        us, sts = batch.solve(fs, tol=1e-11)
        for p, u, st, ref, kind in zip(probs, us, sts, refs, kinds):
            _check(p, u, ref, 1e-11, fp64=kind == "fp64")
            assert st["res"] <= 1e-11 * st["bnorm"], (rep, st)


def test_batch_holding_one_plan_twice(dev):
    """Two entries on one plan (one workspace) are solved one after the other."""
    p = W.manufactured(2, 63, 128, 0.5, k=8)
    plan = _plan(p, schedule="staged")
    batch = mg.Batch([plan, plan]).bind()
    us, sts = batch.solve([_cuda(p.f, dev), _cuda(2.0 * p.f, dev)], tol=1e-12)
    ref = _modewise_reference(p)
    for u, scale in zip(us, (1.0, 2.0)):
        assert np.abs(u.cpu().numpy() - scale * ref).max() <= 1e-10 * scale * np.abs(ref).max()


def test_stall_in_one_side_by_side_instance_is_reported(dev):
    """A zero progress bound on one of three staged plans: its coarse launch
    stops and the batch reports the stall; the others are unaffected, and with
    the bound restored the whole batch solves correctly."""
    probs = [W.manufactured(2, 63, 128, a, r=3.0, k=8) for a in (0.3, 0.5, 0.7)]
    plans = [_plan(p, schedule="staged") for p in probs]
    batch = mg.Batch(plans).bind()
    fs = [_cuda(p.f, dev) for p in probs]
    plans[1].set_progress_limit(0)
    with pytest.raises(mg.MgwrError) as ei:
        batch.solve(fs, tol=1e-12)
    assert ei.value.code == mg.MGWR_ERR_HIP and "stalled" in str(ei.value)
    plans[1].set_progress_limit(1 << 22)
    us, sts = batch.solve(fs, tol=1e-12)
    for p, u in zip(probs, us):
        _check(p, u, _modewise_reference(p), 1e-12)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_xcd_queues_give_the_same_results(dev, precision):
    """Pipelined launches deal their work items to per-XCD queues by default
    (the dispatch order checked on the device) or take them from one global
    ticket: the same stages run the same arithmetic either way, so batched
    and single solves agree bit for bit, and match the oracle."""
    probs = [W.manufactured(1, 127, 512, a, r=(2 - a) / a, k=8) for a in (0.3, 0.5, 0.7)]
    probs.append(W.manufactured(2, 31, 128, 0.4, r=3.0, k=8))
    plans = [_plan(p, schedule="pipelined", precision=precision) for p in probs]
    fs = [_cuda(p.f, dev) for p in probs]
    batch = mg.Batch(plans).bind()
    out = {}
    for on in (True, False):
        prev = mg.set_xcd_queues(on)
        try:
            assert plans[0].xcd_queues_in_use() == on
            us, sts = batch.solve(fs, tol=1e-11)
            u1, st1 = plans[0].solve(fs[0], tol=1e-11)
            out[on] = ([u.cpu().numpy() for u in us], [s["cycles"] for s in sts], u1.cpu().numpy(), st1["cycles"])
        finally:
            mg.set_xcd_queues(prev)
    a, b = out[True], out[False]
    assert a[1] == b[1] and a[3] == b[3]
    assert all(np.array_equal(x, y) for x, y in zip(a[0], b[0])) and np.array_equal(a[2], b[2])
    for p, u in zip(probs, a[0]):
        ref = _modewise_reference(p)
        err = np.abs(u - ref).max() / np.abs(ref).max()
        assert err < (1e-10 if precision == "fp64" else 1e-8), (p.name, err)
