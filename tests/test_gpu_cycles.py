"""GPU iterates after a fixed number of cycles against the oracle's cycle
(Algorithm 2 written out, oracle/mgwr.py), float64, element by element.

The other parity tests compare converged solutions with the direct solution;
these compare the iterate itself after one, two and three cycles, so a cycle
that still converges but computes a different iteration (a transfer weight, a
colour order, a coarse operator, the defect formed from the last half-sweep's
changes) fails here.  Every float64 form of the cycle is covered: staged and
pipelined schedules, colour-split and natural storage (2D), the defect marches
(tolerance below 1e-10) and the zebra defects (tolerance 1e-8), V and W
cycles with several smoothing counts, from zero and from a random iterate.
"""
import numpy as np
import pytest

import oracle
import oracle.mgwr as omg
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1706_07632_amd as mg  # noqa: E402  (fails loudly if the library is missing)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


# dim, n, M, alpha, r, k, nu1, nu2, gamma, with_g
CASES = {
    "1d_v11": (1, 63, 128, 0.5, 3.0, 8, 1, 1, 1, False),
    "1d_w21": (1, 127, 96, 0.3, 17 / 3, 10, 2, 1, 2, True),
    "1d_v01": (1, 63, 80, 0.7, 2.0, 8, 0, 1, 1, False),
    "2d_v11": (2, 31, 64, 0.4, 3.0, 10, 1, 1, 1, False),
    "2d_w11": (2, 15, 48, 0.6, 2.5, 8, 1, 1, 2, True),
    "2d_v10": (2, 31, 40, 0.5, 3.0, 8, 1, 0, 1, False),
    # time leaves shorter than 16 (M = 37: leaves of 9, 9, 9 and 10 levels;
    # M = 33: 16, 8 and 9) and a 3 x 3 grid whose next level is the
    # one-point coarsest grid
    "1d_ragged": (1, 31, 37, 0.45, 2.5, 6, 1, 1, 1, True),
    "2d_ragged": (2, 7, 33, 0.55, 2.0, 6, 1, 1, 1, True),
    "2d_n3_w": (2, 3, 20, 0.5, 2.0, 6, 1, 1, 2, False),
}
FORMS = [(s, lay, tol) for s in ("staged", "pipelined") for lay in ("split", "natural") for tol in (1e-8, 1e-14)]


def _params():
    out = []
    for name, c in CASES.items():
        for s, lay, tol in FORMS:
            if c[0] == 1 and lay == "natural":
                continue            # 1D has one storage
            out.append(pytest.param(name, s, lay, tol, id=f"{name}-{s}-{lay if c[0] == 2 else '1d'}-{tol:g}"))
    return out


def _problem(name):
    dim, n, M, alpha, r, k, nu1, nu2, gamma, with_g = CASES[name]
    rng = np.random.default_rng(sum(map(ord, name)))
    t = W.graded_mesh(M, 1.0, r)
    N = n ** dim
    f = rng.standard_normal((M, N))
    g = rng.standard_normal(N) if with_g else None
    U0 = rng.standard_normal((M, N))
    Rt = oracle.hmatrix_dense(t, alpha, k, 16)
    B = oracle.rhs(f, t, alpha, g)
    return dict(dim=dim, n=n, M=M, alpha=alpha, k=k, t=t, nu1=nu1, nu2=nu2, gamma=gamma, f=f, g=g, U0=U0,
                Rt=Rt, B=B)


def _cuda(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("name,schedule,layout,tol", _params())
def test_iterates_match_the_oracle_cycle(dev, name, schedule, layout, tol):
    P = _problem(name)
    dim, n = P["dim"], P["n"]
    print("case", name, schedule, layout, tol, flush=True)
    kw = dict(k=P["k"], t=P["t"], nu1=P["nu1"], nu2=P["nu2"], gamma=P["gamma"], schedule=schedule)
    okw = dict(nu1=P["nu1"], nu2=P["nu2"], gamma=P["gamma"])
    f = _cuda(P["f"], dev)
    g = None if P["g"] is None else _cuda(P["g"], dev)
    # three cycles from zero, in one solve
    plan = mg.Plan(dim, n, P["M"], P["alpha"], max_cycles=3, **kw)
    if dim == 2:
        plan.set_layout(layout)
    plan.bind()
    u, st = plan.solve(f, g, tol=tol, allow_unconverged=True)
    assert st["cycles"] == 3, st
    ref3 = omg.cycles(P["Rt"], P["B"], dim, n, 1.0, 3, **okw)[-1]
    e3 = _rel(u.cpu().numpy(), ref3)
    plan.close()
    # one cycle at a time from a random iterate, each against the oracle's
    # cycle from the library's previous iterate
    plan = mg.Plan(dim, n, P["M"], P["alpha"], max_cycles=1, **kw)
    if dim == 2:
        plan.set_layout(layout)
    plan.bind()
    U = P["U0"]
    worst = 0.0
    for c in range(2):
        u = _cuda(U, dev)
        _, st = plan.solve(f, g, tol=tol, u=u, guess=True, allow_unconverged=True)
        assert st["cycles"] == 1, st
        want = omg.cycle(P["Rt"], U, P["B"], dim, n, 1.0, **okw)
        U = u.cpu().numpy()
        worst = max(worst, _rel(U, want))
    plan.close()
    print(f"{name} {schedule} {layout} tol={tol:g}: three cycles from zero {e3:.2e}, "
          f"single cycles from a random iterate {worst:.2e}", flush=True)
    assert e3 < 1e-10 and worst < 1e-10, (e3, worst)


MIXED = [pytest.param(name, s, lay, inner, id=f"{name}-{s}-{lay if CASES[name][0] == 2 else '1d'}-inner{inner}")
         for name in ("1d_v11", "1d_w21", "2d_v11", "2d_w11") for s in ("staged", "pipelined")
         for lay in (("split", "natural") if CASES[name][0] == 2 else ("split",)) for inner in (1, 2)]


@pytest.mark.parametrize("name,schedule,layout,inner", MIXED)
def test_float32_inner_cycles_follow_the_oracle_cycle(dev, name, schedule, layout, inner):
    """Float32 inner cycles on A e = r with the float64 residual between them:
    a cycle is affine, u + cycle(0, b - A u) = cycle(u, b), so after c inner
    cycles in all (however they are grouped into refinement steps) the iterate
    is the oracle's after c cycles up to float32 rounding.  Bound: a float32
    cycle's line solves of M <= 128 unknowns lose about M eps_32 = 8e-6
    relative, and the contracting iteration does not amplify earlier losses
    beyond a factor 1 / (1 - rho) < 2 here: 1e-4 leaves a margin of 6."""
    P = _problem(name)
    dim, n = P["dim"], P["n"]
    print("case", name, schedule, layout, "inner", inner, flush=True)
    okw = dict(nu1=P["nu1"], nu2=P["nu2"], gamma=P["gamma"])
    plan = mg.Plan(dim, n, P["M"], P["alpha"], k=P["k"], t=P["t"], nu1=P["nu1"], nu2=P["nu2"], gamma=P["gamma"],
                   schedule=schedule, precision="mixed", inner_cycles=inner, max_cycles=3)
    if dim == 2:
        plan.set_layout(layout)
    plan.bind()
    f = _cuda(P["f"], dev)
    g = None if P["g"] is None else _cuda(P["g"], dev)
    u, st = plan.solve(f, g, tol=1e-8, allow_unconverged=True)
    plan.close()
    c = st["cycles"]
    assert 1 <= c <= 3, st
    ref = omg.cycles(P["Rt"], P["B"], dim, n, 1.0, c, **okw)[-1]
    e = _rel(u.cpu().numpy(), ref)
    print(f"{name} {schedule} {layout} inner={inner}: {c} float32 cycles ({st['refinements']} refinements), "
          f"relative difference to the oracle's float64 iterate {e:.2e}", flush=True)
    assert e < 1e-4, (c, e)


BATCH = [  # dim, n, M, alpha, r, k, schedule, with_g
    (1, 63, 96, 0.5, 3.0, 8, "pipelined", False),
    (2, 15, 64, 0.3, 17 / 3, 10, "pipelined", True),
    (2, 31, 48, 0.7, 2.0, 8, "staged", False),
    (1, 127, 64, 0.4, 4.0, 10, "staged", True),
    (2, 31, 80, 0.6, 2.5, 10, "pipelined", False),
    (2, 15, 32, 0.5, 3.0, 8, "staged", False),
]


@pytest.mark.parametrize("tol", [1e-8, 1e-14])
def test_batch_iterates_match_the_oracle_cycle(dev, tol):
    """Uneven instances in one batch (the pipelined ones merged into one
    graph-replayed launch, the staged ones side by side on their own streams),
    two cycles each, twice in a row (the second solve replays the captured
    launch): every instance's iterate against the oracle's two cycles."""
    rng = np.random.default_rng(77)
    probs, plans = [], []
    for dim, n, M, alpha, r, k, sched, with_g in BATCH:
        t = W.graded_mesh(M, 1.0, r)
        N = n ** dim
        f = rng.standard_normal((M, N))
        g = rng.standard_normal(N) if with_g else None
        Rt = oracle.hmatrix_dense(t, alpha, k, 16)
        ref = omg.cycles(Rt, oracle.rhs(f, t, alpha, g), dim, n, 1.0, 2)[-1]
        probs.append((f, g, ref))
        plans.append(mg.Plan(dim, n, M, alpha, k=k, t=t, schedule=sched, max_cycles=2).bind())
    batch = mg.Batch(plans, graph=True).bind()
    fs = [_cuda(f, dev) for f, _, _ in probs]
    gs = [None if g is None else _cuda(g, dev) for _, g, _ in probs]
    us = [torch.empty_like(f) for f in fs]
    for rep in range(2):
        us, sts = batch.solve(fs, gs, tol=tol, us=us, allow_unconverged=True)
        errs = [_rel(u.cpu().numpy(), ref) for u, (_, _, ref) in zip(us, probs)]
        print(f"tol={tol:g} solve {rep}: cycles {[s['cycles'] for s in sts]}, relative differences "
              + " ".join(f"{e:.1e}" for e in errs), flush=True)
        assert all(s["cycles"] == 2 for s in sts), sts
        assert max(errs) < 1e-10, errs
    print("graph replays", batch.graph_replays(), flush=True)
    assert batch.graph_replays() >= 1
    batch.close()
    for pl in plans:
        pl.close()


def test_full_side_by_side_batch_iterates_match_the_oracle_cycle(dev):
    """Ten staged instances (at least one per worker thread: their coarse
    pipelined launch then starts one level below the single-solve rule) and
    two pipelined ones, two cycles each, against the oracle's two cycles."""
    rng = np.random.default_rng(91)
    shapes = [(2, 31, 32), (2, 31, 48), (2, 31, 40), (2, 63, 32), (2, 31, 64), (2, 31, 36),
              (1, 127, 48), (1, 63, 64), (1, 255, 32), (1, 127, 40)]
    probs, plans = [], []
    for j, (dim, n, M) in enumerate(shapes + [(2, 15, 48), (1, 31, 64)]):
        alpha = float(rng.uniform(0.25, 0.85))
        t = W.graded_mesh(M, 1.0, (2 - alpha) / alpha)
        N = n ** dim
        f = rng.standard_normal((M, N))
        Rt = oracle.hmatrix_dense(t, alpha, 8, 16)
        ref = omg.cycles(Rt, oracle.rhs(f, t, alpha, None), dim, n, 1.0, 2)[-1]
        probs.append((f, ref))
        plans.append(mg.Plan(dim, n, M, alpha, k=8, t=t, max_cycles=2,
                             schedule="staged" if j < len(shapes) else "pipelined").bind())
    batch = mg.Batch(plans, graph=True).bind()
    fs = [_cuda(f, dev) for f, _ in probs]
    us = [torch.empty_like(f) for f in fs]
    for rep in range(2):
        us, sts = batch.solve(fs, tol=1e-8, us=us, allow_unconverged=True)
        errs = [_rel(u.cpu().numpy(), ref) for u, (_, ref) in zip(us, probs)]
        print(f"solve {rep}: worst relative difference {max(errs):.2e}", flush=True)
        assert all(s["cycles"] == 2 for s in sts), sts
        assert max(errs) < 1e-10, errs
    batch.close()
    for pl in plans:
        pl.close()
