"""GPU parity of the learned initial guess (through the C ABI) against the
float64 network oracle, and the warm-started solve judged by the oracle.

Weights are rounded to bfloat16 on the host first, so that the library's
bfloat16 copies are exact.  Inference runs on the bfloat16 matrix cores, which
round every convolution input to bfloat16: it is compared with the oracle
that rounds at the same place (act_bf16).  Both sides take that rounding from
float32 sums accumulated in different orders, so an activation next to a
rounding boundary can land one bfloat16 step apart; the bound FWD_TOL covers a
few such flips, and every check also asserts that the output is much closer to
the rounding oracle than to the unrounded one (a wrong operand layout or a
missing rounding fails that).  Training runs the float32 kernels; its
gradient is compared with the unrounded oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import net as N

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1706_07632_amd as mg  # noqa: E402
from paper_1706_07632_amd import learn  # noqa: E402


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def bf16_params(channels, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    out = np.zeros(N.param_count(channels), dtype=np.float32)
    off = 0
    for cin, cout in zip(channels[:-1], channels[1:]):
        nw = cout * cin * 9
        out[off:off + nw] = rng.uniform(-1, 1, nw) * np.sqrt(3.0 / (cin * 9)) * scale
        out[off + nw:off + nw + cout] = rng.uniform(-0.1, 0.1, cout)
        off += nw + cout
    return N.bf16_round(out)


FWD_TOL = 4e-4


def assert_inference_matches(y, params, channels, x, nsig, h, h_min=0.0):
    ref = N.forward(params.astype(np.float64), channels, x.astype(np.float64), nsig, h, h_min=h_min, act_bf16=True)
    plain = N.forward(params.astype(np.float64), channels, x.astype(np.float64), nsig, h, h_min=h_min)
    scale = np.abs(ref).max()
    err = np.abs(y - ref).max() / scale
    err_plain = np.abs(y - plain).max() / scale
    print(f"  inference vs rounding oracle {err:.2e}, vs unrounded oracle {err_plain:.2e}", flush=True)
    assert err <= FWD_TOL, err
    assert np.median(np.abs(y - ref)) <= 1e-5 * scale
    assert err < 0.25 * err_plain, (err, err_plain)


def make(channels, nsig, params, max_bhw):
    net = mg.Net(channels, nsig, max_bhw)
    net.set_params(params)
    return net


CASES = [
    # channels, nsignal, B, H, W
    ([6, 8, 8, 3], 3, 2, 1, 31),
    ([6, 8, 8, 3], 3, 2, 15, 15),
    ([35, 64, 64, 64, 32], 32, 2, 1, 255),
    ([35, 64, 64, 64, 32], 32, 1, 31, 31),
]


@pytest.mark.parametrize("channels,nsig,B,H,W", CASES)
def test_forward_matches_oracle(dev, channels, nsig, B, H, W):
    print(f"forward {channels} B={B} H={H} W={W}", flush=True)
    p = bf16_params(channels, 11)
    net = make(channels, nsig, p, B * H * W)
    rng = np.random.default_rng(12)
    x = rng.standard_normal((B, channels[0] - 1, H, W)).astype(np.float32)
    h = 1.0 / (W + 1)
    y = net.forward(torch.as_tensor(x, device=dev), h).cpu().numpy()
    assert_inference_matches(y, p, channels, x, nsig, h)


@pytest.mark.parametrize("H,W", [(1, 63), (15, 15)])
def test_finest_level_cutoff_matches_oracle(dev, H, W):
    channels, nsig, B = [6, 8, 8, 3], 3, 2
    p = bf16_params(channels, 13)
    net = make(channels, nsig, p, B * H * W)
    h = 1.0 / (W + 1)
    net.set_finest(2 * h)   # the finest level is left out
    rng = np.random.default_rng(14)
    x = rng.standard_normal((B, channels[0] - 1, H, W)).astype(np.float32)
    t = rng.standard_normal((B, channels[-1], H, W)).astype(np.float32) * 1e-3
    xd, td = torch.as_tensor(x, device=dev), torch.as_tensor(t, device=dev)
    y = net.forward(xd, h).cpu().numpy()
    assert_inference_matches(y, p, channels, x, nsig, h, h_min=2 * h)
    _, g = net.gradient(xd, td, h)
    _, rg = N.gradient(p.astype(np.float64), channels, x.astype(np.float64), t.astype(np.float64), nsig, h,
                       h_min=2 * h)
    assert np.abs(g.cpu().numpy() - rg).max() <= 1e-3 * np.abs(rg).max()


@pytest.mark.parametrize("channels,nsig,B,H,W", CASES)
def test_gradient_matches_oracle(dev, channels, nsig, B, H, W):
    print(f"gradient {channels} B={B} H={H} W={W}", flush=True)
    p = bf16_params(channels, 21)
    net = make(channels, nsig, p, B * H * W)
    rng = np.random.default_rng(22)
    x = rng.standard_normal((B, channels[0] - 1, H, W)).astype(np.float32)
    t = rng.standard_normal((B, channels[-1], H, W)).astype(np.float32) * 1e-3
    h = 1.0 / (W + 1)
    loss, g = net.gradient(torch.as_tensor(x, device=dev), torch.as_tensor(t, device=dev), h)
    g = g.cpu().numpy().astype(np.float64)
    rloss, rg = N.gradient(p.astype(np.float64), channels, x.astype(np.float64), t.astype(np.float64), nsig, h)
    assert abs(loss - rloss) <= 1e-4 * rloss
    # per layer: float32 sums over B*H*W products
    off = 0
    for cin, cout in zip(channels[:-1], channels[1:]):
        for lo, cnt in ((off, cout * cin * 9), (off + cout * cin * 9, cout)):
            a, b = g[lo:lo + cnt], rg[lo:lo + cnt]
            assert np.abs(a - b).max() <= 1e-3 * np.abs(b).max() + 1e-30, (cin, cout, np.abs(a - b).max())
        off += cout * cin * 9 + cout


def test_adam_step_matches_oracle(dev):
    channels, nsig = [6, 8, 3], 3
    p = bf16_params(channels, 31)
    net = make(channels, nsig, p, 2 * 31)
    rng = np.random.default_rng(32)
    x = torch.as_tensor(rng.standard_normal((2, 5, 1, 31)).astype(np.float32), device=dev)
    t = torch.as_tensor(rng.standard_normal((2, 3, 1, 31)).astype(np.float32), device=dev)
    h = 1.0 / 32
    m = np.zeros(p.size)
    v = np.zeros(p.size)
    pr = p.astype(np.float64)
    for step in (1, 2, 3):
        _, g = net.gradient(x, t, h)
        g = g.cpu().numpy().astype(np.float64)
        net.step = step - 1
        net.train_step(x, t, h, lr=1e-2)
        pr, m, v = N.adam_step(pr, g, m, v, step, lr=1e-2)
        dp = net.params.cpu().numpy().astype(np.float64)
        assert np.abs(dp - pr).max() <= 1e-5 * np.abs(pr).max()
        pr = dp  # follow the device's float32 master weights
    # the bfloat16 copies of the weights were refreshed by the update (biases stay float32)
    y = net.forward(x, h).cpu().numpy()
    pw = net.params.cpu().numpy().copy()
    off = 0
    for cin, cout in zip(channels[:-1], channels[1:]):
        pw[off:off + cout * cin * 9] = N.bf16_round(pw[off:off + cout * cin * 9])
        off += cout * cin * 9 + cout
    assert_inference_matches(y, pw, channels, x.cpu().numpy(), nsig, h)


def test_net_rejects_bad_shapes(dev):
    net = make([6, 4, 3], 3, bf16_params([6, 4, 3], 1), 64)
    with pytest.raises(mg.MgwrError):
        net.forward(torch.zeros((1, 5, 1, 30), dtype=torch.float32, device=dev), 0.1)   # W not 2^p - 1
    with pytest.raises(mg.MgwrError):
        net.forward(torch.zeros((1, 5, 3, 7), dtype=torch.float32, device=dev), 0.1)    # H neither 1 nor W
    with pytest.raises(mg.MgwrError):
        net.forward(torch.zeros((1, 5, 1, 127), dtype=torch.float32, device=dev), 0.1)  # over capacity


def _problem(dim, n, M, seed):
    return W.warm_start_family(dim, n, M, np.random.default_rng([seed, 0]), k=8)


def _plan(p, **kw):
    return mg.Plan(p.dim, p.n, p.M, p.alpha, k=p.k, r=p.r, t=p.t, **kw).bind()


def _oracle_guess(p, params, channels, plan):
    """Oracle of the predicted iterate and its float64 residual norm."""
    rows = learn.slice_rows(p.M)
    b = oracle.rhs(p.f, p.t, p.alpha, None)
    x, scale = N.warm_start_input(b, rows, p.alpha, p.r, p.dim, p.n)
    y = N.forward(params.astype(np.float64), channels, x.astype(np.float32).astype(np.float64), len(rows),
                  1.0 / (p.n + 1), act_bf16=True)
    U0 = N.time_interp(scale * y[0].reshape(len(rows), -1), rows, p.t, alpha=p.alpha)
    Rt = plan.export_dense()
    r = oracle.residual(Rt, U0, b, p.dim, p.n, p.length)
    return U0, float(np.abs(r).max()), Rt, b


@pytest.mark.parametrize("dim,n,M,schedule", [(1, 63, 128, "auto"), (1, 127, 256, "staged"), (2, 15, 64, "auto")])
def test_warm_start_guess_and_solution_match_oracle(dev, dim, n, M, schedule):
    print(f"warm start guess dim={dim} n={n} M={M} {schedule}", flush=True)
    p = _problem(dim, n, M, 41)
    ch = learn.channels()
    params = bf16_params(ch, 42, scale=0.5)
    net = make(ch, 32, params, p.N)
    plan = _plan(p, schedule=schedule)
    learn.attach(plan, net)
    f = torch.as_tensor(p.f, dtype=torch.float64, device=dev)
    u, st = plan.solve(f, tol=1e-10, warm_start=True, warm_res0=True)
    U0, res0, Rt, b = _oracle_guess(p, params, ch, plan)
    assert abs(st["warm_res0"] - res0) <= 1e-3 * res0, (st["warm_res0"], res0)
    U = oracle.timestep_solve(Rt, b, p.dim, p.n, p.length)
    r = oracle.residual(Rt, u.cpu().numpy(), b, p.dim, p.n, p.length)
    assert np.abs(r).max() <= 1.5e-10 * np.abs(b).max()
    assert np.abs(u.cpu().numpy() - U).max() <= 1e-8 * np.abs(U).max()


def test_inference_graph_replays_match_eager_inference(dev):
    """The solver replays its inference from a captured graph: three
    warm-started solves with other work in between (eager inference on
    another input, another plan's solve, a weight update) each give the
    prediction the oracle computes for the weights of that moment."""
    p = _problem(1, 63, 128, 91)
    ch = learn.channels()
    params = bf16_params(ch, 92, scale=0.5)
    net = make(ch, 32, params, 4 * p.N)
    plan = _plan(p)
    learn.attach(plan, net)
    other_p = _problem(1, 31, 64, 93)
    other = _plan(other_p)
    f = torch.as_tensor(p.f, dtype=torch.float64, device=dev)
    for rep in range(3):
        if rep == 2:   # new weights: the replay must read them
            params = bf16_params(ch, 94, scale=0.5)
            net.set_params(params)
        _, st = plan.solve(f, tol=1e-10, warm_start=True, warm_res0=True)
        res0 = _oracle_guess(p, params, ch, plan)[1]
        assert abs(st["warm_res0"] - res0) <= 1e-3 * res0, (rep, st["warm_res0"], res0)
        net.forward(torch.randn((2, 34, 1, 63), dtype=torch.float32, device=dev), 1.0 / 64)   # eager use
        other.solve(torch.as_tensor(other_p.f, dtype=torch.float64, device=dev), tol=1e-10)
        torch.cuda.synchronize()


@pytest.mark.parametrize("schedule", ["auto", "staged"])
def test_warm_start_falls_back_on_nan_weights(dev, schedule):
    p = _problem(1, 63, 128, 51)
    ch = learn.channels()
    net = mg.Net(ch, 32, p.N)
    plan = _plan(p, schedule=schedule)
    f = torch.as_tensor(p.f, dtype=torch.float64, device=dev)
    plan.solve(f, tol=1e-10)
    _, st0 = plan.solve(f, tol=1e-10)   # with the learned cycle count
    learn.attach(plan, net)
    # non-finite weights written after attaching (a blob with them is refused)
    net.set_params(np.full(N.param_count(ch), np.nan, dtype=np.float32))
    u, st = plan.solve(f, tol=1e-10, warm_start=True, warm_res0=True)
    assert st["used_warm_start"] == 0 and not np.isfinite(st["warm_res0"])
    assert st["cycles"] == st0["cycles"]
    assert st["res"] <= 1e-10 * st["bnorm"]


@pytest.mark.parametrize("schedule", ["auto", "staged"])
def test_warm_start_falls_back_on_a_bad_prediction(dev, schedule):
    # a finite prediction so far off (1e30 on every slice) that the first
    # cycles from it cannot bring the residual below ||b||
    p = _problem(1, 63, 128, 61)
    ch = learn.channels()
    params = np.zeros(N.param_count(ch), dtype=np.float32)
    params[-ch[-1]:] = 1e30     # biases of the last layer
    net = make(ch, 32, params, p.N)
    plan = _plan(p, schedule=schedule)
    learn.attach(plan, net)
    f = torch.as_tensor(p.f, dtype=torch.float64, device=dev)
    u, st = plan.solve(f, tol=1e-10, warm_start=True, warm_res0=True)
    assert np.isfinite(st["warm_res0"]) and st["warm_res0"] > st["bnorm"]
    assert st["used_warm_start"] == 0
    assert st["res"] <= 1e-10 * st["bnorm"]
    b = oracle.rhs(p.f, p.t, p.alpha, None)
    r = oracle.residual(plan.export_dense(), u.cpu().numpy(), b, p.dim, p.n, p.length)
    assert np.abs(r).max() <= 1.5e-10 * np.abs(b).max()


@pytest.mark.parametrize("schedule", ["auto", "staged"])
def test_nan_prediction_is_dropped_without_the_residual_flag(dev, schedule):
    """The prediction's defect is evaluated whether or not MGWR_WARM_RES0 is
    given, so a non-finite prediction never reaches the cycles."""
    p = _problem(1, 63, 128, 52)
    ch = learn.channels()
    net = mg.Net(ch, 32, p.N)
    plan = _plan(p, schedule=schedule)
    learn.attach(plan, net)
    net.set_params(np.full(N.param_count(ch), np.nan, dtype=np.float32))
    f = torch.as_tensor(p.f, dtype=torch.float64, device=dev)
    u, st = plan.solve(f, tol=1e-10, warm_start=True)
    assert st["used_warm_start"] == 0 and np.isnan(st["warm_res0"])
    assert st["res"] <= 1e-10 * st["bnorm"] and np.isfinite(u.cpu().numpy()).all()


def test_warm_start_with_zero_network_is_the_zero_iterate(dev):
    p = _problem(1, 63, 128, 71)
    ch = learn.channels()
    net = make(ch, 32, np.zeros(N.param_count(ch), dtype=np.float32), p.N)
    plan = _plan(p)
    f = torch.as_tensor(p.f, dtype=torch.float64, device=dev)
    plan.solve(f, tol=1e-10)
    u0, st0 = plan.solve(f, tol=1e-10)   # with the learned cycle count
    learn.attach(plan, net)
    u1, st1 = plan.solve(f, tol=1e-10, warm_start=True, warm_res0=True)
    assert st1["used_warm_start"] == 1 and st1["warm_res0"] == st1["bnorm"]
    assert st1["cycles"] == st0["cycles"]
    assert torch.allclose(u0, u1, rtol=0, atol=1e-13 * float(u0.abs().max()))


def test_set_warm_start_validates(dev):
    p = _problem(1, 63, 128, 81)
    plan = _plan(p)
    small = make([4, 4, 2], 1, bf16_params([4, 4, 2], 1), p.N)
    with pytest.raises(mg.MgwrError):
        plan.set_warm_start(small, [10, 20])            # channel counts do not match
    ch = learn.channels()
    net = make(ch, 32, bf16_params(ch, 2), 16)
    with pytest.raises(mg.MgwrError):
        learn.attach(plan, net)                         # bound for fewer than N points
    net2 = make(ch, 32, bf16_params(ch, 2), p.N)
    with pytest.raises(mg.MgwrError):
        plan.set_warm_start(net2, list(range(31, -1, -1)))  # rows not increasing
    f = torch.as_tensor(p.f, dtype=torch.float64, device=dev)
    with pytest.raises(mg.MgwrError):
        plan.solve(f, tol=1e-10, warm_start=True)       # nothing attached


def test_learned_gain_small(dev):
    """What a briefly trained network gains over the zero iterate on held-out
    instances (1D, n = 63, M = 128): cycles and float64 residual of the
    prediction, before and after training."""
    dim, n, M = 1, 63, 128
    X, Y, _ = learn.generate(dim, n, M, 96, seed=7, k=8)
    h = 1.0 / (n + 1)
    net = learn.make_net(16 * n, seed=3)
    held = [W.warm_start_family(dim, n, M, np.random.default_rng([9999, i]), k=8) for i in range(6)]

    def run(trained):
        out = []
        for p in held:
            plan = _plan(p)
            learn.attach(plan, net)
            f = torch.as_tensor(p.f, dtype=torch.float64, device=dev)
            # each form twice: the second solve runs with the cycle count the first one learned
            for _ in range(2):
                _, s0 = plan.solve(f, tol=1e-8)
            for _ in range(2):
                _, s1 = plan.solve(f, tol=1e-8, warm_start=True, warm_res0=True)
            assert s0["res"] <= 1e-8 * s0["bnorm"] and s1["res"] <= 1e-8 * s1["bnorm"]
            out.append((s0["cycles"], s1["cycles"], s1["used_warm_start"], s1["warm_res0"] / s1["bnorm"]))
            plan.close()
        return out

    Xh, Yh, _ = learn.generate(dim, n, M, 8, seed=9999, k=8)   # the held-out instances
    loss_before = learn.evaluate_loss(net, Xh, Yh, h)
    before = run(False)
    learn.train(net, X, Y, h, steps=600, batch=16, lr=2e-3)
    loss_after = learn.evaluate_loss(net, Xh, Yh, h)
    after = run(True)
    for tag, rows, loss in (("untrained", before, loss_before), ("trained", after, loss_after)):
        c0 = sum(r[0] for r in rows)
        c1 = sum(r[1] for r in rows)
        print(f"{tag}: held-out loss {loss:.3e}, zero-iterate cycles {c0}, warm-start cycles {c1}, accepted "
              f"{sum(r[2] for r in rows)}/{len(rows)}, median warm res0/||b|| "
              f"{np.median([r[3] for r in rows]):.3e}", flush=True)
    # training on solver output makes the prediction of unseen solutions better
    assert loss_after < 0.5 * loss_before
    # and it saves cycles on them against the zero iterate, every prediction
    # accepted by the float64 residual judge
    assert sum(r[2] for r in after) == len(after)
    assert sum(r[1] for r in after) < sum(r[0] for r in after), after


def test_model_blob_loads_through_the_library(dev):
    """mgwr_model_load: a blob with the network's weights gives the same
    warm-started solve as weights set directly; a corrupt or mismatched blob
    is refused with MGWR_ERR_MODEL and the plan keeps its network."""
    p = _problem(1, 63, 128, 45)
    ch = learn.channels()
    params = bf16_params(ch, 46, scale=0.5)
    rows = learn.slice_rows(p.M)
    f = torch.as_tensor(p.f, dtype=torch.float64, device=dev)
    net_a = make(ch, 32, params, p.N)
    plan_a = _plan(p)
    plan_a.set_warm_start(net_a, rows)
    ua, sa = plan_a.solve(f, tol=1e-10, warm_start=True)
    net_b = mg.Net(ch, 32, p.N)                   # different initial weights
    plan_b = _plan(p)
    blob = mg.model_blob(ch, 32, rows, 0.0, params)
    plan_b.load_model(net_b, blob)
    ub, sb = plan_b.solve(f, tol=1e-10, warm_start=True)
    assert sa["warm_res0"] == sb["warm_res0"] and sa["cycles"] == sb["cycles"]
    assert torch.equal(ua, ub)
    bad = bytearray(blob)
    bad[200] ^= 0xFF
    for broken, other_net in ((bytes(bad), net_b), (b"", net_b), (mg.model_blob([35, 16, 32], 32, rows, 0.0,
                               np.zeros(N.param_count([35, 16, 32]), np.float32)), net_b)):
        with pytest.raises(mg.MgwrError) as ei:
            plan_b.load_model(other_net, broken)
        assert ei.value.code == mg.MGWR_ERR_MODEL
    # still the loaded network: the same prediction bit for bit (the solve from
    # it now runs with the cycle count the first one learned)
    uc, sc = plan_b.solve(f, tol=1e-10, warm_start=True)
    assert sc["warm_res0"] == sb["warm_res0"] and sc["used_warm_start"] == 1
    assert float((uc - ub).abs().max()) <= 1e-9 * float(ub.abs().max())


@pytest.mark.parametrize("schedule", ["pipelined", "staged"])
def test_plausible_but_poor_network_is_rejected(dev, schedule):
    """Moderate constant last-layer biases: a finite, smooth-looking
    prediction several times larger than the solution.  After its first
    cycles the residual is well above what the zero iterate reaches in as
    many cycles, so the judge drops it (used_warm_start 0) and the solve still
    meets the tolerance, the oracle confirming the result."""
    p = _problem(1, 63, 128, 62)
    ch = learn.channels()
    params = np.zeros(N.param_count(ch), dtype=np.float32)
    params[-ch[-1]:] = 4.0
    net = mg.Net(ch, 32, p.N)
    plan = _plan(p, schedule=schedule)
    f = torch.as_tensor(p.f, dtype=torch.float64, device=dev)
    plan.solve(f, tol=1e-10)                          # the zero iterate's rate for the judge
    _, st0 = plan.solve(f, tol=1e-10)
    learn.attach(plan, net)
    net.set_params(params)
    u, st = plan.solve(f, tol=1e-10, warm_start=True)
    first = st["history"][0] / st["bnorm"] if st["history"] else float("nan")
    print(f"{schedule}: warm res0/||b|| {st['warm_res0'] / st['bnorm']:.3e}, first recorded step "
          f"{first:.3e}, zero-start rate {st0['avg_factor']:.3f}, cycles {st['cycles']} vs {st0['cycles']}", flush=True)
    assert np.isfinite(st["warm_res0"]) and st["used_warm_start"] == 0
    assert st["res"] <= 1e-10 * st["bnorm"]
    b = oracle.rhs(p.f, p.t, p.alpha, None)
    r = oracle.residual(plan.export_dense(), u.cpu().numpy(), b, p.dim, p.n, p.length)
    assert np.abs(r).max() <= 1.5e-10 * np.abs(b).max()


def test_warm_started_batch_runs_side_by_side_like_one_by_one(dev):
    """Staged instances sharing one network, solved as a batch with warm
    starts (their predictions take turns on the network while the cycles run
    on worker streams): the same predictions and solutions as solving them
    one by one, each against the oracle."""
    ch = learn.channels()
    params = bf16_params(ch, 47, scale=0.5)
    probs = [_problem(2, 31, 64, 300 + i) for i in range(5)]
    net = make(ch, 32, params, probs[0].N)
    fs = [torch.as_tensor(p.f, dtype=torch.float64, device=dev) for p in probs]
    single = []
    for p, f in zip(probs, fs):
        pl = _plan(p, schedule="staged")
        learn.attach(pl, net)
        single.append(pl.solve(f, tol=1e-11, warm_start=True))
    plans = [_plan(p, schedule="staged") for p in probs]
    for pl in plans:
        learn.attach(pl, net)
    batch = mg.Batch(plans).bind()
    for rep in range(2):
        us, sts = batch.solve(fs, tol=1e-11, warm_start=True)
        for p, pl, u, st, (u1, st1) in zip(probs, plans, us, sts, single):
            assert st["warm_res0"] == st1["warm_res0"] and st["used_warm_start"] == st1["used_warm_start"]
            assert float((u - u1).abs().max()) <= 1e-10 * float(u1.abs().max())
            Rt = pl.export_dense()
            B = oracle.rhs(p.f, p.t, p.alpha, None)
            ref = oracle.timestep_solve(Rt, B, p.dim, p.n, p.length)
            assert np.abs(u.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()
