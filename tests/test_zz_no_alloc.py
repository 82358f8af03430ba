"""The entry point that allocates nothing (mgwr_solve_static, the library's
static device array as the workspace), called through the C ABI and checked
against mgwr_solve on a plan bound to its own workspace: two calls in a row,
the second with a smaller input; the results against the oracle too."""
import ctypes

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


def _static(plan, f, g, tol, u, flags=0):
    st = mg.Stats()
    stream = torch.cuda.current_stream(f.device)
    rc = mg.lib().mgwr_solve_static(plan._h, ctypes.c_void_p(stream.cuda_stream), mg._dptr(f), mg._dptr(g),
                                    float(tol), mg._dptr(u), flags, ctypes.byref(st))
    return rc, st.as_dict()


CASES = [  # dim, n, M, alpha, r, schedule, with an initial value: the second is the smaller input
    (1, 255, 512, 0.5, 3.0, "auto", True),
    (2, 15, 128, 0.4, 4.0, "staged", False),
]


def test_static_workspace_solve_matches_bound_solve(dev):
    for call, (dim, n, M, alpha, r, schedule, with_g) in enumerate(CASES):
        print(f"static call {call}: dim={dim} n={n} M={M} {schedule}", flush=True)
        p = W.manufactured(dim, n, M, alpha, r=r, k=10)
        rng = np.random.default_rng([23, call])
        F = rng.standard_normal((M, p.N))
        # (a rough initial value on a strongly graded mesh makes ||b|| dwarf the
        # solution, a_{1,1} ~ dt_1^-alpha: the smaller case goes without one)
        G = rng.standard_normal(p.N) if with_g else None
        f = torch.as_tensor(F, dtype=torch.float64, device=dev)
        g = None if G is None else torch.as_tensor(G, dtype=torch.float64, device=dev)
        tol = 1e-11
        bound = mg.Plan(dim, n, M, alpha, k=10, t=p.t, schedule=schedule).bind()
        u_ref, st_ref = bound.solve(f, g, tol=tol)
        plain = mg.Plan(dim, n, M, alpha, k=10, t=p.t, schedule=schedule)    # never bound
        u = torch.full_like(f, float("nan"))
        rc, st = _static(plain, f, g, tol, u)
        assert rc == mg.MGWR_OK, mg.lib().mgwr_last_error()
        torch.cuda.synchronize()
        U, Uref = u.cpu().numpy(), u_ref.cpu().numpy()
        assert np.max(np.abs(U - Uref)) <= 1e-10 * np.max(np.abs(Uref)), call
        assert st["res"] <= tol * st["bnorm"] and st["cycles"] == st_ref["cycles"]
        Rt = oracle.hmatrix_dense(p.t, alpha, 10)
        B = oracle.rhs(F, p.t, alpha, G)
        ref = oracle.timestep_solve(Rt, B, dim, n, 1.0)
        assert np.max(np.abs(U - ref)) <= 1e-10 * np.max(np.abs(ref))
        assert np.max(np.abs(oracle.residual(Rt, U, B, dim, n, 1.0))) <= 1.2 * tol * np.max(np.abs(B))
        # a plan bound to its own workspace keeps working after a static call on it
        rc, _ = _static(bound, f, g, tol, torch.empty_like(f))
        assert rc == mg.MGWR_OK
        u2, st2 = bound.solve(f, g, tol=tol)
        assert float((u2 - u_ref).abs().max()) <= 1e-10 * float(u_ref.abs().max())


def test_static_workspace_limits(dev):
    big = mg.Plan(2, 127, 256, 0.5, k=10, r=3.0)          # about 99 MiB of workspace
    assert big.workspace_bytes() > (64 << 20)
    f = torch.zeros((256, 127 * 127), dtype=torch.float64, device=dev)
    rc, _ = _static(big, f, None, 1e-8, torch.empty_like(f))
    assert rc == mg.MGWR_ERR_INVALID_ARG and "static workspace" in mg.lib().mgwr_last_error().decode()
    small = mg.Plan(1, 63, 128, 0.5, k=8, r=3.0)
    f = torch.ones((128, 63), dtype=torch.float64, device=dev)
    rc, _ = _static(small, f, None, 1e-8, torch.empty_like(f), flags=mg.MGWR_WARM_START)
    assert rc == mg.MGWR_ERR_INVALID_ARG
