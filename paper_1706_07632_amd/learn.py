"""Training and use of the learned initial guess.

The network (Net, a band-pyramid stack of 3x3 convolutions run by the
library's own kernels) maps the right-hand side at `nslices` time rows, plus
the constant channels alpha and r/10, to the solution at those rows.  Its
training data are solutions that the solver itself computes (plain float64
MGWR to a tight tolerance) on seeded instances of
`workloads.warm_start_family`; training runs the library's forward, backward
and Adam kernels.  In a solve the prediction is interpolated in time and
judged by the method's own float64 residual (MGWR_WARM_START).

Command line (on a GPU):
    python -m paper_1706_07632_amd.learn --dim 1 --n 255 --M 1024 --count 512 \
        --steps 3000 --out weights.npz
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import Net, Plan, model_blob

NSLICES = 32
HIDDEN = 64
LAYERS = 4


def slice_rows(M: int, nslices: int = NSLICES) -> list[int]:
    """Time rows of the network's slices: rows s*M/nslices - 1, s = 1..nslices
    (the last one is the final time level)."""
    if M < nslices:
        raise ValueError("M must be at least the number of slices")
    return [s * M // nslices - 1 for s in range(1, nslices + 1)]


def channels(nslices: int = NSLICES, hidden: int = HIDDEN, layers: int = LAYERS) -> list[int]:
    """[slices + alpha + r/10 + level value, hidden..., slices]."""
    return [nslices + 3] + [hidden] * (layers - 1) + [nslices]


def make_net(max_bhw: int, nslices: int = NSLICES, hidden: int = HIDDEN, layers: int = LAYERS, seed: int = 0):
    return Net(channels(nslices, hidden, layers), nslices, max_bhw, seed=seed)


def grid_shape(dim: int, n: int):
    return (1, n) if dim == 1 else (n, n)


def _device_source(p, torch, dev):
    """f [M][N] on the device from the instance's sine modes."""
    import workloads as W
    f = torch.zeros((p.M, p.N), dtype=torch.float64, device=dev)
    for kvec, prof in p.modes:
        f.add_(torch.outer(torch.as_tensor(prof, dtype=torch.float64, device=dev),
                           torch.as_tensor(W.sine_mode(p.n, p.dim, p.length, kvec), dtype=torch.float64, device=dev)))
    return f


def generate(dim: int, n: int, M: int, count: int, seed: int, tol: float = 1e-10, k: int = 10,
             nslices: int = NSLICES, log=None, group: int = 1, seconds: float = 0.0):
    """Solver-generated samples: X [count][nslices+2][H][W] (f at the slice
    rows over ||f||_inf, alpha, r/10) and Y [count][nslices][H][W] (the
    float64 MGWR solution at those rows over ||f||_inf), float32 on the GPU.
    Instances [seed, i] of workloads.warm_start_family; sources are built on
    the device from their sine modes; with group > 1 that many instances are
    solved as one batch (their staged solves side by side), and the host
    set-up of the next group's plans runs on worker threads meanwhile.  With
    seconds > 0 generation stops after the first group that ends past that
    wall time; the arrays are then cut to the samples made."""
    import concurrent.futures as cf

    import torch
    import workloads as W
    from . import Batch
    H, Wd = grid_shape(dim, n)
    rows = slice_rows(M, nslices)
    dev = torch.device("cuda", torch.cuda.current_device())
    X = torch.empty((count, nslices + 2, H, Wd), dtype=torch.float32, device=dev)
    Y = torch.empty((count, nslices, H, Wd), dtype=torch.float32, device=dev)
    ridx = torch.tensor(rows, device=dev)
    cycles = []
    t0 = time.time()

    def make(i):
        p = W.warm_start_family(dim, n, M, np.random.default_rng([seed, i]), k=k, build_f=False)
        return p, Plan(dim, n, M, p.alpha, k=p.k, r=p.r, t=p.t)

    starts = list(range(0, count, group))
    last_log = t0
    with cf.ThreadPoolExecutor(max_workers=8) as pool:
        pending = [pool.submit(make, i) for i in range(starts[0], min(count, starts[0] + group))]
        for gi, s0 in enumerate(starts):
            items = [fut.result() for fut in pending]
            nxt = starts[gi + 1] if gi + 1 < len(starts) else None
            pending = [pool.submit(make, i) for i in range(nxt, min(count, nxt + group))] if nxt is not None else []
            probs = [it[0] for it in items]
            plans = [it[1].bind() for it in items]
            fs = [_device_source(p, torch, dev) for p in probs]
            if len(plans) > 1:
                us, sts = Batch(plans).bind().solve(fs, tol=tol)
            else:
                u, st = plans[0].solve(fs[0], tol=tol)
                us, sts = [u], [st]
            for j, (p, f, u, st) in enumerate(zip(probs, fs, us, sts)):
                i = s0 + j
                scale = f.abs().max()
                X[i, :nslices] = (f.index_select(0, ridx) / scale).reshape(nslices, H, Wd).float()
                X[i, nslices] = p.alpha
                X[i, nslices + 1] = p.r / 10.0
                Y[i] = (u.index_select(0, ridx) / scale).reshape(nslices, H, Wd).float()
                cycles.append(st["cycles"])
            for pl in plans:
                pl.close()
            now = time.time()
            done = min(count, s0 + group)
            if log and (now - last_log > 30 or done >= count):
                last_log = now
                log(f"generated {done}/{count} samples ({now - t0:.1f} s)")
            if seconds > 0 and now - t0 > seconds and done < count:
                for fut in pending:
                    fut.result()[1].close()
                if log:
                    log(f"generation stopped at its time budget: {done} samples ({now - t0:.1f} s)")
                return X[:done].clone(), Y[:done].clone(), cycles
    return X, Y, cycles


def train(net, X, Y, h: float, steps: int, batch: int = 16, lr: float = 1e-3, lr_end: float = 1e-5,
          seed: int = 0, log=None, log_every: int = 250, seconds: float = 0.0):
    """Adam with a cosine learning-rate decay on random minibatches.  With
    seconds > 0 the step count is cut, after timing the first 50 steps, to
    what fits that wall time (the schedule then spans the steps that run)."""
    import torch
    g = torch.Generator(device=X.device)
    g.manual_seed(seed)
    losses = []
    t0 = time.time()
    it = 0
    while it < steps:
        if seconds > 0 and it == 50:
            torch.cuda.synchronize()
            per = (time.time() - t0) / 50
            steps = max(51, min(steps, int(seconds / per)))
            if log:
                log(f"{per * 1e3:.1f} ms per step: {steps} steps fit the time budget")
        idx = torch.randint(0, X.shape[0], (batch,), device=X.device, generator=g)
        xb = X.index_select(0, idx).contiguous()
        yb = Y.index_select(0, idx).contiguous()
        cur = lr_end + 0.5 * (lr - lr_end) * (1 + math.cos(math.pi * it / max(1, steps)))
        want = (it % log_every == 0) or it == steps - 1
        loss = net.train_step(xb, yb, h, lr=cur, want_loss=want)
        if want:
            losses.append((it, loss))
            if log:
                log(f"step {it} loss {loss:.4e} lr {cur:.2e} ({time.time() - t0:.1f} s)")
        it += 1
    return losses, steps


def evaluate_loss(net, X, Y, h: float, batch: int = 16) -> float:
    tot, cnt = 0.0, 0
    for s in range(0, X.shape[0], batch):
        xb, yb = X[s:s + batch].contiguous(), Y[s:s + batch].contiguous()
        loss, _ = net.gradient(xb, yb, h)
        tot += loss * xb.shape[0]
        cnt += xb.shape[0]
    return tot / max(1, cnt)


def gain(net, problems, tol: float = 1e-8, precision: str = "fp64", repeats: int = 2, log=None,
         inner_cycles: int = 1):
    """Cycles and solve times with the zero iterate and with the warm start on
    `problems` (workloads.Problem); each form is solved `repeats` times on the
    same plan and the last solve counts (it runs with the cycle count the
    earlier ones learned)."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    rows = []
    for p in problems:
        plan = Plan(p.dim, p.n, p.M, p.alpha, k=p.k, r=p.r, t=p.t, precision=precision,
                    inner_cycles=inner_cycles if precision != "fp64" else 1).bind()
        attach(plan, net)
        f = torch.as_tensor(p.f, dtype=torch.float64, device=dev)
        out = {}
        for form, ws in (("zero", False), ("warm", True)):
            for _ in range(repeats):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st = plan.solve(f, tol=tol, warm_start=ws, warm_res0=ws)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            out[form] = {"cycles": st["cycles"], "seconds": dt, "rel_res": st["res"] / st["bnorm"],
                         "used_warm_start": st["used_warm_start"], "warm_res0": st["warm_res0"] / st["bnorm"]}
        rows.append(out)
        plan.close()
        if log:
            log(f"alpha={p.alpha:.3f}: zero {out['zero']['cycles']} cycles {out['zero']['seconds'] * 1e3:.1f} ms, "
                f"warm {out['warm']['cycles']} cycles {out['warm']['seconds'] * 1e3:.1f} ms "
                f"(accepted {out['warm']['used_warm_start']}, res0/||b|| {out['warm']['warm_res0']:.2e})")
    return rows


def save(net, path: str, meta: dict):
    params = net.params.detach().float().cpu().numpy()
    np.savez(path, params=params, channels=np.array(net.channels, dtype=np.int32),
             nsignal=np.array(net.nsignal, dtype=np.int32), meta=np.array(json.dumps(meta)))


def load(path: str, max_bhw: int):
    """(Net with the stored weights, metadata dict); bands finer than the
    training grid are left out."""
    with np.load(path, allow_pickle=False) as z:
        params = z["params"]
        ch = [int(c) for c in z["channels"]]
        nsig = int(z["nsignal"])
        meta = json.loads(str(z["meta"]))
    net = Net(ch, nsig, max_bhw)
    net.set_params(params)
    net.set_finest(meta.get("h_min", 0.0))
    return net, meta


def blob_for(net, M: int, nslices: int = NSLICES) -> bytes:
    """The weight blob of `net` (its current master weights and finest-band
    cut-off) with the slice rows of an M-step mesh."""
    params = net.params.detach().float().cpu().numpy()
    return model_blob(net.channels, net.nsignal, slice_rows(M, nslices), getattr(net, "h_min", 0.0), params)


def attach(plan, net, nslices: int = NSLICES):
    """Attach `net` to `plan` for warm-started solves at the plan's slice rows,
    through the library's weight-blob loader (mgwr_model_load)."""
    plan.load_model(net, blob_for(net, plan.M, nslices))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--dim", type=int, default=1)
    ap.add_argument("--n", type=int, default=255)
    ap.add_argument("--M", type=int, default=1024)
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--val", type=int, default=32)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", required=True)
    ap.add_argument("--gen-tol", type=float, default=1e-10,
                    help="relative residual of the solver runs that produce the targets (the float64 floor is "
                         "about 2e-10 at h = 1/1024)")
    ap.add_argument("--eval-n", type=int, default=0, help="held-out evaluation grid (0: skip)")
    ap.add_argument("--eval-M", type=int, default=0)
    ap.add_argument("--eval-count", type=int, default=4)
    ap.add_argument("--group", type=int, default=16, help="training instances solved together as one batch")
    ap.add_argument("--gen-seconds", type=float, default=0.0, help="wall-time budget of the sample generation")
    ap.add_argument("--train-seconds", type=float, default=0.0, help="wall-time budget of the training")
    a = ap.parse_args(argv)
    import torch

    def log(msg):
        print(msg, flush=True)

    H, Wd = grid_shape(a.dim, a.n)
    h = 1.0 / (a.n + 1)
    log(f"generating {a.count} + {a.val} samples: dim={a.dim} n={a.n} M={a.M}")
    X, Y, cyc = generate(a.dim, a.n, a.M, a.count, a.seed, tol=a.gen_tol, log=log, group=a.group,
                         seconds=a.gen_seconds)
    a.count = X.shape[0]
    Xv, Yv, _ = generate(a.dim, a.n, a.M, a.val, a.seed + 1000, tol=a.gen_tol, group=a.group)
    log(f"solver cycles per sample: mean {np.mean(cyc):.2f}")
    net = make_net(max(a.batch, 16) * H * Wd, seed=a.seed)
    losses, a.steps = train(net, X, Y, h, a.steps, a.batch, a.lr, log=log, seconds=a.train_seconds)
    vloss = evaluate_loss(net, Xv, Yv, h)
    log(f"validation loss {vloss:.4e}")
    meta = {"dim": a.dim, "n": a.n, "M": a.M, "count": a.count, "seed": a.seed, "steps": a.steps,
            "batch": a.batch, "lr": a.lr, "final_train_loss": losses[-1][1], "val_loss": vloss,
            "family": "workloads.warm_start_family", "nslices": NSLICES, "h_min": h}
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    save(net, a.out, meta)
    log(json.dumps(meta))
    if a.eval_n:
        import workloads as W
        probs = [W.warm_start_family(a.dim, a.eval_n, a.eval_M, np.random.default_rng([100001, i]))
                 for i in range(a.eval_count)]
        big = make_net(a.eval_n ** a.dim, seed=0)
        big.set_params(net.params.detach().cpu().numpy())
        big.set_finest(h)
        for precision in ("fp64", "mixed"):
            log(f"held-out gain at n={a.eval_n} M={a.eval_M} ({precision})")
            rows = gain(big, probs, precision=precision, log=log, inner_cycles=2 if a.dim == 2 else 1)
            z = sum(r["zero"]["seconds"] for r in rows)
            w = sum(r["warm"]["seconds"] for r in rows)
            log(f"total: zero {sum(r['zero']['cycles'] for r in rows)} cycles {z:.3f} s, warm "
                f"{sum(r['warm']['cycles'] for r in rows)} cycles {w:.3f} s, speed-up {z / w:.3f}")
    torch.cuda.synchronize()
    return 0


if __name__ == "__main__":
    sys.exit(main())
