#!/usr/bin/env python3
"""Throughput of the H-matrix MGWR solver on one MI355X.

Metric: space-time unknowns (N*M) per second to 1e-8 relative residual
(||b - A u||_inf <= 1e-8 ||b||_inf, float64 residual), plain float64 against
mixed precision and the learned warm start.

Headline (`value`): the batched workload, 64 uneven 2D instances of the
seeded random-Fourier family (sides {63, 127, 255}, M in {256, 512, 1024,
2048}, alpha ~ U[0.2, 0.9], r = (2 - alpha)/alpha, k = 10, leaf 16, V(1,1),
zero initial guess), 1.63e9 unknowns per step, solved as one batch in
float64.  One step = one batch solve; sources resident in HBM before timing.

`forms` holds, each with its own roofline and CPU baseline:
* the batched workload with float32 inner cycles (float64 residual), with
  bfloat16 low-rank factors, and with one merged pipelined launch for all
  instances;
* 2D n = 255, M = 1024 (manufactured solution): float64, mixed, and both
  warm-started by the committed network;
* the learned warm start at its evaluation point (2D n = 255, M = 1024,
  held-out instances of its training family): zero iterate against the
  network's prediction, float64 and mixed;
* 1D n = 1023, M = 4096, alpha in {0.3, 0.5, 0.7} as one merged launch.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time


ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 (vector and matrix)
PEAK_FP32_TFLOPS = 157.3    # MI355X dense FP32 (matrix; the mixed inner cycles multiply in float32)
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of a workload's dominant kernel from rocprofv3
# FETCH_SIZE / WRITE_SIZE runs (KiB per dispatch) scaled by what the same
# counters read for a 1 GiB device copy (--copy-probe: fetch x 2.000, write
# x 1.000).  Keyed by the SHA-256 of kernels.hip and of mgwr.cpp (the
# launch schedule) they were taken on; a different source reports null.
# batched: the side-by-side phase of one
# batch solve (every kernel of the staged instances, the second solve of the
# run); large2d: the average float64 SMOOTH march; large1d: the timed
# pipelined launch (profiles/ holds the runs).
_SHA = "49d8b39a4ff58e7e56d84f97005c125dfcbb75cfbe8220df102681c8f69bd63d"
_SCHED = "c1b8cbeacc2aebeaacf8280053e8f6c3a6e5aa6678d851682e6c47291949a5c5"
TRAFFIC = {
    "batched_fp64": (_SHA, _SCHED, 1.2598e12 + 5.9479e11),
    "large2d_fp64": (_SHA, _SCHED, 3.5508e8 + 1.6939e8),
    "large1d_fp64": (_SHA, _SCHED, 4.0701e10 + 1.0359e10),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="all",
                    choices=["all", "batched", "large2d", "learned2d", "large1d", "small1d", "paper1d"],
                    help="all: the batched headline and every form; otherwise only that workload's forms")
    ap.add_argument("--batch-count", type=int, default=64, help="instances of the batched workload")
    ap.add_argument("--batch-schedule", default="auto", choices=["auto", "pipelined", "autotune"],
                    help="batched workload: the plans' AUTO rule, every instance pipelined (one merged launch), "
                         "or the autotuner per (n, M) bucket")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--inner-cycles", type=int, default=0,
                    help="float32 V-cycles per float64 refinement step of the mixed forms; 0: each workload's "
                         "measured best (batched 3, 2D n=255 2, 1D 1)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--xcd-queues", action="store_true",
                    help="deal the pipelined launches' work items to per-XCD queues (off by default)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--value-only", action="store_true",
                    help="time only the float64 form of the selected workload (the headline with --workload all; "
                         "no other forms, no CPU baseline): the command the kernel profiles are taken on")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB three times on the device (counter calibration) and exit")
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="hardware queues of the process (GPU_MAX_HW_QUEUES, set before HIP starts; 1-32)")
    return ap.parse_args()


def set_hw_queues(n):
    """Hardware queues per process; HIP reads GPU_MAX_HW_QUEUES when it
    initialises, so this runs before the first device call.  The batched
    workload's staged instances run on 8 worker streams; with HIP's default
    of 4 queues two streams share each queue and their launches wait for one
    another.  Measured per batch solve: 938 ms with 4 queues, 925 with 8, 919
    with 16; 32 queues or 12-16 workers no faster."""
    if not 1 <= n <= 32:
        raise SystemExit("--hw-queues must be between 1 and 32")
    os.environ["GPU_MAX_HW_QUEUES"] = str(n)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def copy_probe():
    import torch
    x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": x.numel() * 8, "copies": 3}), flush=True)


def source_sha(name):
    with open(os.path.join(ROOT, "paper_1706_07632_amd", "csrc", name), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def kernel_sha():
    return source_sha("kernels.hip")


def schedule_sha():
    return source_sha("mgwr.cpp")


def traffic_for(key):
    entry = TRAFFIC.get(key)
    if entry is None or entry[0] != kernel_sha() or entry[1] != schedule_sha():
        return None
    return entry[2]


# ---- timing helpers -----------------------------------------------------------

def time_plans(plans, fs, us, tol, steps, warmup, torch, warm_start=False):
    """Wall time of `steps` passes over the instances (one plan each), after
    `warmup` untimed passes; per-launch event timing covers the timed passes."""
    stats = []
    for _ in range(warmup):
        for pl, f, u in zip(plans, fs, us):
            pl.solve(f, tol=tol, u=u, warm_start=warm_start)
    for pl in plans:
        pl.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for pl, f, u in zip(plans, fs, us):
            stats.append(pl.solve(f, tol=tol, u=u, warm_start=warm_start)[1])
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    timing = merge_timing([pl.timing() for pl in plans])
    for pl in plans:
        pl.timing(False)
    return secs, stats[-len(plans):], timing


def time_batch(batch, plans, fs, us, tol, steps, warmup, torch, warm_start=False):
    """Wall time of `steps` batch solves after `warmup` untimed ones; the
    batch's timing (event-timed merged launches, the side-by-side phase of
    staged instances) and the plans' own launches cover the timed solves."""
    for _ in range(warmup):
        batch.solve(fs, tol=tol, us=us, warm_start=warm_start)
    batch.timing(True)
    for pl in plans:
        pl.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = None
    for _ in range(steps):
        _, st = batch.solve(fs, tol=tol, us=us, warm_start=warm_start)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    timing = merge_timing([batch.timing(False)] + [pl.timing() for pl in plans])
    for pl in plans:
        pl.timing(False)
    return secs, st, timing


def merge_timing(timings):
    out = {}
    for tm in timings:
        for cls, v in tm.items():
            o = out.setdefault(cls, {"launches": 0, "ms": 0.0, "flops": 0.0, "bytes": 0.0})
            for key in o:
                o[key] += v[key]
    return out


KERNEL_NAMES = {
    "pipe64": "pipeline_kernel (K time-pipelined V-cycles: zebra line relaxation with H-forward substitution, "
              "defects, grid transfers; float64, or float32 inner cycles)",
    "smooth64": "march_kernel<double, SMOOTH> (zebra half-sweep: H-forward substitution of every line)",
    "smooth32": "march_kernel<float, SMOOTH> (float32 zebra half-sweep)",
    "defect64": "march_kernel<double, RESID> (defect: H-matrix product and stencil)",
    "coarse": "pipeline_kernel (coarse levels of a staged cycle)",
    "side": "staged instances solved side by side (march_kernel and pipeline_kernel launches on 8 streams)",
}


def roofline(timing, precision, traffic_key=None):
    """Dominant kernel class (by summed duration) and its algorithmic rate:
    algorithmic flops per launch / average event-measured launch duration,
    against the peak of the arithmetic it runs (FP64 MFMA, or FP32 MFMA for
    the float32 inner cycles).  The side-by-side class is one host-timed
    entry per batch solve (its launches overlap on several streams)."""
    cands = {k: v for k, v in timing.items() if v["launches"] and v["flops"] > 0}
    if not cands:
        return None
    dom = max(cands, key=lambda k: cands[k]["ms"])
    v = cands[dom]
    peak = PEAK_FP64_TFLOPS if (precision == "fp64" or dom.endswith("64")) else PEAK_FP32_TFLOPS
    achieved = v["flops"] / (v["ms"] * 1e-3) / 1e12
    out = {"bound": "mfma", "kernel": KERNEL_NAMES.get(dom, dom), "class": dom, "achieved": achieved,
           "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
           "traffic": traffic_for(traffic_key) if traffic_key else None,
           "algorithmic_flops_per_launch": v["flops"] / v["launches"],
           "algorithmic_bytes_per_launch": v["bytes"] / v["launches"],
           "avg_launch_us": 1e3 * v["ms"] / v["launches"], "launches": v["launches"]}
    if dom == "side":
        out["basis"] = "host wall time of the side-by-side phase (overlapping launches on 8 streams)"
    return out


def kernels_table(timing):
    return {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                "avg_us": round(1e3 * v["ms"] / max(1, v["launches"]), 2),
                "TFLOP/s": round(v["flops"] / max(v["ms"], 1e-9) * 1e-9, 3),
                "GB/s": round(v["bytes"] / max(v["ms"], 1e-9) * 1e-6, 1)}
            for k, v in timing.items() if v["launches"]}


# ---- CPU baseline: the oracle on the host cores --------------------------------

def cpu_baseline(probs, rows, label, one_thread_rows=None):
    """The float64 oracle (direct time marching: history sum by BLAS, banded
    solve in 1D, type-I sine transforms in 2D) on the host cores, on a bounded
    sample: the first `rows[i]` time levels of each instance in `probs`
    (R~ assembly excluded).  unknowns/s = sum N rows / time.  The same sample's
    first instance is also timed with one BLAS thread."""
    import numpy as np

    import oracle
    from threadpoolctl import threadpool_info, threadpool_limits
    nproc = os.cpu_count() or 1
    try:
        threads = max(int(x.get("num_threads", 1)) for x in threadpool_info()) if threadpool_info() else 1
    except Exception:
        threads = 1
    prep = []
    for p, m in zip(probs, rows):
        Rt = oracle.hmatrix_dense(p.t, p.alpha, p.k, p.leaf)
        if p.f is not None:
            B = oracle.rhs(p.f[:m], p.t, p.alpha, p.g)
        else:
            B = np.zeros((m, p.N))
            for kvec, prof in p.modes:
                import workloads as W
                B += np.outer(prof[:m], W.sine_mode(p.n, p.dim, p.length, kvec))
        prep.append((p, m, Rt, B))
    secs, unknowns = 0.0, 0
    for p, m, Rt, B in prep:
        t0 = time.perf_counter()
        oracle.timestep_solve(Rt, B, p.dim, p.n, p.length, m_stop=m)
        secs += time.perf_counter() - t0
        unknowns += p.N * m
    out = {"value": unknowns / secs, "unit": "unknowns/s", "cores": threads, "nproc": nproc, "kind": "oracle",
           "sample": f"{label}: the first {', '.join(str(m) for m in rows)} time levels of "
                     f"{len(probs)} instance(s) ({unknowns:.3e} unknowns, {secs:.2f} s), R~ assembly excluded"}
    p, m, Rt, B = prep[0]
    m1 = one_thread_rows or m
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        oracle.timestep_solve(Rt, B[:m1], p.dim, p.n, p.length, m_stop=m1)
        s1 = time.perf_counter() - t0
    out["one_thread"] = {"value": p.N * m1 / s1, "sample": f"first {m1} levels of the first instance ({s1:.2f} s)"}
    return out


# ---- workloads ---------------------------------------------------------------

def batched_sources(probs, torch, dev):
    import workloads as W
    fs = []
    for p in probs:
        f = torch.zeros((p.M, p.N), dtype=torch.float64, device=dev)
        for kvec, prof in p.modes:
            f.add_(torch.outer(torch.as_tensor(prof, dtype=torch.float64, device=dev),
                               torch.as_tensor(W.sine_mode(p.n, 2, 1.0, kvec), dtype=torch.float64, device=dev)))
        fs.append(f)
    return fs


# Float32 cycles per float64 refinement step of the mixed forms, measured per
# workload (unknowns/s to 1e-8 for 1..6): more cycles per step amortise the
# float64 defect and the host-side stopping test, until a step's float32
# cycles reduce the residual less than the count suggests and cycles are
# wasted (2D n=255, M=1024: 10, 10, 12, 12, 15, 18 cycles for 1..6).
BEST_INNER = {"batched": 3, "large2d": 2, "learned2d": 2, "large1d": 1, "small1d": 1}


def inner_for(args, workload):
    return args.inner_cycles if args.inner_cycles > 0 else BEST_INNER[workload]


def batched_forms(args, torch, mg, dev):
    """The batched workload in float64 (the headline), float32 inner cycles,
    bfloat16 factors, and (with the AUTO rule) every instance pipelined."""
    import workloads as W
    probs = W.batched_instances(count=args.batch_count, build_f="modes")
    fs = batched_sources(probs, torch, dev)
    us = [torch.empty_like(f) for f in fs]
    unknowns = sum(p.N * p.M for p in probs)
    variants = [("fp64", "fp64", args.batch_schedule)]
    if not args.no_mixed:
        variants += [("mixed_fp32", "mixed", args.batch_schedule), ("mixed_bf16", "mixed_bf16", args.batch_schedule)]
    if not args.value_only and args.batch_schedule == "auto":
        variants += [("fp64_one_launch", "fp64", "pipelined"), ("mixed_fp32_one_launch", "mixed", "pipelined")]
        if args.no_mixed:
            variants.pop()
    out = {}
    for name, precision, sched in variants:
        t0 = time.perf_counter()
        plans = [mg.Plan(2, p.n, p.M, p.alpha, k=p.k, r=p.r, t=p.t, precision=precision,
                         inner_cycles=inner_for(args, "batched") if precision != "fp64" else 1,
                         schedule="pipelined" if sched == "pipelined" else "auto").bind() for p in probs]
        setup_s = time.perf_counter() - t0
        tuned = {}
        if sched == "autotune":
            for p, pl, f, u in zip(probs, plans, fs, us):
                key = (p.n, p.M)
                if key not in tuned:
                    tuned[key] = pl.autotune(f, tol=args.tol, u=u)
        batch = mg.Batch(plans, graph=True).bind()
        secs, st, timing = time_batch(batch, plans, fs, us, args.tol, args.steps, args.warmup, torch)
        out[name] = {"value": unknowns * args.steps / secs, "ms_per_step": 1e3 * secs / args.steps,
                     "inner_cycles": inner_for(args, "batched") if precision != "fp64" else None,
                     "cycles_total": sum(s["cycles"] for s in st),
                     "max_rel_res": max(s["res"] / s["bnorm"] for s in st),
                     "setup_s": round(setup_s, 2), "graph_replays": batch.graph_replays(),
                     "pipelined_instances": sum(pl.tuned()["schedule"] == "pipelined" for pl in plans),
                     "roofline": roofline(timing, precision, f"batched_{name}"),
                     "kernels": kernels_table(timing)}
        log(f"batched {name}: {out[name]['value']:.3e} unknowns/s, {out[name]['ms_per_step']:.1f} ms/step")
        batch.close()
        for pl in plans:
            pl.close()
    cpu = None
    if not args.no_cpu_baseline:
        # one instance of each side: the first seeded instances with n = 63, 127, 255
        pick = []
        for side in (63, 127, 255):
            pick.append(next(p for p in probs if p.n == side))
        rows = [min(p.M, 2048 if p.n < 255 else 1024) for p in pick]
        cpu = cpu_baseline(pick, rows, "batched workload, one instance per side", one_thread_rows=512)
        for v in out.values():
            v["cpu_baseline"] = cpu
    cfg = {"workload": f"batched: {len(probs)} uneven 2D instances, sides {{63,127,255}}, M {{256,512,1024,2048}}, "
                       "alpha~U[0.2,0.9], r=(2-a)/a, k=10, leaf 16, V(1,1), random-Fourier sources",
           "instances": len(probs), "unknowns": unknowns, "tol": args.tol,
           "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
           "schedules": ("auto: pipelined when the finest half-sweep has at most 256 chains of 16 columns, "
                         "else staged (side by side on 8 streams) with the coarse levels pipelined")
           if args.batch_schedule == "auto" else args.batch_schedule}
    return out, cfg, cpu


def single_forms(name, probs, args, torch, mg, dev, learned=None, variants=None):
    """Float64, mixed and (optionally) warm-started solves of `probs`; several
    instances run as one batch (one merged launch when pipelined)."""
    fs = [torch.as_tensor(p.f, dtype=torch.float64, device=dev) for p in probs]
    us = [torch.empty_like(f) for f in fs]
    unknowns = sum(p.N * p.M for p in probs)
    out = {}
    variants = variants or [("fp64", "fp64", False), ("mixed", "mixed", False)]
    for form, precision, warm in variants:
        if precision != "fp64" and args.no_mixed:
            continue
        if warm and (args.no_learned or learned is None):
            continue
        plans = [mg.Plan(p.dim, p.n, p.M, p.alpha, k=p.k, r=p.r, t=p.t, length=p.length, leaf=p.leaf,
                         precision=precision, inner_cycles=inner_for(args, name) if precision != "fp64" else 1).bind()
                 for p in probs]
        if warm:
            from paper_1706_07632_amd import learn
            for pl, f, u in zip(plans, fs, us):
                pl.solve(f, tol=args.tol, u=u)       # the zero iterate's rate for the warm-start judge
                learn.attach(pl, learned)
        if len(plans) > 1:
            batch = mg.Batch(plans).bind()
            secs, st, timing = time_batch(batch, plans, fs, us, args.tol, args.steps, args.warmup, torch,
                                          warm_start=warm)
        else:
            secs, st, timing = time_plans(plans, fs, us, args.tol, args.steps, args.warmup, torch, warm_start=warm)
        out[form] = {"value": unknowns * args.steps / secs, "ms_per_step": 1e3 * secs / args.steps,
                     "cycles": [s["cycles"] for s in st], "rel_res": [s["res"] / s["bnorm"] for s in st],
                     "roofline": roofline(timing, precision, f"{name}_{form}"), "kernels": kernels_table(timing)}
        if precision != "fp64":
            out[form]["refinements"] = [s["refinements"] for s in st]
            out[form]["inner_cycles"] = inner_for(args, name)
        if warm:
            out[form]["used_warm_start"] = [s["used_warm_start"] for s in st]
            out[form]["warm_res0_rel"] = [s["warm_res0"] / s["bnorm"] for s in st]
        log(f"{name} {form}: {out[form]['value']:.3e} unknowns/s, cycles {out[form]['cycles']}")
        for pl in plans:
            pl.close()
    return out


# The paper's first experiment at its largest grid (x in (0, pi), f = 0,
# g = sin x, N x M = 2048 x 2048, i.e. 2047 interior points and 2048 graded
# steps, r = (2 - alpha)/alpha, k = 20, V(0,1), residual reduced by 1e-10):
# cycles and seconds of the draft rows of its iteration table (commented out
# in the paper's source; MATLAB on a 2.7 GHz Core i5 laptop).  Context only.
PAPER_1D_DRAFT = {0.2: (11, 685.09), 0.4: (9, 598.86), 0.6: (7, 502.67), 0.8: (7, 553.54)}
PAPER_HARDWARE = "MATLAB, MacBook Pro, Intel Core i5 2.7 GHz, 8 GB (draft timings, float64 inferred)"


def paper_forms(args, torch, mg, dev):
    """The paper's 1D experiment at 2048 x 2048, one solve at a time, next to
    its draft timings."""
    import workloads as W
    per, secs_all, unknowns_all = {}, 0.0, 0
    for a, (pc, ps) in PAPER_1D_DRAFT.items():
        p = W.paper_1d_mittag_leffler(2047, 2048, a, k=20)
        plan = mg.Plan(1, p.n, p.M, a, k=20, t=p.t, length=p.length, nu1=0, nu2=1, max_cycles=60).bind()
        f = torch.zeros((p.M, p.n), dtype=torch.float64, device=dev)
        g = torch.as_tensor(p.g, dtype=torch.float64, device=dev)
        u = torch.empty_like(f)
        for _ in range(max(args.warmup, 1)):
            plan.solve(f, g, tol=1e-10, u=u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, st = plan.solve(f, g, tol=1e-10, u=u)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        nm = p.n * p.M
        per[str(a)] = {"seconds": dt, "cycles": st["cycles"], "unknowns_per_s": nm / dt,
                       "paper_draft": {"seconds": ps, "cycles": pc, "unknowns_per_s": nm / ps}}
        secs_all += dt
        unknowns_all += nm
        plan.close()
        log(f"paper1d alpha={a}: {dt * 1e3:.2f} ms, cycles {st['cycles']} (paper draft {ps} s, {pc} cycles)")
    return {"value": unknowns_all / secs_all, "ms_per_step": 1e3 * secs_all, "per_alpha": per,
            "context": "the paper's own problem, grid and stopping rule (1e-10); its draft times are quoted as "
                       "context, not as a baseline (another machine, MATLAB)",
            "paper_hardware": PAPER_HARDWARE}


def load_net(dim, max_bhw):
    from paper_1706_07632_amd import learn
    path = os.path.join(ROOT, "paper_1706_07632_amd", "weights", f"warm{dim}d.npz")
    if not os.path.exists(path):
        return None, None
    return learn.load(path, max_bhw)


def main():
    args = parse()
    if args.value_only:
        args.no_mixed = args.no_learned = args.no_cpu_baseline = True
    if args.copy_probe:
        copy_probe()
        return
    set_hw_queues(args.hw_queues)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU: --gpus must be 1 (sharding across GPUs is "
                                   "described in the design notes, not implemented)"}))
        sys.exit(2)
    import torch

    import paper_1706_07632_amd as mg
    import workloads as W
    dev = torch.device("cuda", 0)
    mg.set_xcd_queues(args.xcd_queues)
    forms, cpu_all = {}, {}
    head = None
    if args.workload in ("all", "batched"):
        bf, cfg, cpu = batched_forms(args, torch, mg, dev)
        forms.update({f"batched_{k}": v for k, v in bf.items()})
        head = ("batched_fp64", cfg, cpu)
    if args.workload == "large2d" or (args.workload == "all" and not args.value_only):
        p = W.config("large2d")
        net, _ = (None, None) if args.no_learned else load_net(2, p.N)
        f2 = single_forms("large2d", [p], args, torch, mg, dev, learned=net,
                          variants=[("fp64", "fp64", False), ("mixed", "mixed", False),
                                    ("fp64_learned", "fp64", True), ("mixed_learned", "mixed", True)])
        cpu = None if args.no_cpu_baseline else cpu_baseline([p], [512], "2D n=255 M=1024", one_thread_rows=256)
        for k, v in f2.items():
            v["cpu_baseline"] = cpu
            forms[f"large2d_{k}"] = v
        if head is None:
            head = ("large2d_fp64", {"workload": "large2d: 2D n=255 M=1024 alpha=0.5 r=3 k=10 leaf 16 V(1,1), "
                                                 "manufactured u=t^0.5 sin(pi x) sin(pi y)",
                                     "N": p.N, "M": p.M, "tol": args.tol}, cpu)
    if (args.workload == "learned2d" or (args.workload == "all" and not args.value_only)) and not args.no_learned:
        import numpy as np
        probs = [W.warm_start_family(2, 255, 1024, np.random.default_rng([100001, i])) for i in range(2)]
        net, meta = load_net(2, probs[0].N)
        if net is not None:
            f5 = single_forms("learned2d", probs, args, torch, mg, dev, learned=net,
                              variants=[("fp64", "fp64", False), ("mixed", "mixed", False),
                                        ("fp64_learned", "fp64", True), ("mixed_learned", "mixed", True)])
            cpu = None if args.no_cpu_baseline else cpu_baseline(probs[:1], [512], "held-out 2D n=255 M=1024",
                                                                 one_thread_rows=256)
            for k, v in f5.items():
                v["cpu_baseline"] = cpu
                v["network"] = {key: meta.get(key) for key in ("dim", "n", "M", "count", "steps", "val_loss")}
                forms[f"learned2d_{k}"] = v
            if head is None and "fp64" in f5:
                head = ("learned2d_fp64", {"workload": "learned2d: 2D n=255 M=1024, two held-out instances of the "
                                                       "warm-start family (seeds [100001, i])",
                                           "N": probs[0].N, "M": probs[0].M, "instances": 2, "tol": args.tol}, cpu)
    if args.workload == "large1d" or (args.workload == "all" and not args.value_only):
        probs = [W.config("large1d", a) for a in (0.3, 0.5, 0.7)]
        f2 = single_forms("large1d", probs, args, torch, mg, dev)
        cpu = None if args.no_cpu_baseline else cpu_baseline(probs, [4096, 4096, 4096], "1D n=1023 M=4096",
                                                             one_thread_rows=1024)
        for k, v in f2.items():
            v["cpu_baseline"] = cpu
            forms[f"large1d_{k}"] = v
        if head is None:
            head = ("large1d_fp64", {"workload": "large1d: 1D n=1023 M=4096 alpha in {0.3,0.5,0.7} r=(2-a)/a "
                                                 "k=10 leaf 16 V(1,1), three instances as one batch",
                                     "N": 1023, "M": 4096, "instances": 3, "tol": args.tol}, cpu)
    if args.workload == "paper1d" or (args.workload == "all" and not args.value_only):
        forms["paper1d_fp64"] = paper_forms(args, torch, mg, dev)
        if head is None:
            head = ("paper1d_fp64", {"workload": "paper1d: the paper's 1D experiment, N x M = 2048 x 2048, "
                                                 "alpha in {0.2,0.4,0.6,0.8}, k=20, V(0,1), to 1e-10",
                                     "N": 2047, "M": 2048, "instances": 4, "tol": 1e-10}, None)
    if args.workload == "small1d":
        p = W.config("small1d")
        f1 = single_forms("small1d", [p], args, torch, mg, dev)
        forms.update({f"small1d_{k}": v for k, v in f1.items()})
        head = ("small1d_fp64", {"workload": "small1d: 1D n=63 M=128 alpha=0.5 r=3 k=8", "tol": args.tol}, None)
    # each form's rate against the float64 form of its workload
    for name, v in forms.items():
        wl, _, form = name.partition("_")
        base = forms.get(f"{wl}_fp64", {}).get("value")
        if form != "fp64" and base and v.get("value"):
            v["vs_fp64"] = v["value"] / base
    key, cfg, cpu = head
    hv = forms[key]
    out = {
        "metric": "space-time unknowns (N*M)/s to 1e-8 rel. residual: plain FP64 vs mixed+learned",
        "value": hv["value"], "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": hv["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (seeded random-Fourier and manufactured sources)",
        "config": cfg, "roofline": hv.get("roofline"),
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    out["forms"] = forms
    out["kernel_source_sha256"] = kernel_sha()
    out["schedule_source_sha256"] = schedule_sha()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
