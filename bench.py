#!/usr/bin/env python3
"""Throughput of the H-matrix MGWR solver on one MI355X.

Metric: space-time unknowns (N*M) per second to 1e-8 relative residual
(||b - A u||_inf <= 1e-8 ||b||_inf, float64 residual).

Workload (default, "large1d"): 1D time-fractional heat equation on (0, 1),
n = 1023 interior points, M = 4096 graded steps t_j = (j/M)^r with
r = (2 - alpha)/alpha, alpha in {0.3, 0.5, 0.7}, k = 10, leaf 16, V(1,1),
manufactured solution u = t^alpha sin(pi x), zero initial guess.  One step =
one solve of each of the three instances.  Sources are synthetic (closed form)
and resident in HBM before timing starts.

Prints one JSON line.  `value` is the plain float64 solver; the mixed-precision
forms (float32 inner cycles, with float32 or bfloat16 low-rank factors) and the
learned warm start are reported next to it under `forms`.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 (vector and matrix)
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

# HBM bytes per batched launch of pipeline_kernel<double> on the large1d
# workload, from rocprofv3 FETCH_SIZE / WRITE_SIZE runs scaled by what the same
# counters read for a 1 GiB device copy (--copy-probe): fetch x 2.000, write x
# 1.000.  Valid only for the kernel source they were taken on.
TRAFFIC_KERNEL_SHA256 = "b7ae4a201aef9f5b3cc2bb90cb065cadb4a1424ed31840ca864a7264db117436"
TRAFFIC_BYTES = {"large1d": (2.000 * 23847061.4 + 1.000 * 8656866.5) * 1024}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large1d", choices=["large1d", "large2d", "small1d", "batched"])
    ap.add_argument("--batch-count", type=int, default=64, help="instances of the batched workload")
    ap.add_argument("--batch-schedule", default="auto", choices=["auto", "autotune"],
                    help="batched workload: the plans' AUTO rule, or the autotuner per (n, M) bucket")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--value-only", action="store_true",
                    help="time only the batched float64 step behind `value` (no other forms, no CPU baseline): "
                         "the command the kernel profiles are taken on")
    ap.add_argument("--cpu-repeats", type=int, default=3)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB three times on the device (counter calibration) and exit")
    return ap.parse_args()


def copy_probe():
    import torch
    x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": x.numel() * 8, "copies": 3}), flush=True)


def traffic_for(workload):
    """Counter-measured HBM bytes per launch, or None when the kernel source
    differs from the one the counters were taken on."""
    import hashlib
    src = os.path.join(ROOT, "paper_1706_07632_amd", "csrc", "kernels.hip")
    try:
        with open(src, "rb") as fh:
            digest = hashlib.sha256(fh.read()).hexdigest()
    except OSError:
        return None
    if digest != TRAFFIC_KERNEL_SHA256:
        return None
    return TRAFFIC_BYTES.get(workload)


def instances(workload):
    import workloads as W
    if workload == "large1d":
        return [W.config("large1d", a) for a in (0.3, 0.5, 0.7)]
    return [W.config(workload)]


def time_form(plans, fs, us, tol, steps, warmup, torch, warm_start=False):
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
            _, st = pl.solve(f, tol=tol, u=u, warm_start=warm_start)
            stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = [pl.timing() for pl in plans]
    for pl in plans:
        pl.timing(False)
    return t1 - t0, stats, timing


def time_batch(batch, fs, us, tol, steps, warmup, torch, warm_start=False, plans=()):
    """Wall time of `steps` batch solves after `warmup` untimed ones; kernel
    timing (the batch's and that of `plans`, which time their own staged
    launches) covers the timed solves only."""
    stats = []
    for _ in range(warmup):
        batch.solve(fs, tol=tol, us=us, warm_start=warm_start)
    batch.timing(True)
    for pl in plans:
        pl.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st = batch.solve(fs, tol=tol, us=us, warm_start=warm_start)
        stats.extend(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = batch.timing(False)
    return t1 - t0, stats, [tm]


def merge_timing(timings):
    out = {}
    for tm in timings:
        for cls, v in tm.items():
            o = out.setdefault(cls, {"launches": 0, "ms": 0.0, "flops": 0.0, "bytes": 0.0})
            for key in o:
                o[key] += v[key]
    return out


def cpu_baseline(probs, repeats):
    """The float64 oracle (direct time marching) on the host cores: one full
    solve of each instance, median of `repeats`; assembly of R~ excluded."""
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max(int(x.get("num_threads", 1)) for x in threadpool_info()) if threadpool_info() else 1
    except Exception:
        cores = os.cpu_count() or 1
    per = []
    total_unknowns = 0
    for p in probs:
        Rt = oracle.hmatrix_dense(p.t, p.alpha, p.k, p.leaf)
        B = oracle.rhs(p.f, p.t, p.alpha, p.g)
        times = []
        for _ in range(repeats):
            t0 = time.perf_counter()
            oracle.timestep_solve(Rt, B, p.dim, p.n, p.length)
            times.append(time.perf_counter() - t0)
        per.append(float(np.median(times)))
        total_unknowns += p.N * p.M
    return {"value": total_unknowns / sum(per), "unit": "unknowns/s", "cores": cores, "kind": "oracle",
            "sample": f"full direct solve of each of the {len(probs)} instances, median of {repeats}, "
                      f"R~ assembly excluded ({sum(per):.2f} s per pass)"}


def learned_forms(args, probs, fs, us, unknowns, mg, torch):
    """Warm-started solves (the trained network's prediction, judged by the
    float64 residual), float64 and mixed, the instances batched as for `value`."""
    from paper_1706_07632_amd import learn
    dim = probs[0].dim
    path = os.path.join(ROOT, "paper_1706_07632_amd", "weights", f"warm{dim}d.npz")
    if not os.path.exists(path):
        return {}
    net, meta = learn.load(path, max(p.N for p in probs))
    out = {}
    for name, precision in (("fp64_learned", "fp64"), ("mixed_learned", "mixed")):
        plans = [mg.Plan(p.dim, p.n, p.M, p.alpha, k=p.k, r=p.r, t=p.t, length=p.length, leaf=p.leaf,
                         precision=precision, inner_cycles=1).bind() for p in probs]
        for pl in plans:
            learn.attach(pl, net)
        if len(plans) > 1:
            batch = mg.Batch(plans).bind()
            secs, st, _ = time_batch(batch, fs, us, args.tol, args.steps, args.warmup, torch, warm_start=True)
        else:
            secs, st, _ = time_form(plans, fs, us, args.tol, args.steps, args.warmup, torch, warm_start=True)
        last = st[-len(probs):]
        out[name] = {"value": unknowns * args.steps / secs, "ms_per_step": 1e3 * secs / args.steps,
                     "cycles": [s["cycles"] for s in last],
                     "used_warm_start": [s["used_warm_start"] for s in last],
                     "warm_res0_rel": [None if s["warm_res0"] != s["warm_res0"] else s["warm_res0"] / s["bnorm"]
                                       for s in last],
                     "rel_res": [s["res"] / s["bnorm"] for s in last],
                     "network": {k: meta[k] for k in ("dim", "n", "M", "count", "steps", "val_loss")}}
    return out


def batched_main(args):
    """The batched workload: `batch_count` uneven 2D instances of the
    random-Fourier family (sides {63, 127, 255}, M in {256..2048}, alpha ~
    U[0.2, 0.9]) solved together: the schedule of each instance by the AUTO
    rule (or, with --batch-schedule autotune, by the autotuner on the first
    instance of its (n, M) bucket), the pipelined instances in one
    merged launch (graph-replayed), the staged ones side by side after it."""
    import torch

    import paper_1706_07632_amd as mg
    import workloads as W
    dev = torch.device("cuda", 0)
    probs = W.batched_instances(count=args.batch_count, build_f="modes")
    fs = []
    for p in probs:
        f = torch.zeros((p.M, p.N), dtype=torch.float64, device=dev)
        for kvec, prof in p.modes:
            f.add_(torch.outer(torch.as_tensor(prof, dtype=torch.float64, device=dev),
                               torch.as_tensor(W.sine_mode(p.n, 2, 1.0, kvec), dtype=torch.float64, device=dev)))
        fs.append(f)
    us = [torch.empty_like(f) for f in fs]
    unknowns = sum(p.N * p.M for p in probs)
    forms, out_timing, tuned = {}, None, {}
    timed_s = 0.0
    for name, precision in (("fp64", "fp64"), ("mixed_fp32", "mixed"), ("mixed_bf16", "mixed_bf16")):
        if name != "fp64" and args.no_mixed:
            continue
        plans = [mg.Plan(2, p.n, p.M, p.alpha, k=p.k, r=p.r, t=p.t, precision=precision, inner_cycles=1).bind()
                 for p in probs]
        t0 = time.perf_counter()
        for p, pl, f, u in zip(probs, plans, fs, us):
            key = (p.n, p.M, precision)
            if key not in tuned and args.batch_schedule == "autotune":
                tuned[key] = pl.autotune(f, tol=args.tol, u=u)
        tune_s = time.perf_counter() - t0
        batch = mg.Batch(plans, graph=True).bind()
        secs, stats, timing = time_batch(batch, fs, us, args.tol, args.steps, args.warmup, torch, plans=plans)
        if out_timing is None:
            timed_s = secs
        last = stats[-len(probs):]
        forms[name] = {"value": unknowns * args.steps / secs, "ms_per_step": 1e3 * secs / args.steps,
                       "cycles_total": sum(s["cycles"] for s in last),
                       "max_rel_res": max(s["res"] / s["bnorm"] for s in last),
                       "autotune_s": round(tune_s, 2), "graph_replays": batch.graph_replays()}
        if out_timing is None:
            out_timing = merge_timing(timing + [pl.timing() for pl in plans])
        batch.close()
        for pl in plans:
            pl.close()
    tm = out_timing
    dom = max(tm, key=lambda k: tm[k]["ms"])
    sm = tm[dom]
    # Staged instances run side by side on several streams, so launches of the
    # dominant class overlap and their summed durations exceed the wall time:
    # the rate is taken over the timed wall time instead (a lower bound).
    achieved = sm["flops"] / timed_s / 1e12 if timed_s > 0 else 0.0
    per_launch = sm["flops"] / (sm["ms"] * 1e-3) / 1e12 if sm["ms"] > 0 else 0.0
    out = {
        "metric": "space-time unknowns (N*M)/s to 1e-8 rel. residual, batched uneven 2D instances",
        "value": forms["fp64"]["value"], "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": forms["fp64"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded random-Fourier sources)",
        "config": {"workload": f"batched: {len(probs)} 2D instances, sides {{63,127,255}}, M {{256..2048}}, "
                               "alpha~U[0.2,0.9], r=(2-a)/a, k=10, leaf 16, V(1,1)",
                   "instances": len(probs), "unknowns": unknowns, "tol": args.tol,
                   "schedules": ({f"n{k[0]}_M{k[1]}_{k[2]}": v for k, v in sorted(tuned.items())}
                                 if args.batch_schedule == "autotune" else
                                 "auto: pipelined when the finest half-sweep has at most 256 chains of 16 columns, "
                                 "else staged with the coarse levels pipelined")},
        "roofline": {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                     "basis": "algorithmic flops of the class over the timed wall time (launches of several "
                              "streams overlap)",
                     "per_launch_achieved": per_launch,
                     "avg_launch_us": 1e3 * sm["ms"] / max(1, sm["launches"]), "launches": sm["launches"]},
        "forms": forms,
        "kernels": {k: {"launches": v["launches"], "ms": round(v["ms"], 3)} for k, v in tm.items() if v["launches"]},
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.value_only:
        args.no_mixed = args.no_learned = args.no_cpu_baseline = True
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU (multi-GPU sharding is not implemented); --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "batched":
        batched_main(args)
        return
    import numpy as np
    import torch

    import paper_1706_07632_amd as mg

    dev = torch.device("cuda", 0)
    probs = instances(args.workload)
    fs = [torch.as_tensor(p.f, dtype=torch.float64, device=dev) for p in probs]
    us = [torch.empty_like(f) for f in fs]
    plans = [mg.Plan(p.dim, p.n, p.M, p.alpha, k=p.k, r=p.r, t=p.t, length=p.length, leaf=p.leaf).bind()
             for p in probs]
    unknowns = sum(p.N * p.M for p in probs)

    # one step = the instances solved together: their pipelined cycles are
    # merged into one launch (a single instance uses the plan directly)
    if len(plans) > 1:
        batch = mg.Batch(plans).bind()
        secs, stats, timing = time_batch(batch, fs, us, args.tol, args.steps, args.warmup, torch)
        seq_secs = None
        if not args.value_only:
            seq_secs, seq_stats, _ = time_form(plans, fs, us, args.tol, args.steps, args.warmup, torch)
    else:
        secs, stats, timing = time_form(plans, fs, us, args.tol, args.steps, args.warmup, torch)
        seq_secs = None
    tm = merge_timing(timing)
    ms_per_step = 1e3 * secs / args.steps
    value = unknowns * args.steps / secs
    # dominant kernel: the time-pipelined cycle kernel when it ran, else the smoother
    dom = "pipe64" if tm["pipe64"]["launches"] else "smooth64"
    dom_name = ("pipeline_kernel<double> (K pipelined V-cycles: zebra line relaxation with H-forward "
                "substitution, defects, grid transfers)" if dom == "pipe64" else
                "march_kernel<double, SMOOTH> (zebra line relaxation, H-forward substitution)")
    sm = tm[dom]
    achieved = sm["flops"] / (sm["ms"] * 1e-3) / 1e12 if sm["ms"] > 0 else 0.0
    avg_launch_us = 1e3 * sm["ms"] / max(1, sm["launches"])
    forms = {"fp64": {"value": value, "ms_per_step": ms_per_step,
                      "cycles": [s["cycles"] for s in stats[:len(probs)]],
                      "rel_res": [s["res"] / s["bnorm"] for s in stats[:len(probs)]]}}
    if seq_secs is not None:
        forms["fp64_one_instance_at_a_time"] = {"value": unknowns * args.steps / seq_secs,
                                                "ms_per_step": 1e3 * seq_secs / args.steps}
    kernels = {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                   "avg_us": round(1e3 * v["ms"] / max(1, v["launches"]), 2),
                   "TFLOP/s": round(v["flops"] / max(v["ms"], 1e-9) * 1e-9, 3),
                   "GB/s": round(v["bytes"] / max(v["ms"], 1e-9) * 1e-6, 1)} for k, v in tm.items() if v["launches"]}

    for name, precision in (("mixed_fp32", "mixed"), ("mixed_bf16", "mixed_bf16")):
        if args.no_mixed:
            break
        mplans = [mg.Plan(p.dim, p.n, p.M, p.alpha, k=p.k, r=p.r, t=p.t, length=p.length, leaf=p.leaf,
                          precision=precision, inner_cycles=1).bind() for p in probs]
        if len(mplans) > 1:
            mbatch = mg.Batch(mplans).bind()
            msecs, mstats, mtiming = time_batch(mbatch, fs, us, args.tol, args.steps, args.warmup, torch)
        else:
            msecs, mstats, mtiming = time_form(mplans, fs, us, args.tol, args.steps, args.warmup, torch)
        mtm = merge_timing(mtiming)
        forms[name] = {"value": unknowns * args.steps / msecs, "ms_per_step": 1e3 * msecs / args.steps,
                       "cycles": [s["cycles"] for s in mstats[:len(probs)]],
                       "refinements": [s["refinements"] for s in mstats[:len(probs)]],
                       "rel_res": [s["res"] / s["bnorm"] for s in mstats[:len(probs)]]}
        forms[name]["kernels"] = {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                                      "avg_us": round(1e3 * v["ms"] / max(1, v["launches"]), 2)}
                                  for k, v in mtm.items() if v["launches"]}

    if not args.no_learned:
        forms.update(learned_forms(args, probs, fs, us, unknowns, mg, torch))

    out = {
        "metric": "space-time unknowns (N*M)/s to 1e-8 rel. residual (plain FP64; mixed and learned forms under forms)",
        "value": value,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (manufactured closed-form source)",
        "config": {"workload": args.workload if args.workload != "large1d" else
                   "large1d: 1D n=1023 M=4096 alpha in {0.3,0.5,0.7} r=(2-a)/a k=10 leaf=16 V(1,1)",
                   "N": probs[0].N, "M": probs[0].M, "instances": len(probs), "tol": args.tol},
        "roofline": {"bound": "mfma", "kernel": dom_name,
                     "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": traffic_for(args.workload) if dom == "pipe64" else None,
                     "algorithmic_bytes": sm["bytes"] / max(1, sm["launches"]),
                     "avg_launch_us": avg_launch_us, "launches": sm["launches"]},
        "forms": forms,
        "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(probs, args.cpu_repeats)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
