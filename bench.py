#!/usr/bin/env python3
"""Benchmark of the batched shifted-rotated evaluation on one MI355X.

One step = one pass of the evaluation hot path over the whole batched
workload: 6 functions x D in {10, 30, 50, 100} x 10 instances x 51 runs x 100
points = 1,224,000 evaluations (FP64 shift, FP32 MFMA rotation, compensated
FP32 objective reduction), inputs resident in HBM.  Inputs are synthetic,
seeded, uniform in [-100, 100]^D; several replicas of the input set rotate
from step to step so that the working set exceeds the 256 MB Infinity Cache.

Prints one JSON line: the throughput (evaluations / s), the roofline of the
dominant kernel (the D = 100 launch, bound by FP32 MFMA; achieved TFLOP/s
from HIP events around that launch on its own stream), and the FP64 CPU
oracle timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
FUNC_NAMES = ["ellipsoid", "rosenbrock", "rastrigin", "schwefel", "griewank", "ackley"]

# HBM traffic of the dominant kernel, from the FETCH_SIZE / WRITE_SIZE counter
# summary committed beside the kernel-trace summaries.  The figure is used
# only while the kernel's sources hash to the value recorded with it.
HBM_PROFILE = os.path.join(ROOT, "profiles", "k_eval_small_D100_hbm_counters.txt")
KERNEL_SOURCES = ["eval.hip", "tile.h", "objective_f32.h", "runtime.h", "runtime.hip", "common.h"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2505_17430_amd", "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the D=100 evaluation kernel, or None when the
    counter summary is missing or was taken on other kernel sources."""
    try:
        with open(HBM_PROFILE) as f:
            kv = dict(l.split(":", 1) for l in f if ":" in l and not l.startswith(" "))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--replicas", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--no-fp64", action="store_true",
                    help="c2: leave out the FP64 comparison legs and C1 (vs_baseline is then null); for "
                         "profiler runs, where their 12,000 small launches are slow")
    ap.add_argument("--one-precision", action="store_true",
                    help="c2: time only --precision (default: also the other single precision, reported beside)")
    ap.add_argument("--workload", default="c2",
                    choices=["c1", "c2", "c3", "c4", "c5", "lshade", "lshade_rs", "jade", "psode", "cso", "ops",
                             "copy"],
                    help="c2 (default): batched evaluation sweep; c1: plain DE; c3: batched PSO; "
                         "c4: batched SHADE; c5: D=1000 evaluation; lshade: the c4 runs as L-SHADE; "
                         "lshade_rs: the c4 runs as L-SHADE-Restart; jade: the c4 runs as JADE with the "
                         "muF/muCR observer; "
                         "psode: the case study's PSO/DE hybrid, batched; "
                         "cso: the large-scale study's CSO runs at D=1000; "
                         "ops: the unfused DE and PSO generation steps at scale; "
                         "copy: 512 MiB device copy "
                         "(calibrates the HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(target_s):
    """FP64 oracle on a bounded sample of the same workload, all host cores."""
    import concurrent.futures as cf
    import oracle as O

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(cores, 64))
    groups = W.c2_groups()
    inst = {}
    for (f, d, k, _) in groups:
        inst[(f, d, k)] = O.instance(f, d, k, W.INSTANCE_SEED)

    def chunk(args):
        f, d, k, X = args
        o, M = inst[(f, d, k)]
        O.errors_soa_f32(f, o, M, X)
        return X.shape[1]

    # calibrate on a few points per group, then scale the sample to ~target_s
    # (capped at the full 5100 points per group, repeating the full sweep
    # when even that is shorter than the target)
    per = 16
    jobs = [(f, d, k, W.uniform_points(W.group_seed(f, d, k, 1), d, per)) for (f, d, k, _) in groups]
    with cf.ThreadPoolExecutor(cores) as ex:
        t0 = time.perf_counter()
        sum(ex.map(chunk, jobs))
        dt = time.perf_counter() - t0
        want = per * target_s / max(dt, 1e-4)
        per = int(max(16, min(5100, want)))
        jobs = [(f, d, k, W.uniform_points(W.group_seed(f, d, k, 2), d, per)) for (f, d, k, _) in groups]
        t0 = time.perf_counter()
        n = 0
        reps = 0
        # whole passes over the sample until the target time is reached
        while reps < 400 and (reps == 0 or time.perf_counter() - t0 < target_s):
            n += sum(ex.map(chunk, jobs))
            reps += 1
        dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{reps} x {per} points per group x {len(groups)} groups (all 6 functions x "
                      f"D in 10,30,50,100 x 10 instances, FP64 C oracle, threads over groups), "
                      f"{n} evaluations in {dt:.1f} s"}


def cpu_accuracy(keep, precision_name, per=8):
    """Part of the CPU-baseline leg: the FP64 oracle evaluates a seeded sample
    of the very points the timed GPU calls evaluated (copied to the host) and
    the GPU's errors there are compared with it, per function, against the
    stated bound max(1e-6, 1e-5 e).  keep: (func, dim, inst, x, err) device
    tensors of one replica, err holding that precision's last results."""
    import oracle as O
    from tests.tolerance import tolerance
    rng = np.random.default_rng(17)
    strict, stated, d100 = {}, {}, {}
    n = 0
    for (f, d, k, x, e) in keep:
        idx = np.sort(rng.choice(x.shape[1], size=per, replace=False))
        X = x[:, idx].cpu().numpy()
        eg = e[idx].cpu().numpy().astype(np.float64)
        o, M = O.instance(f, d, k, W.INSTANCE_SEED)
        eo = O.errors_soa_f32(f, o, M, X)
        dev = np.abs(eg - eo)
        r = float(np.max(dev / np.maximum(1e-6, 1e-5 * np.abs(eo))))
        rs = float(np.max(dev / tolerance(f, o, M, X, eo)))
        name = FUNC_NAMES[f]
        strict[name] = max(strict.get(name, 0.0), r)
        stated[name] = max(stated.get(name, 0.0), rs)
        if d == 100:
            d100[name] = max(d100.get(name, 0.0), r)
        n += per
    return {"bound": "|de| <= max(1e-6, 1e-5 e) vs the FP64 oracle at the same float point; Rosenbrock "
                     "adds 4 eps32 |x - o|_2 |grad_z e|_1 (the float rounding of the shifted point)",
            "precision": precision_name, "points": n,
            "worst_dev_over_max_1e-6_1e-5e": {k: round(v, 4) for k, v in strict.items()},
            "worst_dev_over_max_1e-6_1e-5e_at_d100": {k: round(v, 4) for k, v in d100.items()},
            "worst_dev_over_stated_bound": {k: round(v, 4) for k, v in stated.items()},
            "within_bound": all(v <= 1.0 for v in stated.values())}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              f"(runs shard across GPUs with no exchange, so one GPU's share is the measured unit)", file=sys.stderr)
        sys.exit(2)
    if a.workload != "c2":
        return run_workload(a)
    import torch
    from paper_2505_17430_amd import sevo as S

    prec = S.FP32 if a.precision == "fp32" else S.SPLIT_BF16
    ctx = S.Context(0, W.BASE_SEED, W.INSTANCE_SEED)
    stream = torch.cuda.current_stream()
    groups = W.c2_groups()
    by_dim = {d: [g for g in groups if g[1] == d] for d in W.C2_DIMS}

    def replicas(dtype, count):
        """`count` replicas of the full input set, generated on the device
        (plumbing only): per dimension the prepared batch and the
        (func, dim, inst, x, err) tensors."""
        gen = torch.Generator(device="cuda")
        out = []
        for r in range(count):
            gen.manual_seed(W.BASE_SEED + r)
            per_dim = {}
            for d, gs in by_dim.items():
                items, keep = [], []
                for (f, dd, k, n) in gs:
                    x = torch.empty((dd, n), dtype=torch.float32, device="cuda")
                    x.uniform_(W.LB, W.UB, generator=gen)
                    x = x.to(dtype)
                    e = torch.empty(n, dtype=dtype, device="cuda")
                    items.append((S.problem(f, dd), k, x, e))
                    keep.append((f, dd, k, x, e))
                per_dim[d] = (items, S.Context.prepare_batch(items), keep)
            out.append(per_dim)
        torch.cuda.synchronize()
        return out

    reps = replicas(torch.float32, a.replicas)
    n_evals = sum(g[3] for g in groups)
    bytes_in = sum(g[3] * (4 * g[1] + 4) for g in groups)

    def timed(prec, reps, steps, warmup, tune=True):
        """Time `steps` steps of the sweep in one precision; returns
        (ms per step, mean D=100 launch ms, tuned launch shapes, ms per step
        of the eager calls).  A step launches one prepared plan
        (sevo_plan_evaluate: descriptor tables resident, launch shapes fixed,
        no host work per call) per dimension class and replica; the same
        sweep through one sevo_evaluate_batch call per class is timed after
        it.  Both do all the work of every step."""
        # launch shapes chosen by the library's autotuner on the first replica
        # (setup, outside the timed region; the choice does not change results)
        tuned = {}
        if tune and not a.no_tune:
            for d in W.C2_DIMS:
                tuned.update(ctx.tune_evaluate(reps[0][d][1], precision=prec, stream=stream))

        plans = [{d: ctx.plan_evaluate(rep[d][1], precision=prec) for d in W.C2_DIMS} for rep in reps]

        def step(i, ev=None, eager=False):
            rep, pl = reps[i % len(reps)], plans[i % len(reps)]
            for d in W.C2_DIMS:
                if ev is not None and d == 100:
                    ev[0].record(stream)
                if eager:
                    ctx.evaluate_batch(rep[d][1], precision=prec, stream=stream)
                else:
                    pl[d].launch(stream)
                if ev is not None and d == 100:
                    ev[1].record(stream)

        def run(eager):
            for w in range(warmup):
                step(w, eager=eager)
            torch.cuda.synchronize()
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(steps)]
            t_start = torch.cuda.Event(enable_timing=True)
            t_end = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            t_start.record(stream)
            for s in range(steps):
                step(s, evs[s], eager)
            t_end.record(stream)
            torch.cuda.synchronize()
            ctx.sync(stream)
            return (t_start.elapsed_time(t_end) / steps,
                    float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs])))

        ms, d100 = run(False)
        ms_eager, _ = run(True)
        # leave replica 0 holding this precision's results (for the accuracy sample)
        step(0)
        torch.cuda.synchronize()
        for pl in plans:
            for p in pl.values():
                p.close()
        return ms, d100, tuned, ms_eager

    def keep0(reps):
        return [t for d in W.C2_DIMS for t in reps[0][d][2]]

    n100 = sum(g[3] for g in by_dim[100])
    flops100 = 2.0 * 100 * 100 * n100
    ms_step, d100_ms, tuned, ms_eager = timed(prec, reps, a.steps, a.warmup)
    value = n_evals / (ms_step / 1e3)
    accuracy = {}
    if not a.no_cpu:
        accuracy[a.precision if a.precision == "fp32" else "split_bf16"] = cpu_accuracy(keep0(reps), a.precision)
    legs = {}
    if not a.one_precision:
        # the other single precision, reported beside (each meets the
        # evaluation tolerance in the parity tests)
        other = S.SPLIT_BF16 if prec == S.FP32 else S.FP32
        oname = "split_bf16" if other == S.SPLIT_BF16 else "fp32"
        o_ms, o_d100, o_tuned, o_eager = timed(other, reps, a.steps, a.warmup)
        if not a.no_cpu:
            accuracy[oname] = cpu_accuracy(keep0(reps), oname)
        for name, pr, ms_, d_, me_ in ((a.precision, prec, ms_step, d100_ms, ms_eager),
                                       (oname, other, o_ms, o_d100, o_eager)):
            legs["split_bf16" if name == "bf16" else name] = {
                "ms_per_step": round(ms_, 4), "evals_per_s": round(n_evals / (ms_ / 1e3), 1),
                "eager_ms_per_step": round(me_, 4),
                "d100_kernel_ms": round(d_, 4),
                "d100_tflops_fp32_equiv": round(flops100 / (d_ / 1e3) / 1e12, 3)}
    fp64, c1, speedup = None, None, None
    if not a.no_fp64:
        # the plain FP64 path over the same sweep: the same batched calls and
        # timing with double inputs, shift, rotation and sum (k_eval_f64), one
        # replica (its working set alone exceeds the Infinity Cache)
        reps64 = replicas(torch.float64, 1)
        f64_steps = max(1, min(a.steps, 10))
        ms64, d100_64, _, ms64_eager = timed(S.FP64, reps64, f64_steps, 1, tune=False)
        # the same in one launch per run: each run's 100-point population of each
        # (function, D, instance) evaluated by its own sevo_evaluate call
        singles = [(S.problem(f, d), k, x[:, r * W.C2_POINTS_PER_RUN:(r + 1) * W.C2_POINTS_PER_RUN],
                    e[r * W.C2_POINTS_PER_RUN:(r + 1) * W.C2_POINTS_PER_RUN])
                   for (f, d, k, x, e) in keep0(reps64) for r in range(W.C2_RUNS)]
        for (pb, k, x, e) in singles[:64]:
            ctx.evaluate(pb, k, x, e, n=x.shape[1], ld=x.stride(0), precision=S.FP64, stream=stream)
        torch.cuda.synchronize()
        p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        p0.record(stream)
        for (pb, k, x, e) in singles:
            ctx.evaluate(pb, k, x, e, n=x.shape[1], ld=x.stride(0), precision=S.FP64, stream=stream)
        p1.record(stream)
        torch.cuda.synchronize()
        ms_per_run = p0.elapsed_time(p1)
        del reps64, singles
        fp64 = {"batched": {"ms_per_step": round(ms64, 4), "evals_per_s": round(n_evals / (ms64 / 1e3), 1),
                            "eager_ms_per_step": round(ms64_eager, 4),
                            "d100_kernel_ms": round(d100_64, 4), "steps": f64_steps,
                            "path": "precision FP64 (k_eval_f64), the same plans, calls and "
                                    "event timing as the single-precision legs"},
                "one_run_per_launch": {"ms_per_step": round(ms_per_run, 3),
                                       "evals_per_s": round(n_evals / (ms_per_run / 1e3), 1),
                                       "launches_per_step": len(groups) * W.C2_RUNS,
                                       "path": "one sevo_evaluate call (FP64) per run's 100-point population"}}
        speedup = ms64 / ms_step
        # C1, the plain DE configuration: the fused FP32 run (graph replay of a
        # plan) against the plain FP64 path's one launch per step
        c1_descs = _run_descs(S, [(S.ALGO_DE, S.RASTRIGIN, 10, 50, 50 * 1001, 0, 0)])
        c1_64, c1r64 = _time_runs(ctx, S, torch, c1_descs, S.FP64, 3, 1, trace_len=250)
        c1_32, c1r32 = _time_runs(ctx, S, torch, c1_descs, S.FP32, 3, 1, trace_len=250, graph=True)
        c1 = {"workload": "plain DE rand/1/bin, one run: Rastrigin D=10, NP=50, F=0.5, CR=0.9, 1000 generations",
              "plain_fp64_ms": round(c1_64, 3), "fused_fp32_ms": round(c1_32, 3),
              "speedup_fused_vs_plain": round(c1_64 / c1_32, 2),
              "evals": int(c1r64[0].fes), "best_e_fp64": c1r64[0].best_e, "best_e_fp32": c1r32[0].best_e}

    achieved = flops100 / (d100_ms / 1e3) / 1e12
    if prec == S.FP32:
        peak, kname = PEAK_FP32_MFMA_TFLOPS, "k_eval_small<25> (D=100 group: 60 items x 5100 points)"
    else:
        # D = 100 runs k_eval_small_bf16<25>: 96 of the 100 coordinates in
        # six bf16 products on the bf16 MFMA, counted against its own peak
        # (the other 4 run on the float MFMA and are not counted)
        achieved *= 6 * 96 / 100
        peak, kname = PEAK_BF16_MFMA_TFLOPS, "k_eval_small_bf16<25> (D=100 group: 60 items x 5100 points)"
    traffic = measured_traffic() if prec == S.FP32 else None
    roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": None if traffic is None else int(traffic),
            "traffic_unit": "HBM bytes per launch (counters, copy-calibrated)",
            "algorithmic_bytes": int(n100 * (4 * 100 + 4)),
            "kernel": kname,
            "kernel_ms": round(d100_ms, 4)}
    out = {
        "metric": "function evals/sec, batched FP32/split-BF16 vs plain FP64, at stated rel. error",
        "value": round(value, 1),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 4),
        "eager_ms_per_step": round(ms_eager, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None if speedup is None else round(speedup, 3),
        "vs_baseline_is": "speed-up over the plain FP64 path on the same sweep (fp64.batched), "
                          "at the asserted bound max(1e-6, 1e-5 e)",
        "dtype": "f32" if prec == S.FP32 else "bf16x6",
        "data": "synthetic",
        "config": {"workload": "batched evaluation: 6 functions x D in {10,30,50,100} x 10 "
                               "instances x 51 runs x 100 points, shifted-rotated, "
                               + ("FP32 MFMA rotation" if prec == S.FP32 else
                                  "split-bf16 rotation (three-term split, six bf16 products) for D=100, "
                                  "FP32 MFMA below")
                               + ", compensated FP32 objective",
                   "evals_per_step": n_evals, "input_bytes_per_step": bytes_in,
                   "replicas": a.replicas, "precision": a.precision,
                   "tiles_per_workgroup": {str(k): v for k, v in sorted(tuned.items())} or "resident grid",
                   "launch": "per step one prepared plan (sevo_plan_evaluate) per dimension class; "
                             "eager_ms_per_step: one sevo_evaluate_batch call per class instead",
                   "tolerance": "|de| <= max(1e-6, 1e-5 e) vs the FP64 oracle for ellipsoid, rastrigin, "
                                "schwefel, griewank, ackley; rosenbrock + 4 eps32 |x - o|_2 |grad_z e|_1 "
                                "(asserted by the parity tests; measured below under accuracy)"},
        "roofline": roof,
    }
    if fp64 is not None:
        out["fp64"] = fp64
        out["c1"] = c1
    if legs:
        out["precisions"] = legs
    if not a.no_cpu:
        out["accuracy"] = accuracy
        out["cpu_baseline"] = cpu_baseline(a.cpu_seconds)
    ctx.close()
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# Whole-run workloads (one line each; the default run measures only the
# evaluation sweep above).

def _line(metric, value, unit, steps, warmup, ms, config, dtype="f32", **extra):
    out = {"metric": metric, "value": round(value, 1), "unit": unit, "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
           "config": config}
    out.update(extra)
    print(json.dumps(out), flush=True)


_ALGO_LSHADE = 3      # SEVO_ALGO_LSHADE
_ALGO_PSODE = 4       # SEVO_ALGO_PSODE
_ALGO_CSO = 5         # SEVO_ALGO_CSO
_ALGO_JADE = 6        # SEVO_ALGO_JADE
_ALGO_LSHADE_RS = 7   # SEVO_ALGO_LSHADE_RS
# SPSO-2011 constants of the spherical update: w = 1 / (2 ln 2), c = 1/2 + ln 2
W_SPSO, C_SPSO = 1.0 / (2.0 * math.log(2.0)), 0.5 + math.log(2.0)


def _pso_settings(spec):
    """(w, c1, c2, topology, velocity) of a run spec: PSODE runs take the case
    study's PSO (spherical update, ring topology), CSO runs their phi in c1,
    the others inertia PSO."""
    if spec[0] == _ALGO_PSODE:
        return W_SPSO, C_SPSO, C_SPSO, 1, 1
    if spec[0] == _ALGO_CSO:
        return 0.7298, W.CSO_PHI, 1.49618, 0, 0
    return 0.7298, 1.49618, 1.49618, 0, 0


# L-SHADE-Restart's convergence threshold on the population's error spread
RESTART_TOL = 1e-8


def _algo_settings(algo):
    """(p, archive bound per individual) of an algorithm id (the product and
    the oracle number algorithms alike): L-SHADE and L-SHADE-Restart take
    L-SHADE's published p = 0.11 and archive 2.6 NP, JADE its p = 0.05 and
    archive NP, the others p = 0.1."""
    if algo in (_ALGO_LSHADE, _ALGO_LSHADE_RS):
        return 0.11, 2.6
    if algo == _ALGO_JADE:
        return 0.05, 1.0
    return 0.1, 2.6


def _run_descs(S, specs):
    """specs: list of (algo, func, dim, np, budget, instance, uid); final NP
    4 for L-SHADE, JADE's c = 0.1."""
    out = []
    for sp in specs:
        (algo, func, dim, np_, budget, inst, uid) = sp
        p, r_arc = _algo_settings(algo)
        w, c1, c2, topo, vel = _pso_settings(sp)
        d = S.RunDesc(S.problem(func, dim), inst, uid, algo, np_, budget, 0.5, 0.9, w,
                      c1, c2, 0.2 * (W.UB - W.LB), p, 6, r_arc, 4, topo, vel)
        d.c = 0.1
        d.restart_tol = RESTART_TOL
        out.append(d)
    return out


def _time_runs(ctx, S, torch, descs, precision, steps, warmup, trace_len=0, graph=False):
    """Mean ms per call of the runs.  graph: the FP32 runs as a plan whose
    launch is captured into a HIP graph once and replayed (persistent fused
    kernels + graph); otherwise one sevo_run call per step."""
    n = len(descs)
    res = torch.zeros((n, 32), dtype=torch.uint8, device="cuda")
    tr = torch.zeros(max(1, n * trace_len), device="cuda") if trace_len else None
    st = torch.cuda.current_stream()
    if graph:
        plan = ctx.plan_run(descs, res, tr, trace_len, precision=precision)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            plan.launch(torch.cuda.current_stream())
        call = g.replay
    else:
        def call():
            ctx.run(descs, res, tr, trace_len, precision=precision, stream=st)
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(steps):
        call()
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    raw = res.cpu().numpy().tobytes()
    rr = [S.RunResult.from_buffer_copy(raw[32 * k: 32 * (k + 1)]) for k in range(n)]
    return ms, rr


def _oracle_runs(specs, seconds):
    """The oracle on as many of the runs as fit ~seconds of host threads."""
    import concurrent.futures as cf
    import oracle as O
    cores = len(os.sched_getaffinity(0))
    keys = ["algo", "func", "dim", "np", "budget", "instance", "run_uid"]

    def one(sp):
        d = dict(zip(keys, sp))
        w, c1, c2, topo, vel = _pso_settings(sp)
        p, r_arc = _algo_settings(d["algo"])
        d.update(lb=W.LB, ub=W.UB, F=0.5, CR=0.9, w=w, c1=c1, c2=c2,
                 vmax=0.2 * (W.UB - W.LB), p=p, H=6, r_arc=r_arc, np_min=4, topology=topo,
                 velocity=vel, c=0.1, restart_tol=RESTART_TOL)
        return O.run(d, W.BASE_SEED, W.INSTANCE_SEED)[0]["fes"]

    t0 = time.perf_counter()
    n = 0
    done = 0
    with cf.ThreadPoolExecutor(cores) as ex:
        while time.perf_counter() - t0 < seconds and done < 50 * len(specs):
            batch = [specs[(done + k) % len(specs)] for k in range(cores)]
            n += sum(ex.map(one, batch))
            done += len(batch)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} runs to completion (cycling over {len(specs)} of the workload's "
                      f"runs), {n} evaluations in {dt:.1f} s"}


def run_workload(a):
    import torch
    if a.workload == "copy":
        src = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(a.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"workload": "copy", "bytes_read_per_copy": src.numel() * 4,
                          "bytes_written_per_copy": src.numel() * 4, "copies": a.steps}), flush=True)
        return
    from paper_2505_17430_amd import sevo as S
    ctx = S.Context(0, W.BASE_SEED, W.INSTANCE_SEED)
    steps = max(1, min(a.steps, 5))
    warm = 1
    metric = "function evals/sec, batched FP32/split-BF16 vs plain FP64, at stated rel. error"
    if a.workload == "ops":
        # the unfused generation steps at scale: 1024 populations of 2048 at
        # D = 30 on one instance, x and u 252 MB each (beyond the 256 MB
        # Infinity Cache together), one sevo_de_step / sevo_pso_step call per
        # generation (variation or update, evaluation, selection or bests)
        R, NP, D = 1024, 2048, 30
        steps = max(1, min(a.steps, 20))
        prob = S.problem(S.RASTRIGIN, D)
        n = R * NP
        st = torch.cuda.current_stream()
        x = torch.empty(R * D * NP, device="cuda"); u = torch.empty_like(x)
        ex = torch.empty(n, device="cuda"); eu = torch.empty_like(ex)
        de = lambda t: S.DEState(R, NP, NP, D * NP, 7, t, x.data_ptr(), ex.data_ptr(),  # noqa: E731
                                 u.data_ptr(), eu.data_ptr(), 0, 0)
        ctx.de_step(prob, 0, de(0), 0.5, 0.9, stream=st)

        def timed_calls(call, t0):
            for k in range(warm):
                call(t0 + k)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for k in range(steps):
                call(t0 + warm + k)
            e1.record(st)
            torch.cuda.synchronize()
            ctx.sync(st)
            return e0.elapsed_time(e1) / steps

        ms_de = timed_calls(lambda t: ctx.de_step(prob, 0, de(t), 0.5, 0.9, stream=st), 1)
        del u, eu
        # DE at the population sizes the method uses (10240 populations of
        # 200, the same 2 million individuals): a run's population fits in
        # LDS and the variation gathers its donors there
        R2, NP2 = 10240, 200
        n2 = R2 * NP2
        x2 = torch.empty(R2 * D * NP2, device="cuda"); u2 = torch.empty_like(x2)
        ex2 = torch.empty(n2, device="cuda"); eu2 = torch.empty_like(ex2)
        de2 = lambda t: S.DEState(R2, NP2, NP2, D * NP2, 11, t, x2.data_ptr(), ex2.data_ptr(),  # noqa: E731
                                  u2.data_ptr(), eu2.data_ptr(), 0, 0)
        ctx.de_step(prob, 0, de2(0), 0.5, 0.9, stream=st)
        ms_de2 = timed_calls(lambda t: ctx.de_step(prob, 0, de2(t), 0.5, 0.9, stream=st), 1)
        del x2, u2, ex2, eu2
        # C4's largest populations: 4096 runs of 200 at D = 100 (80 KB each,
        # staged through LDS in slabs of rows), 328 MB per population buffer
        R3, NP3, D3 = 4096, 200, 100
        n3 = R3 * NP3
        prob3 = S.problem(S.RASTRIGIN, D3)
        x3 = torch.empty(R3 * D3 * NP3, device="cuda"); u3 = torch.empty_like(x3)
        ex3 = torch.empty(n3, device="cuda"); eu3 = torch.empty_like(ex3)
        de3 = lambda t: S.DEState(R3, NP3, NP3, D3 * NP3, 13, t, x3.data_ptr(), ex3.data_ptr(),  # noqa: E731
                                  u3.data_ptr(), eu3.data_ptr(), 0, 0)
        ctx.de_step(prob3, 0, de3(0), 0.5, 0.9, stream=st)
        ms_de3 = timed_calls(lambda t: ctx.de_step(prob3, 0, de3(t), 0.5, 0.9, stream=st), 1)
        del x3, u3, ex3, eu3
        v = torch.empty_like(x); p = torch.empty_like(x)
        ep = torch.empty(n, device="cuda"); gb = torch.zeros(R, dtype=torch.int32, device="cuda")
        ps = lambda t: S.PSOState(R, NP, NP, D * NP, 9, t, x.data_ptr(), v.data_ptr(),  # noqa: E731
                                  p.data_ptr(), ex.data_ptr(), ep.data_ptr(), gb.data_ptr())
        vmax = 0.2 * (W.UB - W.LB)
        ctx.pso_step(prob, 0, ps(0), 0.7298, 1.49618, 1.49618, vmax, stream=st)
        ms_pso = timed_calls(lambda t: ctx.pso_step(prob, 0, ps(t), 0.7298, 1.49618, 1.49618, vmax,
                                                    stream=st), 1)
        # minimum HBM bytes per individual and generation: DE reads x, writes
        # u, the evaluation reads u and writes e(u), the selection reads both
        # errors (12 D + 12; the copy of winning trials is not counted); PSO
        # reads x, v, p and writes x, v, the evaluation reads x and writes
        # e(x), the bests read both errors (24 D + 12)
        b_de, b_pso = n * (12 * D + 12), n * (24 * D + 12)
        gbs_de = b_de / (ms_de / 1e3) / 1e9
        gbs_pso = b_pso / (ms_pso / 1e3) / 1e9
        del x, v, p, ex, ep
        # the memory-bound side of the evaluation: D = 10 (2 D^2 = 200 FLOP
        # per 44 B), 64 items of 262,144 points, 738 MB read per call
        DE_, NE = 10, 1 << 18
        xs = [torch.empty((DE_, NE), device="cuda").uniform_(W.LB, W.UB) for _ in range(64)]
        es = [torch.empty(NE, device="cuda") for _ in range(64)]
        batch = S.Context.prepare_batch([(S.problem(S.RASTRIGIN, DE_), k % 10, xs[k], es[k]) for k in range(64)])
        ctx.tune_evaluate(batch, stream=st)
        ms_ev = timed_calls(lambda t: ctx.evaluate_batch(batch, stream=st), 0)
        b_ev = 64 * NE * (4 * DE_ + 4)
        gbs_ev = b_ev / (ms_ev / 1e3) / 1e9
        _line(metric, n / (ms_de / 1e3), "evals/s", steps, warm, ms_de,
              {"workload": "unfused DE rand/1/bin generation steps (sevo_de_step): 1024 populations x 2048 "
                           "at D=30, Rastrigin, one instance, one call per generation; PSO iterations "
                           "(sevo_pso_step) beside", "individuals": n},
              roofline={"bound": "hbm", "achieved": round(gbs_de, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": round(gbs_de / PEAK_HBM_GBS, 4), "traffic": None,
                        "kernel": "the DE step's three launches (variation, evaluation, selection)",
                        "algorithmic_bytes": b_de},
              de_np200={"evals_per_s": round(n2 / (ms_de2 / 1e3), 1), "ms": round(ms_de2, 4),
                        "achieved_gbs": round(n2 * (12 * D + 12) / (ms_de2 / 1e3) / 1e9, 1),
                        "note": "10240 populations x 200 at D=30 (donors gathered from LDS)"},
              de_np200_d100={"evals_per_s": round(n3 / (ms_de3 / 1e3), 1), "ms": round(ms_de3, 4),
                             "achieved_gbs": round(n3 * (12 * D3 + 12) / (ms_de3 / 1e3) / 1e9, 1),
                             "note": "4096 populations x 200 at D=100, C4's largest (staged in slabs of rows)"},
              pso={"evals_per_s": round(n / (ms_pso / 1e3), 1), "ms": round(ms_pso, 4),
                   "achieved_gbs": round(gbs_pso, 1), "frac": round(gbs_pso / PEAK_HBM_GBS, 4),
                   "algorithmic_bytes": b_pso},
              evaluation_d10={"evals_per_s": round(64 * NE / (ms_ev / 1e3), 1), "ms": round(ms_ev, 4),
                              "achieved_gbs": round(gbs_ev, 1), "frac": round(gbs_ev / PEAK_HBM_GBS, 4),
                              "algorithmic_bytes": b_ev,
                              "note": "64 items x 262144 points, Rastrigin D=10, batched evaluation"})
    elif a.workload == "c1":
        spec = [(S.ALGO_DE, S.RASTRIGIN, 10, 50, 50 * 1001, 0, 0)]
        descs = _run_descs(S, spec)
        ms64, r64 = _time_runs(ctx, S, torch, descs, S.FP64, steps, warm, trace_len=250)
        ms32, r32 = _time_runs(ctx, S, torch, descs, S.FP32, steps, warm, trace_len=250, graph=True)
        ev = r64[0].fes
        extra = {"fused_fp32": {"evals_per_s": ev / (ms32 / 1e3), "ms": ms32,
                                "best_e": r32[0].best_e, "launch": "HIP graph replay of a plan"},
                 "plain_fp64": {"evals_per_s": ev / (ms64 / 1e3), "ms": ms64, "best_e": r64[0].best_e},
                 "speedup_fused_vs_plain": ms64 / ms32}
        if not a.no_cpu:
            extra["cpu_baseline"] = _oracle_runs(spec, 10)
        _line(metric, ev / (ms64 / 1e3), "evals/s", steps, warm, ms64,
              {"workload": "plain DE rand/1/bin, one run: Rastrigin D=10, NP=50, F=0.5, CR=0.9, "
                           "1000 generations, FP64 one-launch-per-step path"}, dtype="f64", **extra)
    elif a.workload == "c3":
        spec = []
        for sw in range(4096):
            f, d, k = W.c3_swarm(sw)
            spec.append((S.ALGO_PSO, f, d, 40, 40 * 2001, k, sw))
        descs = _run_descs(S, spec)
        ms, rr = _time_runs(ctx, S, torch, descs, S.FP32, steps, warm, graph=True)
        ev = sum(r.fes for r in rr)
        # one swarm per launch: a sample of 24 swarms (8 per dimension), each its own call
        sample = [descs[i] for i in range(0, 4096, 4096 // 24)][:24]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        res = torch.zeros((1, 32), dtype=torch.uint8, device="cuda")
        st = torch.cuda.current_stream()
        ctx.run(sample[:1], res, stream=st)
        torch.cuda.synchronize()
        e0.record(st)
        for d in sample:
            ctx.run([d], res, stream=st)
        e1.record(st)
        torch.cuda.synchronize()
        per_swarm_ms = e0.elapsed_time(e1) / len(sample)
        extra = {"one_swarm_per_launch": {"ms_per_swarm": per_swarm_ms,
                                          "projected_ms_4096": per_swarm_ms * 4096,
                                          "evals_per_s": (40 * 2001) / (per_swarm_ms / 1e3)},
                 "speedup_batched_vs_per_launch": per_swarm_ms * 4096 / ms}
        if not a.no_cpu:
            extra["cpu_baseline"] = _oracle_runs(spec[::64], 10)
        _line(metric, ev / (ms / 1e3), "evals/s", steps, warm, ms,
              {"workload": "batched PSO: 4096 swarms x 40 particles, D in {10,30,50} x 6 functions x "
                           "10 instances, 2000 iterations, persistent fused kernels (one launch per "
                           "dimension class) replayed from a HIP graph",
               "evals": ev}, **extra)
    elif a.workload in ("jade", "lshade_rs"):
        algo = S.ALGO_JADE if a.workload == "jade" else S.ALGO_LSHADE_RS
        spec = []
        for r in range(2048):
            f, d, k, np_ = W.c4_run(r)
            spec.append((algo, f, d, np_, 10000 * d, k, r))
        descs = _run_descs(S, spec)
        n = len(descs)
        res = torch.zeros((n, 32), dtype=torch.uint8, device="cuda")
        st = torch.cuda.current_stream()
        extra = {}
        if algo == S.ALGO_JADE:
            # with the parameter observer: (muF, muCR) after every generation
            mu_len = max(d.budget // d.np for d in descs) + 2
            mu = torch.empty(n * mu_len * 2, device="cuda")
            call = lambda: ctx.run_observed(descs, res, mu, mu_len, stream=st)  # noqa: E731
        else:
            call = lambda: ctx.run(descs, res, stream=st)  # noqa: E731
        call()   # warm-up (kernel set-up, instances)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        call()
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        raw = res.cpu().numpy().tobytes()
        rr = [S.RunResult.from_buffer_copy(raw[32 * k: 32 * (k + 1)]) for k in range(n)]
        ev = sum(r.fes for r in rr)
        extra["successes"] = sum(r.success for r in rr)
        if algo == S.ALGO_JADE:
            # the case study's curve: mean over runs of (muF, muCR) per generation
            m = mu.view(n, mu_len, 2).cpu().numpy()
            mean = np.nanmean(m, axis=0)
            extra["mean_mu_by_generation"] = {str(g): [round(float(mean[g, 0]), 4), round(float(mean[g, 1]), 4)]
                                              for g in (0, 1, 10, 100, 500) if g < mu_len}
        else:
            extra["restarts"] = sum(r.restarts for r in rr)
        if not a.no_cpu:
            extra["cpu_baseline"] = _oracle_runs([spec[(k * 129) % 2048] for k in range(16)], 10)
        _line(metric, ev / (ms / 1e3), "evals/s", 1, 1, ms,
              {"workload": ("batched JADE with the muF/muCR observer: 2048 runs, D in {10,30,50,100}, "
                            "NP = min(18 D, 200), budget 10000 D, p = 0.05, c = 0.1, archive NP"
                            if algo == S.ALGO_JADE else
                            "batched L-SHADE-Restart: 2048 runs, D in {10,30,50,100}, NP from min(18 D, 200) "
                            "down to 4 per restart, budget 10000 D, p = 0.11, H = 6, archive 2.6 NP, "
                            f"restart once the population's error spread <= {RESTART_TOL:g}") +
                           ", persistent fused kernels, one call", "evals": ev}, **extra)
    elif a.workload in ("c4", "lshade"):
        algo = S.ALGO_SHADE if a.workload == "c4" else S.ALGO_LSHADE
        spec = []
        for r in range(2048):
            f, d, k, np_ = W.c4_run(r)
            spec.append((algo, f, d, np_, 10000 * d, k, r))
        descs = _run_descs(S, spec)
        ms, rr = _time_runs(ctx, S, torch, descs, S.FP32, 1, 0, graph=True)
        ev = sum(r.fes for r in rr)
        succ = sum(r.success for r in rr)
        extra = {"successes": succ}
        if not a.no_cpu:
            # 16 runs, 4 per dimension (run r has D = (10, 30, 50, 100)[r mod 4]; a
            # stride of 129 runs steps through the four)
            extra["cpu_baseline"] = _oracle_runs([spec[(k * 129) % 2048] for k in range(16)], 10)
        _line(metric, ev / (ms / 1e3), "evals/s", 1, 0, ms,
              {"workload": ("batched SHADE: 2048 runs, D in {10,30,50,100}, NP = min(18 D, 200), "
                            "budget 10000 D, p = 0.1, H = 6" if a.workload == "c4" else
                            "batched L-SHADE: 2048 runs, D in {10,30,50,100}, NP from min(18 D, 200) "
                            "down to 4, budget 10000 D, p = 0.11, H = 6, archive 2.6 NP") +
                           ", persistent fused kernels replayed from a HIP graph", "evals": ev}, **extra)
    elif a.workload == "psode":
        spec = []
        for r in range(4096):
            f, d, k, np_ = W.psode_run(r)
            spec.append((S.ALGO_PSODE, f, d, np_, 1000 * d, k, r))
        descs = _run_descs(S, spec)
        ms, rr = _time_runs(ctx, S, torch, descs, S.FP32, steps, warm, graph=True)
        ev = sum(r.fes for r in rr)
        be = sorted(r.best_e for r in rr)
        extra = {"median_best_e": be[len(be) // 2]}
        if not a.no_cpu:
            extra["cpu_baseline"] = _oracle_runs(spec[:16], 10)
        _line(metric, ev / (ms / 1e3), "evals/s", steps, warm, ms,
              {"workload": "batched PSODE (pairwise/3 selection, the case study's hybrid): 4096 runs, "
                           "Rosenbrock D=30 x 10 instances, NP=100, budget 1000 D; PSO half spherical "
                           "update with ring topology, DE half SHADE p = 0.1, H = 6; persistent fused "
                           "kernels replayed from a HIP graph", "evals": ev}, **extra)
    elif a.workload == "cso":
        spec = [W.cso_run(r) for r in range(W.CSO_RUNS)]
        descs = [S.RunDesc(S.problem(f, d), k, r, S.ALGO_CSO, m, budget, 0.5, 0.9, 0.7298, W.CSO_PHI, 1.49618,
                           0.2 * (W.UB - W.LB), 0.1, 6, 2.6, 4, 0, 0)
                 for r, (f, d, k, m, budget) in enumerate(spec)]
        out = {}
        for prec, name in ((S.SPLIT_BF16, "split_bf16"), (S.FP32, "fp32")):
            res = torch.zeros((len(descs), 32), dtype=torch.uint8, device="cuda")
            st = torch.cuda.current_stream()
            plan = ctx.plan_run(descs, res, precision=prec)
            plan.launch(st)                      # warm-up: one whole job
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            plan.launch(st)
            e1.record(st)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            plan.close()
            raw = res.cpu().numpy().tobytes()
            rr = [S.RunResult.from_buffer_copy(raw[32 * k: 32 * (k + 1)]) for k in range(len(descs))]
            ev = sum(r.fes for r in rr)
            out[name] = {"ms": ms, "evals_per_s": ev / (ms / 1e3),
                         "median_best_e": sorted(r.best_e for r in rr)[len(rr) // 2]}
        bf = out["split_bf16"]
        extra = {"precisions": out}
        if not a.no_cpu:
            # whole FP64 runs at D = 1000 take hours: the sample is 16 of the
            # workload's runs truncated to the initial swarm and 4 iterations
            short = [(S.ALGO_CSO, f, d, m, m + 4 * (m // 2), k, r) for r, (f, d, k, m, _) in enumerate(spec[:16])]
            extra["cpu_baseline"] = _oracle_runs(short, 10)
        _line(metric, bf["evals_per_s"], "evals/s", 1, 1, bf["ms"],
              {"workload": "large scale: CSO, 30 runs (6 functions x 5 runs) at D=1000, swarm 300, "
                           "1e6 evaluations each, phi = 0.1; per iteration one update launch and the "
                           "batched split-bf16 evaluation of all runs' losers", "evals": ev},
              dtype="bf16x6", **extra)
    elif a.workload == "c5":
        out = {}
        for prec, name in ((S.SPLIT_BF16, "split_bf16"), (S.FP32, "fp32")):
            items = []
            for f in (S.ELLIPSOID, S.RASTRIGIN):
                x = torch.empty((1000, 6400), device="cuda").uniform_(W.LB, W.UB)
                e = torch.empty(6400, device="cuda")
                items.append((S.problem(f, 1000), 0, x, e))
            batch = S.Context.prepare_batch(items)
            st = torch.cuda.current_stream()
            for _ in range(3):
                ctx.evaluate_batch(batch, precision=prec, stream=st)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 20
            e0.record(st)
            for _ in range(reps):
                ctx.evaluate_batch(batch, precision=prec, stream=st)
            e1.record(st)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            ev = 2 * 6400
            fl = 2.0 * 1000 * 1000 * ev
            out[name] = {"ms": ms, "evals_per_s": ev / (ms / 1e3),
                         "tflops_fp32_equiv": fl / (ms / 1e3) / 1e12}
        bf = out["split_bf16"]
        roof = {"bound": "mfma", "achieved": round(6 * 2.0e6 * 12800 / (bf["ms"] / 1e3) / 1e12, 2),
                "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s", "traffic": None,
                "note": "6 bf16 products per rotation flop (three-term split of both operands); whole call "
                        "(operand pre-pass, GEMM, combine)"}
        roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
        _line(metric, bf["evals_per_s"], "evals/s", reps, 3, bf["ms"],
              {"workload": "large scale: D=1000 Ellipsoid and Rastrigin, 64 runs x 100 points each, "
                           "split-bf16 rotation on MFMA"}, dtype="bf16x6", precisions=out, roofline=roof)
    ctx.close()


if __name__ == "__main__":
    main()
