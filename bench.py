#!/usr/bin/env python3
"""Throughput of the per-fold training Gram path on one MI355X.

One step = the whole hot path over one batch of synthetic input:
cvgram_create (fold bookkeeping, statistics, grouped Gram) + every fold's 12
distinct training products (4 X^T X + 8 X^T Y classes) + cvgram_destroy.
Inputs are resident in HBM before timing starts.

Prints ONE JSON line.  ``value`` is sets/s, a set being one fold's
(X^T X, X^T Y) pair for one combination: P * 12 sets per step.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}  # TFLOP/s dense MFMA, MI355X
HBM_PEAK = 8000.0  # GB/s
# stated relative Frobenius error bounds of the mixed modes (per fold, class
# and output, against FP64)
MIXED_BOUND = {"fp32": 1e-6, "bf16x3": 2e-5}


def f_alg(n, k, m):
    """Algorithmic flops of one Gram pass over all rows: the upper triangle
    of X^T X (N K (K+1)) and all of X^T Y (2 N K M)."""
    return n * k * (k + 1) + 2 * n * k * m


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="fp64", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--workload", type=int, default=2, choices=[2, 3],
                    help="headline workload: 2 = spectra N=1e5 K=512 (default), "
                         "3 = precision-stress N=1e6 K=1024 (for profiling one mode)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline legs")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-vs-FP64 block on the precision-stress workload")
    ap.add_argument("--mixed-steps", type=int, default=5)
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched block (256 independent problems, graph replay)")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB: the "
                         "reference dispatch that scales HBM byte counters in a profile")
    return ap.parse_args()


def cpu_legs(X, Y, fold, P, gpu_xx, gpu_xy, budget_s):
    """CPU baselines on the host cores: the oracle on a bounded sample (one
    fold, all 12 classes) and the paper's fast algorithm on all folds."""
    from oracle import cv_oracle as O
    from oracle import fast_cpu
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        threads = os.cpu_count()
    t0 = time.perf_counter()
    oxx, oxy = O.fold_all_classes(X, Y, fold, 0, ddof=1)
    t_or = time.perf_counter() - t0
    errs = []
    for c in range(4):
        errs.append(np.linalg.norm(gpu_xx[0, c] - oxx[c]) / np.linalg.norm(oxx[c]))
    for c in range(8):
        errs.append(np.linalg.norm(gpu_xy[0, c] - oxy[c]) / np.linalg.norm(oxy[c]))
    cpu = {"value": 12.0 / t_or, "unit": "sets/s", "cores": int(threads), "kind": "oracle",
           "sample": f"fold 0 of {P}, all 12 distinct classes, FP64 naive baseline",
           "seconds": round(t_or, 3)}
    fast = None
    if t_or < budget_s:
        t0 = time.perf_counter()
        for _ in fast_cpu.fast_all_folds(X, Y, fold, ddof=1):
            pass
        t_fast = time.perf_counter() - t0
        fast = {"value": P * 12.0 / t_fast, "unit": "sets/s", "cores": int(threads),
                "kind": "paper fast algorithm (Algorithm 7, all classes), FP64 NumPy",
                "sample": f"all {P} folds", "seconds": round(t_fast, 3)}
    return cpu, fast, float(max(errs))


def measure(cv, torch, Xd, Yd, fd, P, K, M, mode, steps, warmup):
    """Time `steps` whole steps (after `warmup`): create + all folds x 12
    classes + destroy.  Stage times come from HIP events on the same stream."""
    odt = torch.float64 if mode == "fp64" else torch.float32
    dev = Xd.device
    xx = torch.empty(P, 4, K, K, dtype=odt, device=dev)
    xy = torch.empty(P, 8, K, M, dtype=odt, device=dev)
    stream = torch.cuda.current_stream()

    def step(timing=False):
        h = cv.cvgram_create(Xd, Yd, fd, 1, 1, 1, 1, ddof=1, mode=mode, stream=stream)
        if timing:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        cv.cvgram_folds_all(h, 0, P, xx, xy)
        st = None
        if timing:
            e1.record(stream)
            st = cv.cvgram_stage_times(h)
        cv.cvgram_destroy(h)
        if timing:
            st["correct"] = e0.elapsed_time(e1)
        return st

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    cv.cvgram_set_stage_timing(True)
    stages = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        stages.append(step(timing=True))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    cv.cvgram_set_stage_timing(False)
    ms = (t1 - t0) * 1e3 / steps
    stage_ms = {k: float(np.mean([s[k] for s in stages])) for k in stages[0]}
    return ms, stage_ms, xx, xy


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1 "
                          "(the multi-GPU sharding is described in DESIGN.md, not built)"}))
        sys.exit(2)
    import torch
    import paper_2401_13185_amd as cv
    from synth import generators as G

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.copy_ref_mib:
        src = torch.empty(args.copy_ref_mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    shape, (X, Y, fold) = G.workload(args.workload)
    N, K, M, P = shape.n, shape.k, shape.m, shape.p
    print(f"[bench] workload {shape.name} generated", file=sys.stderr, flush=True)
    Xd = torch.from_numpy(X).to(dev)
    Yd = torch.from_numpy(Y).to(dev)
    fd = torch.from_numpy(fold).to(dev)
    ms, stage_ms, xx, xy = measure(cv, torch, Xd, Yd, fd, P, K, M, args.mode, args.steps,
                                   args.warmup)
    print("[bench] headline timed steps done", file=sys.stderr, flush=True)

    sets = P * 12
    flops = f_alg(N, K, M)
    gram_tflops = flops / (stage_ms["gram"] * 1e-3) / 1e12
    kname = {"fp64": "gram_f64_kernel", "fp32": "gram_f32_kernel", "bf16x3": "gram_bf16x3_kernel"}
    out = {
        "metric": "per-fold train Gram sets/s (12 distinct centering/scaling classes per fold)",
        "value": sets / (ms * 1e-3),
        "unit": "sets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3+f32acc"}[args.mode],
        "data": "synthetic",
        "config": {"workload": shape.name, "N": N, "K": K, "M": M, "P": P, "folds": {"dirichlet": "Dirichlet(2)", "near_equal": "near-equal"}[shape.folds],
                   "mode": args.mode, "classes_per_fold": 12, "ddof": 1},
        "tflops_alg": flops / (ms * 1e-3) / 1e12,
        "stage_ms": stage_ms,
        "roofline": {"bound": "mfma", "kernel": kname[args.mode], "achieved": gram_tflops,
                     "peak": PEAK[args.mode], "unit": "TFLOP/s",
                     "frac": gram_tflops / PEAK[args.mode], "traffic": None},
    }
    if not args.no_cpu:
        torch.cuda.synchronize()
        gxx = xx.double().cpu().numpy()
        gxy = xy.double().cpu().numpy()
        cpu, fast, err = cpu_legs(X, Y, fold, P, gxx, gxy, args.cpu_seconds)
        out["cpu_baseline"] = cpu
        if fast:
            out["cpu_fast"] = fast
        out["max_rel_err_vs_oracle_fold0"] = err
    del xx, xy
    if not args.no_mixed:
        out["mixed"] = mixed_block(cv, torch, G, dev, args)
    if not args.no_batch:
        out["batched"] = batched_block(cv, torch, G, dev, args)
    print(json.dumps(out))


def mixed_block(cv, torch, G, dev, args):
    """Mixed precision vs plain FP64 on the precision-stress workload (FP32
    input, column means in [1e3, 1e4]): sets/s and Gram TFLOP/s per mode, and
    each mixed mode's worst relative Frobenius error over all folds and
    classes against the FP64 GPU form (itself within 1e-10 of the oracle)."""
    shape, (X, Y, fold) = G.workload(3)
    N, K, M, P = shape.n, shape.k, shape.m, shape.p
    print(f"[bench] workload {shape.name} generated", file=sys.stderr, flush=True)
    Xd = torch.from_numpy(X).to(dev)
    Yd = torch.from_numpy(Y).to(dev)
    fd = torch.from_numpy(fold).to(dev)
    del X, Y
    flops = f_alg(N, K, M)
    res = {"workload": shape.name, "classes_per_fold": 12, "modes": {}}
    ref = None
    for mode in ("fp64", "fp32", "bf16x3"):
        ms, st, xx, xy = measure(cv, torch, Xd, Yd, fd, P, K, M, mode, args.mixed_steps, 1)
        g = flops / (st["gram"] * 1e-3) / 1e12
        r = {"sets_per_s": P * 12 / (ms * 1e-3), "ms_per_step": ms, "stage_ms": st,
             "gram_tflops_alg": g, "gram_frac_of_peak": g / PEAK[mode], "peak_tflops": PEAK[mode]}
        if mode == "fp64":
            ref = (xx, xy)
        else:
            worst = 0.0
            for q in range(P):
                for c in range(4):
                    a, b = xx[q, c].double(), ref[0][q, c]
                    worst = max(worst, (torch.linalg.norm(a - b) / torch.linalg.norm(b)).item())
                for c in range(8):
                    a, b = xy[q, c].double(), ref[1][q, c]
                    worst = max(worst, (torch.linalg.norm(a - b) / torch.linalg.norm(b)).item())
            r["max_rel_err_vs_fp64"] = worst
            r["stated_bound"] = MIXED_BOUND[mode]
            r["within_bound"] = worst <= MIXED_BOUND[mode]
            del xx, xy
        res["modes"][mode] = r
        print(f"[bench] mixed-block mode {mode} done", file=sys.stderr, flush=True)
    f64 = res["modes"]["fp64"]["ms_per_step"]
    for mode in ("fp32", "bf16x3"):
        res["modes"][mode]["speedup_vs_fp64"] = f64 / res["modes"][mode]["ms_per_step"]
    return res


def batched_block(cv, torch, G, dev, args):
    """256 independent problems of different N, K, M, P (spectra, FP32,
    Dirichlet(2) folds) in one batch: the whole pipeline (12 classes per
    fold) captured in a HIP graph, replayed `batch_steps` times, FP64 and
    bf16x3 on the same inputs; bf16x3's worst relative Frobenius error
    against FP64 over every problem, fold and class."""
    shapes = G.batch_shapes(256)
    probs = [G.batch_problem_device(s, i, dev) for i, s in enumerate(shapes)]
    torch.cuda.synchronize()
    print("[bench] batched workload generated", file=sys.stderr, flush=True)
    n_sets = sum(s.p for s in shapes) * 12
    flops = sum(f_alg(s.n, s.k, s.m) for s in shapes)
    res = {"workload": "256 problems: N log-uniform [1e3, 2e5], K in {64,128,256,512}, "
                       "M in 1..16, P in 3..20, spectra fp32, Dirichlet(2) folds",
           "sets_per_step": n_sets, "total_rows": sum(s.n for s in shapes),
           "f_alg_total": flops, "modes": {}}
    outs = {}
    for mode in ("fp64", "bf16x3"):
        t0 = time.perf_counter()
        b = cv.cvgram_batch_create(probs, ddof=1, mode=mode)
        torch.cuda.synchronize()
        t_plan = time.perf_counter() - t0
        cv.cvgram_batch_run(b)          # warm
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.batch_steps):
            cv.cvgram_batch_run(b)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.batch_steps
        res["modes"][mode] = {"ms_per_step": ms, "sets_per_s": n_sets / (ms * 1e-3),
                              "tflops_alg": flops / (ms * 1e-3) / 1e12,
                              "plan_seconds": round(t_plan, 3)}
        outs[mode] = b
        print(f"[bench] batched mode {mode} done", file=sys.stderr, flush=True)
    worst = 0.0
    for (xa, ya), (xb, yb) in zip(outs["bf16x3"].outs, outs["fp64"].outs):
        num = torch.linalg.matrix_norm(xa.double() - xb)
        den = torch.linalg.matrix_norm(xb)
        worst = max(worst, (num / den).max().item())
        num = torch.linalg.matrix_norm(ya.double() - yb)
        den = torch.linalg.matrix_norm(yb)
        worst = max(worst, (num / den).max().item())
    r = res["modes"]["bf16x3"]
    r["max_rel_err_vs_fp64"] = worst
    r["stated_bound"] = MIXED_BOUND["bf16x3"]
    r["within_bound"] = worst <= MIXED_BOUND["bf16x3"]
    r["speedup_vs_fp64"] = res["modes"]["fp64"]["ms_per_step"] / r["ms_per_step"]
    for b in outs.values():
        cv.cvgram_batch_destroy(b)
    return res


if __name__ == "__main__":
    main()
