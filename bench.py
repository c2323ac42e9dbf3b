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


def f_exec(n, k, m, mode, tile=None):
    """Flops the Gram launch executes (matrix-core work, not algorithmic):
    whole tiles above the diagonal; on a diagonal tile, FP64 / FP32 with
    128-wide tiles compute the 36 upper-triangle 16 x 16 blocks of 64 and
    one (M <= 16) or two (M <= 32) 16-column K x M blocks per block row,
    otherwise (BF16X3, 64-wide tiles) three waves of four take the upper
    quadrants and the fourth a 32-column K x M block; M > 32 uses separate
    K x M tiles.  Three bf16 products per product in BF16X3."""
    T = tile or (64 if k <= 64 else 128)
    nt = -(-k // T)
    pairs = T == 128 and mode != "bf16x3"
    entries = (nt * (nt + 1) // 2 - nt) * T * T
    if pairs:
        entries += nt * 36 * 256
        if 0 < m <= 32:
            entries += nt * 8 * (1 if m <= 16 else 2) * 256
    else:
        entries += nt * (3 * T * T // 4)
        if 0 < m <= 32:
            entries += nt * T * 32
    if m > 32:
        entries += nt * (-(-m // T)) * T * T
    return 2 * n * entries * (3 if mode == "bf16x3" else 1)


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
    ap.add_argument("--c5", action="store_true",
                    help="add the large single-problem block (N=2e6, K=4096, M=64, P=64, fp32 "
                         "input): bf16x3 vs the FP64 form, folds streamed in chunks")
    ap.add_argument("--psweep", action="store_true",
                    help="add the fold-count sweep on the spectra shape (N=1e5, K=512, M=8; "
                         "P = 3 .. 100000, near-equal folds, FP64): Gram time flat in P")
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
    # the oracle on folds 0, 1, ... until about half the budget is spent
    # (at least one fold); the GPU result is checked on every fold it covers
    t0 = time.perf_counter()
    errs = []
    n_or = 0
    while n_or < P:
        oxx, oxy = O.fold_all_classes(X, Y, fold, n_or, ddof=1)
        for c in range(4):
            errs.append(np.linalg.norm(gpu_xx[n_or, c] - oxx[c]) / np.linalg.norm(oxx[c]))
        for c in range(8):
            errs.append(np.linalg.norm(gpu_xy[n_or, c] - oxy[c]) / np.linalg.norm(oxy[c]))
        n_or += 1
        if time.perf_counter() - t0 >= 0.5 * budget_s:
            break
    t_or = time.perf_counter() - t0
    errs = [float(e) for e in errs]
    cpu = {"value": 12.0 * n_or / t_or, "unit": "sets/s", "cores": int(threads), "kind": "oracle",
           "sample": f"folds 0..{n_or - 1} of {P}, all 12 distinct classes each, FP64 naive "
                     f"baseline",
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
    return cpu, fast, errs


def measure(cv, torch, Xd, Yd, fd, P, K, M, mode, steps, warmup):
    """Time `steps` whole steps (after `warmup`): create + all folds x 12
    classes + destroy, back to back with no host synchronisation between
    them.  Stage times come from a separate pass of steps with the library's
    HIP events on (those steps wait for their events)."""
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
            e1.synchronize()
            st["correct"] = e0.elapsed_time(e1)
        return st

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / steps
    # stage breakdown (and the Gram launch time behind the roofline)
    cv.cvgram_set_stage_timing(True)
    stages = [step(timing=True) for _ in range(max(3, min(steps, 20)))]
    torch.cuda.synchronize()
    cv.cvgram_set_stage_timing(False)
    stage_ms = {k: float(np.mean([s[k] for s in stages])) for k in stages[0]}
    return ms, stage_ms, xx, xy


def measure_single(cv, torch, Xd, Yd, fd, P, K, M, mode, steps, warmup):
    """The paper's own target, one combination (center and scale X and Y):
    create + cvgram_fold for every fold + destroy.  Returns ms per step."""
    odt = torch.float64 if mode == "fp64" else torch.float32
    xx = torch.empty(K, K, dtype=odt, device=Xd.device)
    xy = torch.empty(K, M, dtype=odt, device=Xd.device)
    stream = torch.cuda.current_stream()

    def step():
        h = cv.cvgram_create(Xd, Yd, fd, 1, 1, 1, 1, ddof=1, mode=mode, stream=stream)
        for p in range(P):
            cv.cvgram_fold(h, p, xx, xy)
        cv.cvgram_destroy(h)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def padded_rows(fold, P):
    """Rows of the packed panels: every fold padded to a multiple of 32."""
    counts = np.bincount(np.asarray(fold), minlength=P)
    return int(((counts + 31) // 32 * 32).sum())


def stage_bandwidth(N, K, M, P, Np, in_bytes, mode, stage_ms):
    """Algorithmic HBM bytes and GB/s of the statistics pass (A2: read X and Y
    once, write the packed operand panels) and of the per-fold corrections
    (A5: read G_p, write 4 K x K + 8 K x M outputs per fold)."""
    e = {"fp64": 8, "fp32": 4, "bf16x3": 4}[mode]
    W = K + M
    tile = 64 if K <= 64 else 128
    Kp = -(-K // tile) * tile
    Wp = Kp + (32 if 0 < M <= 32 else -(-M // tile) * tile)
    a2 = N * W * in_bytes + Np * Wp * e
    ob = 8 if mode == "fp64" else 4
    a5 = P * ((4 * K * K + 8 * K * M) * ob + (K * (K + 1) // 2 + K * M) * 8) + K * W * 8
    return {"A2_stats_pack": {"bytes": a2, "GB_per_s": a2 / (stage_ms["stats"] * 1e-3) / 1e9},
            "A5_corrections": {"bytes": a5, "GB_per_s": a5 / (stage_ms["correct"] * 1e-3) / 1e9}}


def source_digest():
    """SHA-256 over the sources that decide what the Gram launch reads and
    writes (kernels and work planning)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("gram.hip", "api.hip", "internal.h"):
        with open(os.path.join(ROOT, "paper_2401_13185_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    counter summary (FETCH_SIZE and WRITE_SIZE, each scaled by the same
    counter's reading for a plain copy), or None when the summary is absent,
    covers another kernel or workload, or was taken on other sources."""
    path = os.path.join(ROOT, "profiles", "gram_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_digest() or kv.get("kernel") != kernel \
            or kv.get("workload") != workload:
        return None
    return float(kv["fetch_bytes_scaled"]) + float(kv["write_bytes_scaled"])


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1 "
                          "(multi-GPU sharding is a design, not built)"}))
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
    tile = 64 if K <= 64 else 128
    kname = {"fp64": f"gram_kernel<0, {tile}>", "fp32": f"gram_kernel<1, {tile}>",
             "bf16x3": f"gram_bf16_kernel<{tile}>"}
    single_ms = measure_single(cv, torch, Xd, Yd, fd, P, K, M, args.mode, max(3, args.steps // 2),
                               1)
    print("[bench] single-combination steps done", file=sys.stderr, flush=True)
    traffic = profiled_traffic(kname[args.mode], shape.name)
    Np = padded_rows(fold, P)
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
                     "frac": gram_tflops / PEAK[args.mode], "traffic": traffic},
        "gram_executed_tflops": f_exec(N, K, M, args.mode) / (stage_ms["gram"] * 1e-3) / 1e12,
        "single_combination": {"combo": "center+scale X and Y (1111)", "sets_per_step": P,
                               "ms_per_step": single_ms, "sets_per_s": P / (single_ms * 1e-3)},
        "hbm": stage_bandwidth(N, K, M, P, Np, X.itemsize, args.mode, stage_ms),
    }
    if not args.no_cpu:
        torch.cuda.synchronize()
        gxx = xx.double().cpu().numpy()
        gxy = xy.double().cpu().numpy()
        cpu, fast, errs = cpu_legs(X, Y, fold, P, gxx, gxy, args.cpu_seconds)
        out["cpu_baseline"] = cpu
        if fast:
            out["cpu_fast"] = fast
        out["max_rel_err_vs_oracle"] = max(errs)  # over the folds the oracle sample covers
        out["median_rel_err_vs_oracle"] = float(np.median(errs))
    del xx, xy
    out["ridge"] = ridge_block(cv, torch, Xd, Yd, fd, P, K, M, args.mode)
    print("[bench] ridge block done", file=sys.stderr, flush=True)
    if not args.no_mixed:
        out["mixed"] = mixed_block(cv, torch, G, dev, args)
    if not args.no_batch:
        out["batched"] = batched_block(cv, torch, G, dev, args)
    if args.c5:
        out["large"] = c5_block(cv, torch, G, dev, args)
    if args.psweep:
        out["p_sweep"] = psweep_block(cv, torch, G, dev, args)
    print(json.dumps(out))


def ridge_block(cv, torch, Xd, Yd, fd, P, K, M, mode, n_lambda=8, reps=3):
    """The per-fold ridge consumer on the headline workload: every fold and
    n_lambda penalties (1e-3 .. 1e4), centred and scaled; one call = the
    products of all folds in FP64, a batched Cholesky of P x n_lambda K x K
    systems and their solves.  Flops per system: K^3/3 + 2 K^2 M."""
    lams = list(np.logspace(-3, 4, n_lambda))
    h = cv.cvgram_create(Xd, Yd, fd, 1, 1, 1, 1, ddof=1, mode=mode)
    out = torch.empty(P, n_lambda, K, M, dtype=torch.float64, device=Xd.device)
    cv.cvgram_ridge(h, 0, P, lams, out)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        cv.cvgram_ridge(h, 0, P, lams, out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    cv.cvgram_destroy(h)
    systems = P * n_lambda
    flops = systems * (K ** 3 / 3 + 2 * K * K * M)
    return {"systems": systems, "K": K, "M": M, "ms_per_call": ms,
            "systems_per_s": systems / (ms * 1e-3), "tflops": flops / (ms * 1e-3) / 1e12}


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
        ge = f_exec(N, K, M, mode) / (st["gram"] * 1e-3) / 1e12
        r = {"sets_per_s": P * 12 / (ms * 1e-3), "ms_per_step": ms, "stage_ms": st,
             "gram_tflops_alg": g, "gram_frac_of_peak": g / PEAK[mode], "peak_tflops": PEAK[mode],
             "gram_executed_tflops": ge, "gram_executed_frac_of_peak": ge / PEAK[mode]}
        if mode == "fp64":
            ref = (xx, xy)
        else:
            errs = []
            for q in range(P):
                for c in range(4):
                    a, b = xx[q, c].double(), ref[0][q, c]
                    errs.append((torch.linalg.norm(a - b) / torch.linalg.norm(b)).item())
                for c in range(8):
                    a, b = xy[q, c].double(), ref[1][q, c]
                    errs.append((torch.linalg.norm(a - b) / torch.linalg.norm(b)).item())
            worst = max(errs)
            r["max_rel_err_vs_fp64"] = worst
            r["median_rel_err_vs_fp64"] = float(np.median(errs))
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


def psweep_block(cv, torch, G, dev, args):
    """Fold-count sweep on the spectra shape (N=1e5, K=512, M=8, FP64 input,
    near-equal folds, FP64 mode): create + every fold's 12 classes, written
    in chunks of at most 64 folds.  The Gram (A3) time should not depend on
    P; the corrections grow with the output size (P x 12 products)."""
    base = G.WORKLOADS[2]
    N, K, M = base.n, base.k, base.m
    X, Y, _ = G.make(base, 2)
    Xd, Yd = torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev)
    CH = 64
    xx = torch.empty(CH, 4, K, K, dtype=torch.float64, device=dev)
    xy = torch.empty(CH, 8, K, M, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    rows = []
    for P in (3, 10, 100, 1000, 3000, 10000, 100000):
        fold = G.folds_near_equal(N, P, G._rng(2, 0, 11, P))
        fd = torch.from_numpy(fold).to(dev)
        for it in range(2):  # the first pass warms the workspace cache
            cv.cvgram_set_stage_timing(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = cv.cvgram_create(Xd, Yd, fd, 1, 1, 1, 1, ddof=1, mode="fp64", stream=stream)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for p0 in range(0, P, CH):
                p1 = min(P, p0 + CH)
                cv.cvgram_folds_all(h, p0, p1, xx[:p1 - p0], xy[:p1 - p0])
            e1.record(stream)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            st = cv.cvgram_stage_times(h)
            cv.cvgram_set_stage_timing(False)
            fused = cv.cvgram_plan_info(h)["fused"]
            cv.cvgram_destroy(h)
        out_bytes = P * (4 * K * K + 8 * K * M) * 8
        rows.append({"P": P, "path": "fused" if fused else "grouped",
                     "seconds": dt, "sets_per_s": P * 12 / dt, "gram_ms": st["gram"],
                     "stage_ms": st, "corrections_ms": e0.elapsed_time(e1),
                     "output_GB_per_s": out_bytes / (e0.elapsed_time(e1) * 1e-3) / 1e9})
        print(f"[bench] p-sweep P={P} done", file=sys.stderr, flush=True)
    del xx, xy, Xd, Yd
    torch.cuda.empty_cache()
    cv.cvgram_trim_cache()
    return {"workload": base.name.replace("P=10", "P swept") + ", near-equal folds",
            "fold_chunk": CH, "rows": rows}


def c5_block(cv, torch, G, dev, args):
    """One large problem (spectra N=2e6, K=4096, M=64, P=64, fp32 input,
    Dirichlet(2) folds): bf16x3 against the FP64 form on the same inputs.
    Folds are written in chunks of 8 (every fold's 12 classes), so only the
    chunk's outputs are resident; sets/s per mode, and bf16x3's worst and
    median relative Frobenius error against FP64 over every fold and class."""
    shape = G.WORKLOADS[5]
    N, K, M, P = shape.n, shape.k, shape.m, shape.p
    X, Y = G.spectra_xy_torch(N, K, M, seed=5_13185, device=dev)
    fold = G.folds_dirichlet(N, P, G._rng(5, 0, 9))
    fd = torch.from_numpy(fold).to(dev)
    torch.cuda.synchronize()
    print("[bench] large workload generated", file=sys.stderr, flush=True)
    CH = 8
    res = {"workload": shape.name + " (torch generator)", "classes_per_fold": 12,
           "fold_chunk": CH, "modes": {}}
    stream = torch.cuda.current_stream()
    handles = {}
    for mode in ("bf16x3", "fp64"):
        odt = torch.float64 if mode == "fp64" else torch.float32
        xx = torch.empty(CH, 4, K, K, dtype=odt, device=dev)
        xy = torch.empty(CH, 8, K, M, dtype=odt, device=dev)
        cv.cvgram_set_stage_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = cv.cvgram_create(X, Y, fd, 1, 1, 1, 1, ddof=1, mode=mode, stream=stream)
        for p0 in range(0, P, CH):
            p1 = min(P, p0 + CH)
            cv.cvgram_folds_all(h, p0, p1, xx[:p1 - p0], xy[:p1 - p0])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = cv.cvgram_stage_times(h)
        cv.cvgram_set_stage_timing(False)
        g = f_alg(N, K, M) / (st["gram"] * 1e-3) / 1e12
        res["modes"][mode] = {"seconds": dt, "sets_per_s": P * 12 / dt, "stage_ms": st,
                              "gram_tflops_alg": g, "gram_frac_of_peak": g / PEAK[mode]}
        handles[mode] = h
        del xx, xy
        print(f"[bench] large-block mode {mode} done", file=sys.stderr, flush=True)
    errs = []
    bx = torch.empty(CH, 4, K, K, dtype=torch.float32, device=dev)
    by = torch.empty(CH, 8, K, M, dtype=torch.float32, device=dev)
    fx = torch.empty(CH, 4, K, K, dtype=torch.float64, device=dev)
    fy = torch.empty(CH, 8, K, M, dtype=torch.float64, device=dev)
    for p0 in range(0, P, CH):
        p1 = min(P, p0 + CH)
        cv.cvgram_folds_all(handles["bf16x3"], p0, p1, bx[:p1 - p0], by[:p1 - p0])
        cv.cvgram_folds_all(handles["fp64"], p0, p1, fx[:p1 - p0], fy[:p1 - p0])
        for a, b in ((bx[:p1 - p0], fx[:p1 - p0]), (by[:p1 - p0], fy[:p1 - p0])):
            num = torch.linalg.matrix_norm(a.double() - b)
            errs.extend((num / torch.linalg.matrix_norm(b)).flatten().tolist())
    for h in handles.values():
        cv.cvgram_destroy(h)
    r = res["modes"]["bf16x3"]
    r["max_rel_err_vs_fp64"] = max(errs)
    r["median_rel_err_vs_fp64"] = float(np.median(errs))
    r["stated_bound"] = MIXED_BOUND["bf16x3"]
    r["within_bound"] = max(errs) <= MIXED_BOUND["bf16x3"]
    r["speedup_vs_fp64"] = res["modes"]["fp64"]["seconds"] / r["seconds"]
    del X, Y, fd, bx, by, fx, fy
    torch.cuda.empty_cache()
    cv.cvgram_trim_cache()
    return res


if __name__ == "__main__":
    main()
