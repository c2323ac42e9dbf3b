"""GPU tests of the batched form: many independent problems of different
N, K, M and P in one pipeline (one launch per stage), captured in a HIP graph.

* every problem's 12 classes against the FP64 oracle (FP64 mode: 1e-10
  relative Frobenius; bf16x3: the stated bound);
* graph replays against eager runs of the same pipeline, bit for bit, with
  the inputs changed between replays and eager work in between;
* the autotuners (one problem, a whole batch) return valid choices that
  later plans use, with results that stay within the mode's bound.
"""
from __future__ import annotations

import numpy as np
import pytest

import paper_2401_13185_amd as cv
from oracle import cv_oracle as O
from synth import generators as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FP64_TOL = 1e-10
BF16X3_BOUND = 2e-5


def _dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    return torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(_dev())


def _relerr(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / nb) if nb else float(np.linalg.norm(a))


SHAPES = [
    # n, k, m, p, values
    (700, 64, 1, 3, "spectra"),
    (1500, 100, 5, 7, "gaussian"),
    (2200, 128, 16, 20, "spectra"),
    (999, 200, 0, 4, "gaussian"),
    (3000, 256, 40, 5, "offset"),
    (1200, 33, 3, 11, "gaussian"),
    (4100, 64, 16, 3, "spectra"),
    (1800, 130, 9, 6, "offset"),
]


def _problems(dtype):
    out = []
    for i, (n, k, m, p, values) in enumerate(SHAPES):
        shape = G.Shape(f"batch case {i}", n, k, m, p, dtype, values, "dirichlet")
        out.append(G.make(shape, 400 + i, 0))
    return out


@pytest.mark.parametrize("mode,dtype", [("fp64", "f64"), ("fp64", "f32"), ("bf16x3", "f32"),
                                        ("fp32", "f32")])
def test_batch_matches_oracle(mode, dtype):
    probs = _problems(dtype)
    print(f"[batch] mode={mode} dtype={dtype} problems={len(probs)}", flush=True)
    dev_probs = [(_t(X), _t(Y) if Y.shape[1] else None, _t(f)) for X, Y, f in probs]
    b = cv.cvgram_batch_create(dev_probs, ddof=1, mode=mode)
    cv.cvgram_batch_run(b)
    torch.cuda.synchronize()
    tol = {"fp64": FP64_TOL, "bf16x3": BF16X3_BOUND, "fp32": 1e-6}[mode]
    for i, (X, Y, f) in enumerate(probs):
        P, scalable = cv.cvgram_batch_problem_info(b, i)
        assert P == int(f.max()) + 1 and scalable
        xx = b.outs[i][0].cpu().numpy()
        xy = b.outs[i][1].cpu().numpy() if b.outs[i][1] is not None else None
        for q in range(P):
            oxx, oxy = O.fold_all_classes(X, Y, f, q, ddof=1)
            for c in range(4):
                e = _relerr(xx[q, c], oxx[c])
                assert e <= tol, (mode, i, q, "XtX", c, e)
                assert np.array_equal(xx[q, c], xx[q, c].T)
            for c in range(8 if Y.shape[1] else 0):
                e = _relerr(xy[q, c], oxy[c])
                assert e <= tol, (mode, i, q, "XtY", c, e)
    cv.cvgram_batch_destroy(b)


@pytest.mark.parametrize("mode", ["fp64", "bf16x3"])
def test_batch_with_smallest_problems(mode):
    # problems of 4 to 65 rows (two-row training partitions, no Y) in one
    # batch with a larger one: their items, slabs and corrections share the
    # launches
    shapes = [(4, 1, 1, 2), (5, 3, 2, 2), (1500, 100, 5, 7), (9, 2, 0, 3), (65, 17, 3, 13)]
    probs = [G.make(G.Shape(f"small batch case {i}", n, k, m, p, "f64", "gaussian",
                            "near_equal"), 470 + i, 0)
             for i, (n, k, m, p) in enumerate(shapes)]
    print(f"[batch] smallest problems mode={mode}", flush=True)
    dev_probs = [(_t(X), _t(Y) if Y.shape[1] else None, _t(f)) for X, Y, f in probs]
    b = cv.cvgram_batch_create(dev_probs, ddof=1, mode=mode)
    cv.cvgram_batch_run(b)
    torch.cuda.synchronize()
    # BF16X3: sums of a few rows do not average the split's rounding out, so
    # every entry is held to the split arithmetic's own bound
    # (tests/sampling.py: split_bf16_bound) and the relative Frobenius bar
    # to the problem with long sums
    from tests import sampling as S
    for i, (X, Y, f) in enumerate(probs):
        P, scalable = cv.cvgram_batch_problem_info(b, i)
        assert P == int(f.max()) + 1 and scalable
        xx = b.outs[i][0].cpu().numpy()
        xy = b.outs[i][1].cpu().numpy() if b.outs[i][1] is not None else None
        for q in range(P):
            oxx, oxy = O.fold_all_classes(X, Y, f, q, ddof=1)
            tol = FP64_TOL if mode == "fp64" else (BF16X3_BOUND if X.shape[0] >= 1000 else None)
            bxx, bxy = S.split_bf16_bound(X, Y, f, q, ddof=1) if mode == "bf16x3" else (None, None)
            for c in range(4):
                e = _relerr(xx[q, c], oxx[c])
                assert tol is None or e <= tol, (mode, i, q, "XtX", c, e)
                if bxx is not None:
                    assert np.all(np.abs(xx[q, c] - oxx[c]) <= bxx[c]), (mode, i, q, "XtX", c)
                assert np.array_equal(xx[q, c], xx[q, c].T)
            for c in range(8 if Y.shape[1] else 0):
                e = _relerr(xy[q, c], oxy[c])
                assert tol is None or e <= tol, (mode, i, q, "XtY", c, e)
                if bxy is not None:
                    assert np.all(np.abs(xy[q, c] - oxy[c]) <= bxy[c]), (mode, i, q, "XtY", c)
    cv.cvgram_batch_destroy(b)


@pytest.mark.parametrize("mode", ["fp64", "bf16x3"])
def test_graph_replays_match_eager_runs(mode):
    probs = _problems("f32" if mode == "bf16x3" else "f64")
    dev_probs = [(_t(X), _t(Y) if Y.shape[1] else None, _t(f)) for X, Y, f in probs]
    b = cv.cvgram_batch_create(dev_probs, ddof=1, mode=mode)
    rng = np.random.default_rng(0)
    for rep in range(3):
        # change the inputs in place (eager torch work between replays)
        for X, Y, _ in dev_probs:
            X.mul_(1.0 + 0.01 * rep).add_(float(rng.uniform(-1, 1)))
            if Y is not None:
                Y.add_(0.5 * rep)
        cv.cvgram_batch_run(b)
        torch.cuda.synchronize()
        graph_out = [(xx.clone(), None if xy is None else xy.clone()) for xx, xy in b.outs]
        for xx, xy in b.outs:           # scribble, then recompute eagerly
            xx.fill_(float("nan"))
            if xy is not None:
                xy.fill_(float("nan"))
        cv.cvgram_batch_run_eager(b)
        torch.cuda.synchronize()
        for (gx, gy), (ex, ey) in zip(graph_out, b.outs):
            assert torch.equal(gx, ex)
            if gy is not None:
                assert torch.equal(gy, ey)
    # the last replay also matches the oracle on the changed inputs
    X, Y, f = (t.cpu().numpy() if t is not None else None for t in dev_probs[2])
    oxx, oxy = O.fold_all_classes(X, Y, f, 1, ddof=1)
    tol = FP64_TOL if mode == "fp64" else BF16X3_BOUND
    for c in range(4):
        assert _relerr(b.outs[2][0][1, c].cpu().numpy(), oxx[c]) <= tol
    cv.cvgram_batch_destroy(b)


def test_batch_equals_single_handles_fp64():
    probs = _problems("f64")
    dev_probs = [(_t(X), _t(Y) if Y.shape[1] else None, _t(f)) for X, Y, f in probs]
    b = cv.cvgram_batch_create(dev_probs, ddof=0, mode="fp64")
    cv.cvgram_batch_run(b)
    for i, (X, Y, f) in enumerate(dev_probs):
        h = cv.cvgram_create(X, Y, f, ddof=0, mode="fp64")
        xx, xy = cv.cvgram_folds_all(h, 0, cv.cvgram_num_folds(h))
        torch.cuda.synchronize()
        d = (torch.linalg.norm(xx - b.outs[i][0]) / torch.linalg.norm(xx)).item()
        assert d <= 1e-13, (i, d)
        cv.cvgram_destroy(h)
    cv.cvgram_batch_destroy(b)


def test_batch_many_problems_sampled():
    """A 64-problem batch of the batched workload's shape family (smaller N):
    every 8th problem against the oracle."""
    shapes = G.batch_shapes(64, n_lo=500, n_hi=6000)
    probs = [G.batch_problem(s, i) for i, s in enumerate(shapes)]
    dev_probs = [(_t(X), _t(Y), _t(f)) for X, Y, f in probs]
    b = cv.cvgram_batch_create(dev_probs, ddof=1, mode="bf16x3")
    cv.cvgram_batch_run(b)
    torch.cuda.synchronize()
    for i in range(0, 64, 8):
        X, Y, f = probs[i]
        P, _ = cv.cvgram_batch_problem_info(b, i)
        for q in (0, P - 1):
            oxx, oxy = O.fold_all_classes(X, Y, f, q, ddof=1)
            for c in range(4):
                assert _relerr(b.outs[i][0][q, c].cpu().numpy(), oxx[c]) <= BF16X3_BOUND, (i, q, c)
            for c in range(8):
                assert _relerr(b.outs[i][1][q, c].cpu().numpy(), oxy[c]) <= BF16X3_BOUND, (i, q, c)
    cv.cvgram_batch_destroy(b)


def test_batch_error_reports_problem_index():
    ok = G.make(G.Shape("ok", 300, 10, 2, 3, "f64", "gaussian", "dirichlet"), 1, 0)
    bad_fold = ok[2].copy()
    bad_fold[bad_fold == 1] = 0          # fold 1 empty -> Definition 1 violated
    probs = [(_t(ok[0]), _t(ok[1]), _t(ok[2])), (_t(ok[0]), _t(ok[1]), _t(bad_fold))]
    with pytest.raises(cv.CVGramError) as ei:
        cv.cvgram_batch_create(probs, mode="fp64")
    assert ei.value.status == 2 and "problem 1" in str(ei.value)


def test_autotune_returns_valid_choice_and_results_stay_correct():
    shape = G.Shape("tune", 20000, 192, 8, 6, "f32", "spectra", "dirichlet")
    X, Y, f = G.make(shape, 77, 0)
    Xd, Yd, fd = _t(X), _t(Y), _t(f)
    tile, items = cv.cvgram_autotune(Xd, Yd, fd, mode="bf16x3")
    print(f"[autotune] tile={tile} items={items}", flush=True)
    assert tile in (64, 128, 256) and items in (512, 1024, 2048, 4096, 8192, 16384)
    h = cv.cvgram_create(Xd, Yd, fd, 1, 1, 1, 1, mode="bf16x3")   # uses the tuned bucket
    xx, xy = cv.cvgram_folds_all(h, 0, 6)
    oxx, oxy = O.fold_all_classes(X, Y, f, 2, ddof=1)
    for c in range(4):
        assert _relerr(xx[2, c].cpu().numpy(), oxx[c]) <= BF16X3_BOUND
    cv.cvgram_destroy(h)


@pytest.mark.parametrize("mode", ["fp64", "bf16x3"])
def test_batch_autotune_choice_used_and_correct(mode):
    probs = _problems("f32")
    dev_probs = [(_t(X), _t(Y) if Y.shape[1] else None, _t(f)) for X, Y, f in probs]
    tile, wide_k, items, ms = cv.cvgram_batch_autotune(dev_probs, mode=mode)
    print(f"[batch autotune] mode={mode} tile={tile} wide_min_k={wide_k} items={items} "
          f"gram_ms={ms:.4f}", flush=True)
    assert tile in (64, 128, 256) and wide_k in (0, 512) and ms > 0
    assert items in (512, 1024, 2048, 4096, 8192, 16384)
    assert wide_k == 0 or tile == 256
    if mode == "fp64":
        assert tile <= 128          # FP64 tiles stop at 128
    b = cv.cvgram_batch_create(dev_probs, ddof=1, mode=mode)
    cv.cvgram_batch_run(b)
    torch.cuda.synchronize()
    bound = FP64_TOL if mode == "fp64" else BF16X3_BOUND
    for i, (X, Y, f) in enumerate(probs):
        P, _ = cv.cvgram_batch_problem_info(b, i)
        xx = b.outs[i][0].cpu().numpy()
        for q in (0, P - 1):
            oxx, _ = O.fold_all_classes(X, Y, f, q, ddof=1)
            for c in range(4):
                assert _relerr(xx[q, c], oxx[c]) <= bound, (mode, i, q, c)
    cv.cvgram_batch_destroy(b)


def test_batch_full_size_sampled():
    """The batched workload at full size, as the bench runs it: 256 problems
    (N log-uniform in [1e3, 2e5], K in {64, 128, 256, 512}, M 1..16, P 3..20,
    values drawn on the device, graph replay).  FP64 mode against the
    oracle on sampled entries of every 16th problem (each entry from the two
    columns it needs, copied to the host); bf16x3 against FP64 on every
    problem, fold and class within the stated bound."""
    shapes = G.batch_shapes(256)
    probs = [G.batch_problem_device(s, i, _dev()) for i, s in enumerate(shapes)]
    torch.cuda.synchronize()
    print("[batch] full-size workload generated", flush=True)
    outs = {}
    for mode in ("fp64", "bf16x3"):
        b = cv.cvgram_batch_create(probs, ddof=1, mode=mode)
        cv.cvgram_batch_run(b)
        torch.cuda.synchronize()
        outs[mode] = b
    worst = 0.0
    for (xa, ya), (xb, yb) in zip(outs["bf16x3"].outs, outs["fp64"].outs):
        for a, r in ((xa, xb), (ya, yb)):
            num = torch.linalg.matrix_norm(a.double() - r)
            worst = max(worst, (num / torch.linalg.matrix_norm(r)).max().item())
    assert worst <= BF16X3_BOUND, worst
    rng = np.random.default_rng(256)
    for i in range(0, 256, 16):
        X, Y, fd = probs[i]
        K, M = X.shape[1], Y.shape[1]
        fold = fd.cpu().numpy()
        P, _ = cv.cvgram_batch_problem_info(outs["fp64"], i)
        pairs_xx = [(int(a), int(c)) for a, c in rng.integers(0, K, size=(6, 2))] + [(K - 1, K - 1)]
        pairs_xy = [(int(a), int(c)) for a, c in zip(rng.integers(0, K, 4), rng.integers(0, M, 4))]
        xcols = sorted({c for pr in pairs_xx for c in pr} | {a for a, _ in pairs_xy})
        ycols = sorted({c for _, c in pairs_xy})
        xm = {c: n for n, c in enumerate(xcols)}
        ym = {c: n for n, c in enumerate(ycols)}
        Xs = X[:, xcols].double().cpu().numpy()
        Ys = Y[:, ycols].double().cpu().numpy()
        sxx = [(xm[a], xm[c]) for a, c in pairs_xx]
        sxy = [(xm[a], ym[c]) for a, c in pairs_xy]
        gx, gy = outs["fp64"].outs[i]
        for q in (0, P - 1):
            for c in range(4):
                ref, _ = O.fold_entries(Xs, Ys, fold, q, *O.XTX_CLASS_COMBO[c], 1, sxx, [])
                got = np.array([gx[q, c, a, d].item() for a, d in pairs_xx])
                scale = gx[q, c].abs().max().item()
                assert np.max(np.abs(got - ref)) <= FP64_TOL * scale, (i, q, c)
            for c in range(8):
                _, ref = O.fold_entries(Xs, Ys, fold, q, *O.XTY_CLASS_COMBO[c], 1, [], sxy)
                got = np.array([gy[q, c, a, d].item() for a, d in pairs_xy])
                scale = gy[q, c].abs().max().item()
                assert np.max(np.abs(got - ref)) <= FP64_TOL * scale, (i, q, c)
    for b in outs.values():
        cv.cvgram_batch_destroy(b)


_TUNE_CHILD = r"""
import sys, numpy as np, torch
sys.path.insert(0, sys.argv[1])
import paper_2401_13185_amd as cv
from synth import generators as G
shape = G.Shape("tune file", 6000, 160, 4, 5, "f32", "spectra", "dirichlet")
X, Y, f = G.make(shape, 91, 0)
dev = torch.device("cuda:0")
Xd, Yd, fd = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (X, Y, f))
if sys.argv[2] == "tune":
    tile, items = cv.cvgram_autotune(Xd, Yd, fd, mode="bf16x3")
    print("CHOICE", tile, items, flush=True)
else:
    h = cv.cvgram_create(Xd, Yd, fd, 1, 1, 1, 1, mode="bf16x3")
    print("PLAN", cv.cvgram_plan_info(h)["tile"], flush=True)
    cv.cvgram_destroy(h)
"""


def test_tune_file_round_trip(tmp_path):
    """An autotuned choice written to CVGRAM_TUNE_FILE (keyed by the device)
    is the plan a later process takes for the same problem."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, CVGRAM_TUNE_FILE=str(tmp_path / "tune.txt"))
    script = tmp_path / "child.py"
    script.write_text(_TUNE_CHILD)
    out = subprocess.run([sys.executable, str(script), root, "tune"], env=env, capture_output=True,
                         text=True, timeout=240)
    assert out.returncode == 0, out.stderr[-2000:]
    tile = int(out.stdout.split("CHOICE")[1].split()[0])
    lines = (tmp_path / "tune.txt").read_text().splitlines()
    print("[tune file]", lines, flush=True)
    assert lines and all(len(ln.split()) == 9 for ln in lines)
    assert all(ln.split()[0].startswith("gfx") for ln in lines)
    out = subprocess.run([sys.executable, str(script), root, "plan"], env=env, capture_output=True,
                         text=True, timeout=240)
    assert out.returncode == 0, out.stderr[-2000:]
    assert int(out.stdout.split("PLAN")[1].split()[0]) == tile
