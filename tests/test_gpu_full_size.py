"""Full-size parity on sampled entries, in the launch configuration the
bench times, against the FP64 oracle.

Entries are sampled by columns: 16 columns of X (the first and the last
among them) and 4 of Y; every X^T X entry among the 16 (diagonals included,
136 distinct) and every X^T Y entry of the 16 x 4 block (64), in all 12
classes, of several folds.  The oracle computes them from those columns of
the training rows (tests/sampling.py).  Bars, per entry, relative to the
entry's Cauchy-Schwarz scale sqrt(U^T U_ii V^T V_jj):
    FP64 mode  1e-10 (and 1e-10 relative Frobenius on the sampled block)
    FP32 mode  MIXED_BOUND["fp32"],  BF16X3 mode  MIXED_BOUND["bf16x3"]
Workloads: the precision-stress problem (offset data, N=1e6, K=1024, M=16,
P=100, FP32 input) in all three modes, folds 0, 37, the smallest and the
largest (and the mixed modes' whole products of every fold against the
FP64 GPU form, relative Frobenius error per class); the spectra shape (N=1e5, K=512, M=8, FP64) with P = 1e4 and
P = 1e5 (leave-one-out, fused fold path, two host waits), folds 0, 4095,
4096, 4097, P/2 and P-1.
"""
from __future__ import annotations

import numpy as np
import pytest

import paper_2401_13185_amd as cv
from synth import generators as G
from tests import sampling as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FP64_TOL = 1e-10
MIXED_BOUND = {"fp32": 1e-6, "bf16x3": 2e-5}


def _dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    return torch.device("cuda:0")


def _sampled_gpu(h, p, xcols, ycols):
    """Fold p's 12 classes restricted to the sampled columns (host FP64)."""
    xx, xy = cv.cvgram_folds_all(h, p, p + 1)
    xi = torch.tensor(xcols, device=xx.device)
    yi = torch.tensor(ycols, device=xx.device)
    gxx = xx[0][:, xi][:, :, xi].double().cpu().numpy()
    gxy = xy[0][:, xi][:, :, yi].double().cpu().numpy()
    del xx, xy
    return gxx, gxy


def _assert_fold(res, tol, label, frob=None):
    for kind in ("xtx", "xty"):
        for c, (ew, fe) in enumerate(res[kind]):
            assert ew <= tol, (label, kind, c, "entry-wise", ew)
            if frob is not None:
                assert fe <= frob, (label, kind, c, "frobenius", fe)


def test_precision_stress_full_size_all_modes_against_oracle():
    dev = _dev()
    shape, (X, Y, fold) = G.workload(3)
    N, K, M, P = shape.n, shape.k, shape.m, shape.p
    print(f"[full] {shape.name}", flush=True)
    rng = np.random.default_rng(1024)
    xcols = S.pick_columns(K, 16, rng)
    ycols = S.pick_columns(M, 4, rng)
    Xs = X[:, xcols].astype(np.float64)
    Ys = Y[:, ycols].astype(np.float64)
    sizes = np.bincount(fold, minlength=P)
    folds = sorted({0, 37, int(np.argmin(sizes)), int(np.argmax(sizes))})
    Xd, Yd, fd = (torch.from_numpy(a).to(dev) for a in (X, Y, fold))
    del X, Y
    refs = {p: S.oracle_block(Xs, Ys, fold, p) for p in folds}
    print(f"[full] oracle blocks of folds {folds} done", flush=True)
    h64 = None
    for mode in ("fp64", "fp32", "bf16x3"):
        h = cv.cvgram_create(Xd, Yd, fd, 1, 1, 1, 1, ddof=1, mode=mode)
        tol = FP64_TOL if mode == "fp64" else MIXED_BOUND[mode]
        w = 0.0
        for p in folds:
            gxx, gxy = _sampled_gpu(h, p, xcols, ycols)
            res = S.compare_block(gxx, gxy, refs[p])
            _assert_fold(res, tol, (mode, p), frob=FP64_TOL if mode == "fp64" else None)
            w = max(w, max(e for kind in res.values() for e, _ in kind))
        print(f"[full] {mode} folds {folds}: worst entry-wise error vs oracle {w:.3e}", flush=True)
        if mode == "fp64":
            h64 = h
            continue
        # every fold's whole products against the FP64 GPU form (itself
        # checked against the oracle above), relative Frobenius per class
        wf = 0.0
        for q0 in range(0, P, 25):
            q1 = min(P, q0 + 25)
            a64, b64 = cv.cvgram_folds_all(h64, q0, q1)
            am, bm = cv.cvgram_folds_all(h, q0, q1)
            ex = (torch.linalg.matrix_norm(am.double() - a64) / torch.linalg.matrix_norm(a64))
            ey = (torch.linalg.matrix_norm(bm.double() - b64) / torch.linalg.matrix_norm(b64))
            wf = max(wf, ex.max().item(), ey.max().item())
            del a64, b64, am, bm
        print(f"[full] {mode} every fold vs FP64 GPU form: worst {wf:.3e}", flush=True)
        assert wf <= MIXED_BOUND[mode], (mode, wf)
        cv.cvgram_destroy(h)
    cv.cvgram_destroy(h64)
    torch.cuda.synchronize()
    del Xd, Yd, fd
    torch.cuda.empty_cache()


def _spectra_case(P, path_expected):
    dev = _dev()
    base = G.WORKLOADS[2]
    N, K, M = base.n, base.k, base.m
    X, Y, _ = G.make(base, 2)
    fold = G.folds_near_equal(N, P, G._rng(2, 0, 11, P))
    print(f"[full] spectra N={N} K={K} M={M} P={P}", flush=True)
    rng = np.random.default_rng(P)
    xcols = S.pick_columns(K, 16, rng)
    ycols = S.pick_columns(M, 4, rng)
    Xs, Ys = X[:, xcols], Y[:, ycols]
    h = cv.cvgram_create(torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev),
                         torch.from_numpy(fold).to(dev), 1, 1, 1, 1, ddof=1, mode="fp64")
    assert cv.cvgram_num_folds(h) == P
    assert cv.cvgram_plan_info(h)["fused"] == (path_expected == "fused")
    folds = sorted({0, 4095, 4096, 4097, P // 2, P - 1})
    w = 0.0
    for p in folds:
        gxx, gxy = _sampled_gpu(h, p, xcols, ycols)
        res = S.compare_fold(gxx, gxy, Xs, Ys, fold, p)
        _assert_fold(res, FP64_TOL, ("P", P, p), frob=FP64_TOL)
        w = max(w, max(e for kind in res.values() for e, _ in kind))
    cv.cvgram_destroy(h)
    torch.cuda.synchronize()
    print(f"[full] P={P} folds {folds}: worst entry-wise error {w:.3e}", flush=True)


def test_spectra_ten_thousand_folds_sampled():
    _spectra_case(10_000, "fused")


def test_spectra_leave_one_out_sampled():
    _spectra_case(100_000, "fused")
