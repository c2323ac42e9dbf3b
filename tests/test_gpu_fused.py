"""GPU parity of the fused fold path (many small folds: rows packed without
per-fold padding, only the full Gram contracted, each fold's validation Gram
formed inside the per-fold corrections) against the FP64 oracle, and its
agreement with the grouped path on the same inputs.

Bars as for the grouped path: FP64 within 1e-10 relative Frobenius error
per fold x class x output (1e-12 between the two GPU paths); mixed modes
within their stated bounds against the FP64 form; X^T X bit-symmetric.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

import paper_2401_13185_amd as cv
from oracle import cv_oracle as O
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


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(_dev())


def _relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a)) if nb == 0.0 else float(np.linalg.norm(a - b) / nb)


class ForcedFoldPath:
    """Force the library's fold path for the handles created inside."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        self.old = os.environ.get("CVGRAM_FOLD_PATH")
        if self.path is None:
            os.environ.pop("CVGRAM_FOLD_PATH", None)
        else:
            os.environ["CVGRAM_FOLD_PATH"] = self.path

    def __exit__(self, *a):
        if self.old is None:
            os.environ.pop("CVGRAM_FOLD_PATH", None)
        else:
            os.environ["CVGRAM_FOLD_PATH"] = self.old


def _run(X, Y, fold, mode="fp64", ddof=1, path=None):
    with ForcedFoldPath(path):
        h = cv.cvgram_create(_t(X), _t(Y) if Y.shape[1] else None, _t(fold.astype(np.int32)),
                             1, 1, 1, 1, ddof=ddof, mode=mode)
    P = cv.cvgram_num_folds(h)
    xx, xy = cv.cvgram_folds_all(h, 0, P)
    torch.cuda.synchronize()
    out = (xx.double().cpu().numpy(),
           xy.double().cpu().numpy() if xy is not None else np.zeros((P, 8, X.shape[1], 0)))
    cv.cvgram_destroy(h)
    return out


def _against_oracle(X, Y, fold, xx, xy, ddof, folds, tol=FP64_TOL, label=""):
    for p in folds:
        oxx, oxy = O.fold_all_classes(X, Y, fold, p, ddof=ddof)
        for c in range(4):
            e = _relerr(xx[p, c], oxx[c])
            assert e <= tol, (label, "XtX", p, c, e)
            assert np.array_equal(xx[p, c], xx[p, c].T), (label, "asymmetric", p, c)
        for c in range(8 if Y.shape[1] else 0):
            e = _relerr(xy[p, c], oxy[c])
            assert e <= tol, (label, "XtY", p, c, e)


def _gaussian(n, k, m, seed):
    rng = np.random.default_rng(seed)
    mu = rng.normal(5.0, 2.0, k)
    X = mu + rng.lognormal(0.0, 0.5, k) * rng.standard_normal((n, k))
    Y = X @ rng.standard_normal((k, m)) + 0.1 * rng.standard_normal((n, m))
    return X, Y


@pytest.mark.parametrize("ddof", [0, 1])
def test_leave_one_out_all_folds(ddof):
    """P = N (one row per fold): the fused path is the default."""
    n, k, m = 150, 24, 3
    print(f"[fused] LOO N={n} K={k} M={m} ddof={ddof}", flush=True)
    X, Y = _gaussian(n, k, m, 11)
    fold = np.random.default_rng(5).permutation(n).astype(np.int32)
    xx, xy = _run(X, Y, fold, ddof=ddof)
    _against_oracle(X, Y, fold, xx, xy, ddof, range(n), label="loo")


@pytest.mark.parametrize("n,k,m,P,seed", [(2500, 40, 5, 100, 1), (1900, 70, 0, 130, 2),
                                          (1200, 33, 40, 64, 3)])
def test_forced_paths_agree_and_match_oracle(n, k, m, P, seed):
    print(f"[fused] forced paths N={n} K={k} M={m} P={P}", flush=True)
    X, Y = _gaussian(n, k, m, seed)
    fold = G.folds_dirichlet(n, P, np.random.default_rng(seed))
    fx, fy = _run(X, Y, fold, path="fused")
    gx, gy = _run(X, Y, fold, path="grouped")
    for p in range(P):
        for c in range(4):
            assert _relerr(fx[p, c], gx[p, c]) <= 1e-12, (p, c)
        for c in range(8 if m else 0):
            assert _relerr(fy[p, c], gy[p, c]) <= 1e-12, (p, c)
    sizes = np.bincount(fold, minlength=P)
    folds = sorted({0, P - 1, int(np.argmin(sizes)), int(np.argmax(sizes))})
    _against_oracle(X, Y, fold, fx, fy, 1, folds, label="fused")


def test_fused_constant_columns():
    """A column constant over all rows, and one constant over every row but
    those of one fold (so constant over T_p for that fold only)."""
    n, k, m, P = 800, 12, 2, 80
    print(f"[fused] constant columns N={n} K={k} P={P}", flush=True)
    X, Y = _gaussian(n, k, m, 7)
    fold = G.folds_near_equal(n, P, np.random.default_rng(7))
    X[:, 3] = 2.5
    X[:, 7] = -1.25
    X[fold == 9, 7] = 4.0
    xx, xy = _run(X, Y, fold, path="fused")
    _against_oracle(X, Y, fold, xx, xy, 1, [0, 9, 10, P - 1], label="const")
    # centred products of the constant column are exactly zero
    assert np.all(xx[0, 2][3] == 0.0) and np.all(xx[9, 2][7] == 0.0)


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
def test_fused_mixed_modes_within_bound(mode):
    n, k, m, P = 3000, 48, 6, 120
    print(f"[fused] mixed {mode} N={n} K={k} P={P}", flush=True)
    shape = G.Shape("offset", n, k, m, P, "f32", "offset", "near_equal")
    X, Y, fold = G.make(shape, 3, problem=7)
    mx, my = _run(X, Y, fold, mode=mode, path="fused")
    fx, fy = _run(X, Y, fold, mode="fp64", path="fused")
    worst = 0.0
    for p in range(P):
        for c in range(4):
            worst = max(worst, _relerr(mx[p, c], fx[p, c]))
        for c in range(8):
            worst = max(worst, _relerr(my[p, c], fy[p, c]))
    print(f"[fused] {mode} worst {worst:.3e}", flush=True)
    assert worst <= MIXED_BOUND[mode]
    _against_oracle(X, Y, fold, fx, fy, 1, [0, P - 1], label="fp64-f32")


def test_batch_mixing_fold_paths_equals_single_handles():
    """One batch holding a leave-one-out problem (fused) and a 5-fold one
    (grouped): the same results as separate handles."""
    X1, Y1 = _gaussian(120, 20, 2, 21)
    f1 = np.random.default_rng(21).permutation(120).astype(np.int32)
    X2, Y2 = _gaussian(1500, 36, 4, 22)
    f2 = G.folds_near_equal(1500, 5, np.random.default_rng(22))
    probs = [(_t(X1), _t(Y1), _t(f1)), (_t(X2), _t(Y2), _t(f2))]
    b = cv.cvgram_batch_create(probs, ddof=1, mode="fp64")
    cv.cvgram_batch_run(b)
    torch.cuda.synchronize()
    for (X, Y, f), (bx, by) in zip([(X1, Y1, f1), (X2, Y2, f2)], b.outs):
        sx, sy = _run(X, Y, f)
        bx = bx.cpu().numpy()
        by = by.cpu().numpy()
        assert np.max(np.abs(bx - sx)) <= 1e-13 * np.max(np.abs(sx))
        assert np.max(np.abs(by - sy)) <= 1e-13 * np.max(np.abs(sy))
    cv.cvgram_batch_destroy(b)


@pytest.mark.parametrize("path", [None, "fused"])
def test_large_P_spectra_full_size_sampled(path):
    """The spectra workload's shape (N=100000, K=512, M=8) with P=1000
    near-equal folds of 100 rows (the chosen path, and the fused one forced):
    folds written in chunks; sampled entries of three folds against the
    oracle, properties on every written fold."""
    shape = G.Shape("spectra P=1000", 100_000, 512, 8, 1000, "f64", "spectra", "near_equal")
    X, Y, fold = G.make(shape, 2, problem=1)
    print(f"[fused] {shape.name} path={path}", flush=True)
    with ForcedFoldPath(path):
        h = cv.cvgram_create(_t(X), _t(Y), _t(fold), 1, 1, 1, 1, ddof=1, mode="fp64")
    assert cv.cvgram_plan_info(h)["fused"] == (path == "fused")
    P = cv.cvgram_num_folds(h)
    assert P == 1000
    K, M = 512, 8
    rng = np.random.default_rng(3)
    for p0 in (0, 500, 990):
        xx, xy = cv.cvgram_folds_all(h, p0, p0 + 10)
        torch.cuda.synchronize()
        xx = xx.cpu().numpy()
        xy = xy.cpu().numpy()
        for q in range(10):
            nt = int((fold != p0 + q).sum())
            assert np.array_equal(xx[q, 3], xx[q, 3].T)
            assert np.allclose(np.diag(xx[q, 3]), nt - 1, rtol=1e-12)
        p = p0 + 3
        xcols = S.pick_columns(K, 16, rng)
        ycols = S.pick_columns(M, 4, rng)
        res = S.compare_fold(xx[3][:, xcols][:, :, xcols], xy[3][:, xcols][:, :, ycols],
                             X[:, xcols], Y[:, ycols], fold, p)
        for kind in ("xtx", "xty"):
            for c, (ew, fe) in enumerate(res[kind]):
                assert ew <= FP64_TOL and fe <= FP64_TOL, (p, kind, c, ew, fe)
    cv.cvgram_destroy(h)


@pytest.mark.parametrize("path", [None, "grouped"])
def test_many_folds_extrema_across_fold_ranges(path):
    """P above one range of folds in the two-level fold totals (leave-one-
    out, P = 700): a column constant except in one row (so constant over T_p
    for that row's fold only), and a column whose two distinct values sit in
    folds of different ranges."""
    n, k, m = 700, 10, 2
    print(f"[fused] extrema across fold ranges P={n} path={path}", flush=True)
    X, Y = _gaussian(n, k, m, 31)
    fold = np.random.default_rng(31).permutation(n).astype(np.int32)
    X[:, 2] = 1.5
    r_odd = int(np.where(fold == 611)[0][0])
    X[r_odd, 2] = 9.0
    X[:, 5] = 0.25
    r_a = int(np.where(fold == 17)[0][0])
    r_b = int(np.where(fold == 530)[0][0])
    X[r_a, 5] = -3.0
    X[r_b, 5] = -3.0
    xx, xy = _run(X, Y, fold, path=path)
    _against_oracle(X, Y, fold, xx, xy, 1, [0, 17, 255, 256, 530, 611, n - 1],
                    label=f"ranges-{path}")
    assert np.all(xx[611, 2][2] == 0.0)          # column 2 constant over T of fold 611
    assert np.any(xx[17, 2][5] != 0.0)           # column 5 still varies without fold 17


def test_plan_info_reports_fold_path():
    """cvgram_plan_info names the path the library chose (and the forced one)."""
    X, Y = _gaussian(600, 20, 2, 3)
    fold = np.random.default_rng(9).permutation(600).astype(np.int32) % 200  # 200 folds of 3
    infos = {}
    for path in (None, "grouped", "fused"):
        with ForcedFoldPath(path):
            h = cv.cvgram_create(_t(X), _t(Y), _t(fold), 1, 0, 1, 0, ddof=1, mode="fp64")
        infos[path] = cv.cvgram_plan_info(h)
        cv.cvgram_destroy(h)
    assert infos[None]["fused"] and infos["fused"]["fused"] and not infos["grouped"]["fused"]
    for info in infos.values():
        assert info["tile"] == 64 and info["items"] > 0 and info["slabs"] > 0


def _fold_products(h, p):
    xx, xy = cv.cvgram_folds_all(h, p, p + 1)
    return xx[0].double().cpu().numpy(), xy[0].double().cpu().numpy()


@pytest.mark.parametrize("n,k,m,ddof,n_random", [(20000, 64, 4, 1, 26), (6000, 16, 2, 0, 10),
                                                 (6000, 16, 2, 1, 10)])
def test_leave_one_out_beyond_4096_folds(n, k, m, ddof, n_random):
    """Leave-one-out with P = N > 4096: the fold sizes come from the second
    host wait (fold_offsets_kernel), the folds' totals span many ranges.  All
    12 classes of folds 0, 4095, 4096, 4097, P-1 and random others against
    the oracle at 1e-10."""
    print(f"[fused] LOO N={n} K={k} M={m} ddof={ddof}", flush=True)
    X, Y = _gaussian(n, k, m, 40 + n + ddof)
    fold = np.random.default_rng(n + ddof).permutation(n).astype(np.int32)
    h = cv.cvgram_create(_t(X), _t(Y), _t(fold), 1, 1, 1, 1, ddof=ddof, mode="fp64")
    assert cv.cvgram_num_folds(h) == n
    assert cv.cvgram_plan_info(h)["fused"]
    rng = np.random.default_rng(7)
    folds = sorted({0, 4095, 4096, 4097, n - 1,
                    *[int(v) for v in rng.choice(n, n_random, replace=False)]})
    worst = 0.0
    for p in folds:
        gxx, gxy = _fold_products(h, p)
        oxx, oxy = O.fold_all_classes(X, Y, fold, p, ddof=ddof)
        for c in range(4):
            e = _relerr(gxx[c], oxx[c])
            worst = max(worst, e)
            assert e <= FP64_TOL, ("XtX", p, c, e)
            assert np.array_equal(gxx[c], gxx[c].T)
        for c in range(8):
            e = _relerr(gxy[c], oxy[c])
            worst = max(worst, e)
            assert e <= FP64_TOL, ("XtY", p, c, e)
    cv.cvgram_destroy(h)
    print(f"[fused] LOO N={n} {len(folds)} folds worst {worst:.3e}", flush=True)
