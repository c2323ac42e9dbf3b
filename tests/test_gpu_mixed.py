"""GPU parity of the mixed-precision modes against the FP64 oracle.

The Gram contraction runs in FP32 MFMA or split-bf16 (bf16x3) MFMA with FP32
accumulation over row blocks of at most 256 rows, combined in FP64 (or, on
bf16x3's 256 x 128 tiles, in FP32 running totals); the statistics and
corrections are FP64.  Bars (relative Frobenius error per
fold x class x output, against the oracle):
    fp32    <= MIXED_BOUND["fp32"]
    bf16x3  <= MIXED_BOUND["bf16x3"]
Fold bookkeeping and training statistics are shared with the FP64 path and
are checked there.
"""
from __future__ import annotations

import numpy as np
import pytest

import paper_2401_13185_amd as cv
from oracle import cv_oracle as O
from synth import generators as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MIXED_BOUND = {"fp32": 1e-6, "bf16x3": 2e-5}


def _dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    return torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(_dev())


def _relerr(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / nb) if nb else float(np.linalg.norm(a))


def _run(X, Y, fold, mode, ddof=1):
    h = cv.cvgram_create(_t(X), _t(Y) if Y.shape[1] else None, _t(fold), 1, 1, 1, 1, ddof=ddof,
                         mode=mode)
    P = cv.cvgram_num_folds(h)
    xx, xy = cv.cvgram_folds_all(h, 0, P)
    torch.cuda.synchronize()
    out = (xx.cpu().numpy(), xy.cpu().numpy() if xy is not None else None)
    cv.cvgram_destroy(h)
    return P, out


CASES = [
    # (n, k, m, p, values, dtype)
    (20000, 200, 16, 10, "offset", "f32"),     # large offsets, FP32 input
    (12000, 256, 8, 7, "spectra", "f32"),      # spectra, exact tile multiple
    (3001, 130, 5, 7, "spectra", "f64"),       # ragged rows/tiles, FP64 input
    (900, 40, 0, 4, "gaussian", "f64"),        # no Y, K below one tile
    (5000, 300, 130, 5, "gaussian", "f32"),    # Y wider than one tile
    (6000, 160, 30, 5, "offset", "f32"),       # 16 < M <= 32 inside diagonal tiles
    (4000, 700, 0, 4, "spectra", "f32"),       # three 256-column blocks, ragged, no Y
    (2000, 2100, 7, 3, "offset", "f32"),       # tiles visited in groups (K > 1920)
]


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_mixed_against_oracle(mode, case):
    n, k, m, p, values, dtype = CASES[case]
    shape = G.Shape(f"{values} N={n} K={k} M={m} P={p} {dtype}", n, k, m, p, dtype, values,
                    "dirichlet")
    X, Y, fold = G.make(shape, 700 + case, 0)
    print(f"[mixed] {mode} {shape.name}", flush=True)
    P, (xx, xy) = _run(X, Y, fold, mode)
    assert xx.dtype == np.float32
    worst = {"xtx": 0.0, "xty": 0.0}
    for q in range(P):
        oxx, oxy = O.fold_all_classes(X, Y, fold, q, ddof=1)
        for c in range(4):
            e = _relerr(xx[q, c], oxx[c])
            worst["xtx"] = max(worst["xtx"], e)
            assert e <= MIXED_BOUND[mode], (mode, shape.name, "XtX", q, c, e)
            assert np.array_equal(xx[q, c], xx[q, c].T)
        for c in range(8 if m else 0):
            e = _relerr(xy[q, c], oxy[c])
            worst["xty"] = max(worst["xty"], e)
            assert e <= MIXED_BOUND[mode], (mode, shape.name, "XtY", q, c, e)
    print(f"[mixed] {mode} {shape.name} worst rel err {worst}", flush=True)


@pytest.mark.parametrize("mode", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("order", ["drift", "sorted"])
def test_rows_ordered_by_a_covariate(mode, order):
    """Offset columns (means in [1e3, 1e4]) whose rows are ordered by a
    covariate: a drift along the rows of 40 column deviations end to end,
    or all rows sorted by column 0.  The first rows then sit far from each
    column's mean; the pivot is taken from rows spread over the whole
    column, so the centred classes cancel no more than on shuffled rows.
    Whole products against the oracle (relative Frobenius per fold x class)
    and every entry against its Cauchy-Schwarz scale, at the mode's bar."""
    from tests import sampling as S
    n, k, m, p = 30000, 96, 4, 6
    rng = np.random.default_rng(77)
    mu = rng.uniform(1e3, 1e4, k)
    sd = rng.uniform(0.1, 1.0, k)
    z = rng.standard_normal((n, k))
    if order == "drift":
        z += 40.0 * (np.arange(n)[:, None] / n - 0.5)
    X = (mu + sd * z).astype(np.float32)
    if order == "sorted":
        X = X[np.argsort(X[:, 0], kind="stable")]
    W = rng.standard_normal((k, m)) / np.sqrt(k)
    Y = (rng.uniform(1e3, 1e4, m) + ((X - mu) / sd) @ W
         + 0.1 * rng.standard_normal((n, m))).astype(np.float32)
    fold = G.folds_dirichlet(n, p, np.random.default_rng(78))
    print(f"[mixed] {mode} rows ordered by {order} N={n} K={k}", flush=True)
    P, (xx, xy) = _run(X, Y, fold, mode)
    tol = 1e-10 if mode == "fp64" else MIXED_BOUND[mode]
    worst = 0.0
    for q in range(P):
        oxx, oxy = O.fold_all_classes(X, Y, fold, q, ddof=1)
        d = {}
        for c, (cx, sx, _, _) in O.XTX_CLASS_COMBO.items():
            d[("x", cx, sx)] = np.diag(oxx[c])
            e = _relerr(xx[q, c], oxx[c])
            ew = S.entrywise_error(xx[q, c], oxx[c], np.sqrt(np.outer(np.diag(oxx[c]),
                                                                     np.diag(oxx[c]))))
            worst = max(worst, e, ew)
            assert e <= tol and ew <= tol, (mode, order, "XtX", q, c, e, ew)
        for c, (cx, sx, cy, sy) in O.XTY_CLASS_COMBO.items():
            yy, _ = O.fold_products(Y, Y, fold, q, cy, sy, cy, sy, ddof=1)
            scale = np.sqrt(np.outer(d[("x", cx, sx)], np.diag(yy)))
            e = _relerr(xy[q, c], oxy[c])
            ew = S.entrywise_error(xy[q, c], oxy[c], scale)
            worst = max(worst, e, ew)
            assert e <= tol and ew <= tol, (mode, order, "XtY", q, c, e, ew)
    print(f"[mixed] {mode} {order}: worst {worst:.3e}", flush=True)
