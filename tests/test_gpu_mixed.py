"""GPU parity of the mixed-precision modes against the FP64 oracle.

The Gram contraction runs in FP32 MFMA or split-bf16 (bf16x3) MFMA with FP32
accumulation over row blocks of at most 256 rows combined in FP64; the
statistics and corrections are FP64.  Bars (relative Frobenius error per
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


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
def test_mixed_precision_stress_full_size_sampled(mode):
    """The precision-stress workload at full size (N=1e6, K=1024, M=16,
    P=100, FP32 input with column means in [1e3, 1e4]): sampled entries of
    three folds against the oracle, every fold against the FP64 GPU form."""
    shape, (X, Y, fold) = G.workload(3)
    print(f"[mixed] {mode} {shape.name}", flush=True)
    Xd, Yd, fd = _t(X), _t(Y), _t(fold)
    h64 = cv.cvgram_create(Xd, Yd, fd, 1, 1, 1, 1, mode="fp64")
    hm = cv.cvgram_create(Xd, Yd, fd, 1, 1, 1, 1, mode=mode)
    P = cv.cvgram_num_folds(hm)
    K, M = X.shape[1], Y.shape[1]
    worst = 0.0
    rng = np.random.default_rng(5)
    for q0 in range(0, P, 25):
        q1 = min(P, q0 + 25)
        a64, b64 = cv.cvgram_folds_all(h64, q0, q1)
        am, bm = cv.cvgram_folds_all(hm, q0, q1)
        for q in range(q1 - q0):
            for c in range(4):
                ref = a64[q, c]
                e = (torch.linalg.norm(am[q, c].double() - ref) / torch.linalg.norm(ref)).item()
                worst = max(worst, e)
                assert e <= MIXED_BOUND[mode], (mode, q0 + q, c, e)
            for c in range(8):
                ref = b64[q, c]
                e = (torch.linalg.norm(bm[q, c].double() - ref) / torch.linalg.norm(ref)).item()
                worst = max(worst, e)
                assert e <= MIXED_BOUND[mode], (mode, q0 + q, c, e)
        if q0 == 0:
            am0, bm0 = am.cpu().numpy(), bm.cpu().numpy()
    print(f"[mixed] {mode} full-size worst rel err vs FP64 GPU form {worst:.3e}", flush=True)
    # sampled entries of fold 0 against the oracle (entry-wise, scaled by the
    # class's largest entry)
    pairs_xx = [(int(a), int(b)) for a, b in rng.integers(0, K, size=(10, 2))] + [(3, 3)]
    pairs_xy = [(int(a), int(b)) for a, b in zip(rng.integers(0, K, 6), rng.integers(0, M, 6))]
    for c in range(4):
        ref, _ = O.fold_entries(X, Y, fold, 0, *O.XTX_CLASS_COMBO[c], 1, pairs_xx, [])
        got = np.array([am0[0, c, i, j] for i, j in pairs_xx], np.float64)
        assert np.max(np.abs(got - ref)) <= 10 * MIXED_BOUND[mode] * np.max(np.abs(am0[0, c])), c
    for c in range(8):
        _, ref = O.fold_entries(X, Y, fold, 0, *O.XTY_CLASS_COMBO[c], 1, [], pairs_xy)
        got = np.array([bm0[0, c, i, j] for i, j in pairs_xy], np.float64)
        assert np.max(np.abs(got - ref)) <= 10 * MIXED_BOUND[mode] * np.max(np.abs(bm0[0, c])), c
    cv.cvgram_destroy(hm)
    cv.cvgram_destroy(h64)
