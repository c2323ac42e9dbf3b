"""GPU parity of the leakage-comparison modes (cvgram_fold_leaky) against the
FP64 oracle's definitions: preprocessing with all-row statistics, and
Lindgren et al.'s Equation (20) as restated in Lemma 11's proof.  These are
comparison modes only; the tests also check that they differ from the
training-partition products (the leak of Section 4.1)."""
from __future__ import annotations

import os

import numpy as np
import pytest

import paper_2401_13185_amd as cv
from oracle import cv_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FP64_TOL = 1e-10


def _t(a):
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def _relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a)) if nb == 0.0 else float(np.linalg.norm(a - b) / nb)


def _data(n, k, m, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(4.0, 1.5, size=(n, k)) + rng.normal(0, 3, size=k)
    Y = X[:, :m] * 0.5 + rng.normal(1.0, 0.5, size=(n, m))
    return X, Y


def _leaky(X, Y, fold, combo, kind, ddof=1, mode="fp64", path=None):
    old = os.environ.get("CVGRAM_FOLD_PATH")
    if path:
        os.environ["CVGRAM_FOLD_PATH"] = path
    try:
        h = cv.cvgram_create(_t(X), _t(Y), _t(fold.astype(np.int32)), *combo, ddof=ddof, mode=mode)
    finally:
        if path:
            if old is None:
                os.environ.pop("CVGRAM_FOLD_PATH", None)
            else:
                os.environ["CVGRAM_FOLD_PATH"] = old
    out = []
    for p in range(cv.cvgram_num_folds(h)):
        xx, xy = cv.cvgram_fold_leaky(h, p, kind)
        torch.cuda.synchronize()
        out.append((xx.double().cpu().numpy(), xy.double().cpu().numpy()))
    cv.cvgram_destroy(h)
    return out


@pytest.mark.parametrize("ddof", [0, 1])
def test_global_statistics_every_combination(ddof):
    X, Y = _data(400, 12, 3, 1)
    fold = np.random.default_rng(1).integers(0, 5, size=400).astype(np.int32)
    fold[:5] = np.arange(5)
    print(f"[leaky] global, all 16 combinations, ddof={ddof}", flush=True)
    for combo in O.COMBOS:
        got = _leaky(X, Y, fold, combo, "global", ddof=ddof)
        for p, (gx, gy) in enumerate(got):
            ox, oy = O.leaky_global_fold(X, Y, fold, p, *combo, ddof=ddof)
            assert _relerr(gx, ox) <= FP64_TOL, (combo, p, "XtX")
            assert _relerr(gy, oy) <= FP64_TOL, (combo, p, "XtY")
            assert np.array_equal(gx, gx.T)


@pytest.mark.parametrize("path", ["grouped", "fused"])
def test_global_statistics_constant_columns_both_paths(path):
    n, P = 320, 80                                   # folds of 4 rows
    X, Y = _data(n, 9, 2, 2)
    X[:, 4] = -2.5                                   # constant over all rows
    fold = np.arange(n, dtype=np.int32) % P
    print(f"[leaky] global, constant column, path={path}", flush=True)
    for combo in [(1, 1, 1, 1), (1, 0, 0, 1), (0, 1, 1, 0)]:
        got = _leaky(X, Y, fold, combo, "global", path=path)
        for p in (0, 41, P - 1):
            ox, oy = O.leaky_global_fold(X, Y, fold, p, *combo, ddof=1)
            assert _relerr(got[p][0], ox) <= FP64_TOL, (combo, p)
            assert _relerr(got[p][1], oy) <= FP64_TOL, (combo, p)
        if combo[0]:
            assert np.all(got[0][0][4] == 0.0)


@pytest.mark.parametrize("path", ["grouped", "fused"])
def test_lindgren_equation20(path):
    n, P = 360, 90
    X, Y = _data(n, 10, 3, 3)
    fold = np.random.default_rng(3).permutation(np.arange(n) % P).astype(np.int32)
    print(f"[leaky] Lindgren, path={path}", flush=True)
    got = _leaky(X, Y, fold, (1, 0, 1, 0), "lindgren", path=path)
    for p in (0, 17, P - 1):
        ox, oy = O.leaky_lindgren_fold(X, Y, fold, p)
        assert _relerr(got[p][0], ox) <= FP64_TOL, p
        assert _relerr(got[p][1], oy) <= FP64_TOL, p
        tx, _ = O.fold_products(X, Y, fold, p, 1, 0, 1, 0, ddof=1)
        assert _relerr(got[p][0], tx) > 1e-6          # the leak is visible


@pytest.mark.parametrize("mode,bound", [("fp32", 1e-6), ("bf16x3", 2e-5)])
def test_global_statistics_mixed_modes(mode, bound):
    X, Y = _data(2000, 40, 4, 4)
    X = X.astype(np.float32)
    Y = Y.astype(np.float32)
    fold = np.arange(2000, dtype=np.int32) % 6
    got = _leaky(X, Y, fold, (1, 1, 1, 1), "global", mode=mode)
    for p in range(6):
        ox, oy = O.leaky_global_fold(X, Y, fold, p, 1, 1, 1, 1, ddof=1)
        assert _relerr(got[p][0], ox) <= bound
        assert _relerr(got[p][1], oy) <= bound


def test_leaky_argument_errors():
    X, Y = _data(50, 4, 1, 5)
    fold = np.arange(50, dtype=np.int32) % 5
    h = cv.cvgram_create(_t(X), _t(Y), _t(fold), 1, 1, 1, 1)
    with pytest.raises(cv.CVGramError) as ei:
        cv.cvgram_fold_leaky(h, 0, "lindgren")       # needs centering only
    assert ei.value.status == 1
    with pytest.raises(cv.CVGramError) as ei:
        cv.cvgram_fold_leaky(h, 5, "global")
    assert ei.value.status == 6
    lib = cv.load()
    assert lib.cvgram_fold_leaky(h.ptr, 0, 3, None, None) == 1
    cv.cvgram_destroy(h)
