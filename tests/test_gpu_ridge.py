"""GPU parity of the per-fold ridge-regression consumer (cvgram_ridge:
blocked Cholesky and triangular solves on the device) against the oracle's
dense solve of the definitional products."""
from __future__ import annotations

import numpy as np
import pytest

import paper_2401_13185_amd as cv
from oracle import cv_oracle as O
from synth import generators as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _t(a):
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def _relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


def _data(n, k, m, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(3.0, 1.0, size=(n, k)) + rng.normal(0, 2, size=k)
    Y = X @ rng.normal(size=(k, m)) / np.sqrt(k) + rng.normal(0, 0.5, size=(n, m))
    return X, Y


# K = 1 and K = M = 64: one live row of a padded block, and exactly one block
# of each without padding.  K <= 512 (Kp <= 512) takes the matrix-core
# backward substitution, 16 columns of B per workgroup (M = 40: three column
# blocks, the last ragged; K = 512, M = 17: every wave's four row tiles, two
# column blocks; M = 130: three 64-row blocks of right-hand sides below the
# matrix, the last with two live rows); K > 512 the row-per-thread path
@pytest.mark.parametrize("n,k,m,P", [(300, 1, 2, 3), (600, 40, 3, 5), (900, 45, 40, 4),
                                     (800, 64, 64, 3), (1500, 70, 1, 3), (1200, 100, 12, 4),
                                     (2000, 100, 130, 3), (1400, 512, 17, 3), (2500, 600, 4, 3)])
def test_ridge_matches_oracle(n, k, m, P):
    X, Y = _data(n, k, m, k)
    fold = np.random.default_rng(k).integers(0, P, size=n).astype(np.int32)
    fold[:P] = np.arange(P)
    lams = [0.0, 0.1, 10.0]
    print(f"[ridge] N={n} K={k} M={m} P={P}", flush=True)
    for combo in [(1, 1, 1, 1), (0, 0, 0, 0), (1, 0, 1, 0), (0, 1, 1, 0)]:
        h = cv.cvgram_create(_t(X), _t(Y), _t(fold), *combo, ddof=1, mode="fp64")
        B = cv.cvgram_ridge(h, 0, P, lams)
        torch.cuda.synchronize()
        B = B.cpu().numpy()
        cv.cvgram_destroy(h)
        for p in range(P):
            for l, lam in enumerate(lams):
                ref = O.ridge_fold(X, Y, fold, p, *combo, 1, lam)
                assert _relerr(B[p, l], ref) <= 1e-8, (combo, p, lam)


def test_ridge_many_blocks_and_fold_subrange():
    """K = 300 (ten block columns of 32, a partial last one), folds 2..5 of 7."""
    X, Y = _data(4000, 300, 6, 9)
    fold = np.arange(4000, dtype=np.int32) % 7
    h = cv.cvgram_create(_t(X), _t(Y), _t(fold), 1, 1, 1, 1, ddof=1)
    lams = [0.5, 50.0]
    B = cv.cvgram_ridge(h, 2, 6, lams)
    torch.cuda.synchronize()
    B = B.cpu().numpy()
    cv.cvgram_destroy(h)
    for f, p in enumerate(range(2, 6)):
        for l, lam in enumerate(lams):
            assert _relerr(B[f, l], O.ridge_fold(X, Y, fold, p, 1, 1, 1, 1, 1, lam)) <= 1e-8


def test_ridge_singular_and_argument_errors():
    X, Y = _data(30, 40, 2, 4)                      # K > |T|: X^T X_T is singular
    fold = np.arange(30, dtype=np.int32) % 3
    h = cv.cvgram_create(_t(X), _t(Y), _t(fold), 1, 0, 1, 0, ddof=1)
    with pytest.raises(cv.CVGramError) as ei:
        cv.cvgram_ridge(h, 0, 3, [0.0])
    assert ei.value.status == 7
    B = cv.cvgram_ridge(h, 0, 3, [1.0])             # regularised: positive definite
    torch.cuda.synchronize()
    ref = O.ridge_fold(X, Y, fold, 1, 1, 0, 1, 0, 1, 1.0)
    assert _relerr(B[1, 0].cpu().numpy(), ref) <= 1e-8
    for args, status in [((0, 4, [1.0]), 6), ((2, 2, [1.0]), 6), ((0, 1, [-1.0]), 1),
                         ((0, 1, [float("nan")]), 1)]:
        with pytest.raises(cv.CVGramError) as ei:
            cv.cvgram_ridge(h, *args)
        assert ei.value.status == status, args
    cv.cvgram_destroy(h)


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
def test_ridge_from_mixed_products(mode):
    X, Y = _data(3000, 64, 4, 12)
    X = X.astype(np.float32)
    Y = Y.astype(np.float32)
    fold = np.arange(3000, dtype=np.int32) % 5
    h = cv.cvgram_create(_t(X), _t(Y), _t(fold), 1, 1, 1, 1, ddof=1, mode=mode)
    B = cv.cvgram_ridge(h, 0, 5, [1.0])
    torch.cuda.synchronize()
    B = B.cpu().numpy()
    cv.cvgram_destroy(h)
    for p in range(5):
        ref = O.ridge_fold(X, Y, fold, p, 1, 1, 1, 1, 1, 1.0)
        assert _relerr(B[p, 0], ref) <= 1e-4, p


def test_ridge_spectra_workload_one_fold():
    shape, (X, Y, fold) = G.workload(2)
    print(f"[ridge] {shape.name}", flush=True)
    h = cv.cvgram_create(_t(X), _t(Y), _t(fold), 1, 1, 1, 1, ddof=1)
    lams = [1e-3, 1.0, 100.0]
    B = cv.cvgram_ridge(h, 0, shape.p, lams)
    torch.cuda.synchronize()
    B = B.cpu().numpy()
    cv.cvgram_destroy(h)
    assert np.all(np.isfinite(B))
    for l, lam in enumerate(lams):
        ref = O.ridge_fold(X, Y, fold, 4, 1, 1, 1, 1, 1, lam)
        assert _relerr(B[4, l], ref) <= 1e-6, lam


def test_ridge_many_systems():
    """256 systems (32 folds x 8 penalties) at K = 384, M = 8 (six block
    steps, trailing-update launches of up to 5 120 workgroups): every system
    against the oracle's products and a dense solve."""
    n, k, m, P = 4000, 384, 8, 32
    X, Y = _data(n, k, m, 31)
    fold = np.random.default_rng(31).integers(0, P, size=n).astype(np.int32)
    fold[:P] = np.arange(P)
    lams = list(np.logspace(-3, 4, 8))
    h = cv.cvgram_create(_t(X), _t(Y), _t(fold), 1, 1, 1, 1, ddof=1)
    print(f"[ridge] N={n} K={k} M={m} P={P} x {len(lams)} penalties", flush=True)
    B = cv.cvgram_ridge(h, 0, P, lams)
    torch.cuda.synchronize()
    B = B.cpu().numpy()
    cv.cvgram_destroy(h)
    for p in range(P):
        xtx, xty = O.fold_products(X, Y, fold, p, 1, 1, 1, 1, 1)
        for l, lam in enumerate(lams):
            ref = np.linalg.solve(xtx + lam * np.eye(k), xty)
            assert _relerr(B[p, l], ref) <= 1e-8, (p, lam)


def test_ridge_many_penalties():
    """65 penalties: one more than travel in the kernel arguments, so they are
    read from a device copy."""
    X, Y = _data(600, 20, 3, 5)
    fold = np.arange(600, dtype=np.int32) % 3
    lams = list(np.logspace(-3, 3, 65))
    h = cv.cvgram_create(_t(X), _t(Y), _t(fold), 1, 1, 1, 1, ddof=1)
    B = cv.cvgram_ridge(h, 0, 3, lams)
    torch.cuda.synchronize()
    B = B.cpu().numpy()
    for p in range(3):
        xtx, xty = O.fold_products(X, Y, fold, p, 1, 1, 1, 1, 1)
        for l in (0, 31, 63, 64):
            ref = np.linalg.solve(xtx + lams[l] * np.eye(20), xty)
            assert _relerr(B[p, l], ref) <= 1e-8, (p, l)
    cv.cvgram_destroy(h)
