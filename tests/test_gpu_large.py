"""The large single problem at full size: spectra N=2,000,000, K=4096, M=64,
P=64, FP32 input, Dirichlet(2) folds (values drawn on the device, as the
bench's large block does), in the launch configuration the bench times.

FP64 mode against the FP64 oracle on sampled entries of three folds (the
smallest, the largest and fold 0): every entry among 16 columns of X and 4
of Y, computed by the oracle from those columns copied to the host, within
1e-10 of its Cauchy-Schwarz scale (tests/sampling.py); BF16X3 mode against the FP64 GPU
form on the same folds' whole products, within the stated bound.
"""
from __future__ import annotations

import numpy as np
import pytest

import paper_2401_13185_amd as cv
from oracle import cv_oracle as O
from synth import generators as G
from tests import sampling as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FP64_TOL = 1e-10
BF16X3_BOUND = 2e-5


def _dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    return torch.device("cuda:0")


def test_large_problem_sampled_and_mixed_bound():
    dev = _dev()
    shape = G.WORKLOADS[5]
    N, K, M, P = shape.n, shape.k, shape.m, shape.p
    print(f"[large] {shape.name}", flush=True)
    X, Y = G.spectra_xy_torch(N, K, M, seed=5_13185, device=dev)
    fold = G.folds_dirichlet(N, P, G._rng(5, 0, 9))
    fd = torch.from_numpy(fold).to(dev)
    sizes = np.bincount(fold, minlength=P)
    folds = sorted({0, int(np.argmin(sizes)), int(np.argmax(sizes))})

    out = {}
    for mode in ("fp64", "bf16x3"):
        odt = torch.float64 if mode == "fp64" else torch.float32
        h = cv.cvgram_create(X, Y, fd, 1, 1, 1, 1, ddof=1, mode=mode)
        res = []
        for p in folds:
            xx = torch.empty(1, 4, K, K, dtype=odt, device=dev)
            xy = torch.empty(1, 8, K, M, dtype=odt, device=dev)
            cv.cvgram_folds_all(h, p, p + 1, xx, xy)
            res.append((xx[0], xy[0]))
        torch.cuda.synchronize()
        cv.cvgram_destroy(h)
        out[mode] = res
        print(f"[large] mode {mode} done", flush=True)

    # BF16X3 against the FP64 GPU form, every class of the checked folds
    worst = 0.0
    for (bx, by), (fx, fy) in zip(out["bf16x3"], out["fp64"]):
        for a, b in ((bx, fx), (by, fy)):
            num = torch.linalg.matrix_norm(a.double() - b)
            worst = max(worst, (num / torch.linalg.matrix_norm(b)).max().item())
    assert worst <= BF16X3_BOUND, worst

    # FP64 against the oracle on sampled entries: every entry among 16 X and
    # 4 Y columns (copied to the host), against its Cauchy-Schwarz scale
    rng = np.random.default_rng(55)
    xcols = S.pick_columns(K, 16, rng)
    ycols = S.pick_columns(M, 4, rng)
    Xs = X[:, xcols].double().cpu().numpy()
    Ys = Y[:, ycols].double().cpu().numpy()
    xi = torch.tensor(xcols, device=dev)
    yi = torch.tensor(ycols, device=dev)
    for (fx, fy), p in zip(out["fp64"], folds):
        gxx = fx[:, xi][:, :, xi].cpu().numpy()
        gxy = fy[:, xi][:, :, yi].cpu().numpy()
        res = S.compare_fold(gxx, gxy, Xs, Ys, fold, p)
        for kind in ("xtx", "xty"):
            for c, (ew, fe) in enumerate(res[kind]):
                assert ew <= FP64_TOL and fe <= FP64_TOL, (p, kind, c, ew, fe)
        # properties that hold at any size
        nt = int((fold != p).sum())
        assert torch.equal(fx[3], fx[3].T)
        assert torch.allclose(torch.diagonal(fx[3]), torch.full((K,), nt - 1.0, dtype=fx.dtype,
                                                                 device=fx.device), rtol=1e-12)
    del X, Y, fd, out
    torch.cuda.empty_cache()
