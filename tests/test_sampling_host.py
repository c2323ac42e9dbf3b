"""CPU checks of the sampled comparison helper used by the full-size GPU
parity tests: the sampled oracle block equals the oracle's full products
restricted to the sampled columns, every entry obeys the Cauchy-Schwarz
bound it is measured against, and a slip planted in one small entry is
found."""
from __future__ import annotations

import numpy as np

from oracle import cv_oracle as O
from tests import sampling as S


def _data(seed=3, n=240, k=12, m=3):
    rng = np.random.default_rng(seed)
    X = rng.normal(4.0, 1.0, (n, k)) * rng.uniform(0.5, 2.0, k)
    Y = X[:, :m] @ rng.normal(size=(m, m)) + rng.normal(0, 0.3, (n, m))
    X[:, 5] = 2.5  # a constant column: centred entries are exact zeros
    fold = rng.permutation(np.arange(n) % 4).astype(np.int32)
    return X, Y, fold


def test_block_equals_full_oracle_on_sampled_columns():
    X, Y, fold = _data()
    xc, yc = [0, 3, 5, 11], [0, 2]
    for p in range(4):
        oxx, oxy = O.fold_all_classes(X, Y, fold, p, ddof=1)
        bxx, bxy, sxx, sxy = S.oracle_block(X[:, xc], Y[:, yc], fold, p, 1)
        for c in range(4):
            assert np.allclose(bxx[c], oxx[c][np.ix_(xc, xc)], rtol=1e-13, atol=1e-11)
            assert np.all(np.abs(bxx[c]) <= sxx[c] * (1 + 1e-12) + 1e-12)
            assert np.allclose(np.diag(sxx[c]), np.abs(np.diag(bxx[c])), rtol=1e-13)
        for c in range(8):
            assert np.allclose(bxy[c], oxy[c][np.ix_(xc, yc)], rtol=1e-13, atol=1e-11)
            assert np.all(np.abs(bxy[c]) <= sxy[c] * (1 + 1e-12) + 1e-12)


def test_entrywise_error_finds_a_slip_in_a_small_entry():
    X, Y, fold = _data()
    xc, yc = [0, 3, 5, 11], [0, 2]
    bxx, bxy, sxx, sxy = S.oracle_block(X[:, xc], Y[:, yc], fold, 1, 1)
    # the centred class's smallest off-diagonal entry, nudged by 1e-6 of its
    # Cauchy-Schwarz scale: the entry-wise error shows the whole slip, the
    # Frobenius error of the block a fraction of it
    c = 2
    a = bxx[c].copy()
    off = ~np.eye(len(xc), dtype=bool) & (sxx[c] > 0)
    i, j = np.argwhere(off)[np.argmin(np.abs(a[off]))]
    a[i, j] += 1e-6 * sxx[c][i, j]
    ew = S.entrywise_error(a, bxx[c], sxx[c])
    assert ew >= 0.99e-6
    assert S.frobenius_error(a, bxx[c]) < 0.5 * ew
    # the constant column's centred entries must be exact zeros
    k5 = xc.index(5)
    assert np.all(bxx[c][k5] == 0) and np.all(sxx[c][k5] == 0)
    b = bxx[c].copy()
    b[k5, 0] = 1e-300
    assert S.entrywise_error(b, bxx[c], sxx[c]) == float("inf")
    assert S.entrywise_error(bxx[c], bxx[c], sxx[c]) == 0.0


def test_pick_columns_keeps_ends_and_is_distinct():
    rng = np.random.default_rng(0)
    cols = S.pick_columns(1024, 16, rng)
    assert cols[0] == 0 and cols[-1] == 1023 and len(set(cols)) == len(cols) == 16
    assert S.pick_columns(5, 16, rng) == [0, 1, 2, 3, 4]


def test_split_bf16_bound_covers_an_emulated_split_product():
    # the bound against a CPU emulation of the split products: hi = bf16(z),
    # lo = bf16(z - hi), hi hi' + hi lo' + lo hi' summed in FP64, with the
    # shift by a column mean rounded to FP32; and it is not vacuous (the
    # emulated error reaches a visible part of it)
    import torch
    from synth import generators as G

    def bf16(a):
        return torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()

    worst = 0.0
    for (n, k, m, p), seed in [((5, 3, 2, 2), 471), ((4, 1, 1, 2), 470), ((65, 17, 3, 13), 474)]:
        X, Y, f = G.make(G.Shape("t", n, k, m, p, "f64", "gaussian", "near_equal"), seed, 0)
        c = X.mean(axis=0).astype(np.float32).astype(np.float64)
        for q in range(p):
            bxx, bxy = S.split_bf16_bound(X, Y, f, q, ddof=1)
            assert len(bxx) == 4 and len(bxy) == 8
            T = f != q
            z = (X[T] - c).astype(np.float32).astype(np.float64)
            hi = bf16(z)
            lo = bf16(z - hi)
            err = np.abs(hi.T @ hi + hi.T @ lo + lo.T @ hi - (X[T] - c).T @ (X[T] - c))
            assert np.all(err <= bxx[0])
            worst = max(worst, float((err / bxx[0]).max()))
    assert worst > 1e-3
