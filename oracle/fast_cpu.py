"""The paper's fast algorithm on the CPU, in FP64 NumPy.

TEST INFRASTRUCTURE ONLY (timing baseline and second cross-check); the
product path never imports it.

Follows Algorithm 7 (fast cross-validation with centering and scaling) in the
paper's order, extended to every class of Table 1:
  full-data products X^T X, X^T Y, means, sums and sums of squares once
  (steps 3-4); per fold the validation-block products (step 8) subtracted
  from the full ones (step 9, Lemmas 2-3); the training mean by the downdate
  of Lemma 7 (steps 10-13); the rank-one centering term |T| * (mean^T mean)
  with the outer product formed first and then multiplied by |T| (step 14 and
  the implementation note of Section 7); the training sums and sums of
  squares by the downdate of Lemma 14 (steps 17-21); the deviation by the
  three-term form of Lemma 12 (steps 22-23); deviations equal to 0 replaced
  by 1 (step 24); and the Hadamard division by the outer product of the
  deviations (steps 25-27, Propositions 15-16, Table 1).

This is the method exactly as printed, with no pivot shift: Lemma 12's form
cancels when a column's mean is large against its spread, so on such data its
deviations are inaccurate (a negative argument of the square root is clamped
to 0 and then replaced by 1).  It is a baseline, not a reference.
"""
from __future__ import annotations

import numpy as np


def fast_all_folds(X, Y, fold_id, ddof: int = 1, folds=None, classes: str = "all"):
    """Yield (p, XtX[4,K,K], XtY[8,K,M]) for each fold p (class order as in
    the oracle).  ``classes="one"`` computes only the centred-and-scaled pair
    (Algorithm 7's own target) and returns it in slot 3 / slot 7."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    f = np.asarray(fold_id).ravel()
    N, K = X.shape
    M = Y.shape[1]
    P = int(f.max()) + 1
    # Algorithm 1 (stable: rows ascending within each fold)
    order = np.argsort(f, kind="stable")
    counts = np.bincount(f, minlength=P)
    offs = np.concatenate([[0], np.cumsum(counts)])
    # steps 3-4
    XTX = X.T @ X
    XTY = X.T @ Y
    mux = X.sum(axis=0) / N
    muy = Y.sum(axis=0) / N
    SX = X.sum(axis=0)
    SY = Y.sum(axis=0)
    SqX = (X * X).sum(axis=0)
    SqY = (Y * Y).sum(axis=0)
    for p in (range(P) if folds is None else folds):
        V = order[offs[p]:offs[p + 1]]
        XV = X[V]
        YV = Y[V]
        # steps 8-9
        XTX_T = XTX - XV.T @ XV
        XTY_T = XTY - XV.T @ YV
        # steps 10-13
        NV = len(V)
        NT = N - NV
        muxV = XV.sum(axis=0) / NV
        muyV = YV.sum(axis=0) / NV
        muxT = (N / NT) * mux - (NV / NT) * muxV
        muyT = (N / NT) * muy - (NV / NT) * muyV
        # steps 14-16
        cXTX_T = XTX_T - NT * np.outer(muxT, muxT)
        cXTY_T = XTY_T - NT * np.outer(muxT, muyT)
        # steps 17-21
        SX_T = SX - XV.sum(axis=0)
        SY_T = SY - YV.sum(axis=0)
        SqX_T = SqX - (XV * XV).sum(axis=0)
        SqY_T = SqY - (YV * YV).sum(axis=0)
        # steps 22-24
        sx = np.sqrt(np.maximum(0.0, (NT * muxT ** 2 + SqX_T - 2 * muxT * SX_T) / (NT - ddof)))
        sy = np.sqrt(np.maximum(0.0, (NT * muyT ** 2 + SqY_T - 2 * muyT * SY_T) / (NT - ddof)))
        sx[sx == 0] = 1.0
        sy[sy == 0] = 1.0
        # steps 25-27 and Table 1
        sxx = np.outer(sx, sx)
        xtx = np.empty((4, K, K))
        xty = np.empty((8, K, M))
        if classes == "one":
            xtx[3] = cXTX_T / sxx
            xty[7] = cXTY_T / np.outer(sx, sy)
            yield p, xtx, xty
            continue
        xtx[0] = XTX_T
        xtx[1] = XTX_T / sxx
        xtx[2] = cXTX_T
        xtx[3] = cXTX_T / sxx
        one_k = np.ones(K)
        one_m = np.ones(M)
        for c, base in ((0, XTY_T), (1, cXTY_T)):
            xty[4 * c + 0] = base
            xty[4 * c + 1] = base / np.outer(one_k, sy)
            xty[4 * c + 2] = base / np.outer(sx, one_m)
            xty[4 * c + 3] = base / np.outer(sx, sy)
        yield p, xtx, xty
