"""Sampled, entry-wise comparison of GPU training products with the oracle.

At sizes where the oracle cannot materialise every product, a test picks a
few columns of X and Y, copies only those columns to the host and lets the
oracle compute every entry among them (each entry needs only its two
columns: centering and scaling are column-wise, Definitions 2-5).

Entry-wise error scale (a reading: the paper states no tolerance): an entry
(i, j) of a Gram product A = U^T V is bounded by Cauchy-Schwarz,
|A_ij| <= ||u_i|| ||v_j|| = sqrt((U^T U)_ii (V^T V)_jj), so an error is
measured against that bound:
    err_ij = |gpu_ij - oracle_ij| / sqrt((U^T U)_ii (V^T V)_jj)
with U, V the preprocessed training columns of the entry's class (X's for
X^T X; X's and Y's for X^T Y, both centred when the class is centred,
Lemma 9).  This is the relative error of the entry measured against the
largest value such an entry can take, so a slip in a small entry (a centred
cross product near zero) is not hidden by the class's largest entries.  A
zero scale (a column constant over T and centred) requires an exact zero.
"""
from __future__ import annotations

import numpy as np

from oracle import cv_oracle as O


def pick_columns(n: int, count: int, rng) -> list[int]:
    """`count` distinct columns of n (always the first and the last)."""
    if n <= count:
        return list(range(n))
    mid = rng.choice(np.arange(1, n - 1), size=count - 2, replace=False)
    return sorted({0, n - 1, *[int(c) for c in mid]})


def oracle_block(Xs, Ys, fold, p: int, ddof: int = 1):
    """Oracle values of every class on the sampled columns of fold p:
    xx[4][kx][kx], xy[8][kx][ky], and the Cauchy-Schwarz scales sxx, sxy of
    the same shapes.  Xs (N x kx) and Ys (N x ky) hold the sampled columns;
    the oracle's products of that column subset are the sampled entries of
    the full products (centering and scaling are column-wise)."""
    xx, xy = O.fold_all_classes(Xs, Ys, fold, p, ddof=ddof)
    # Y's preprocessed squared norms: Y taken as the X of a second call
    yy, _ = O.fold_all_classes(Ys, Ys[:, :0], fold, p, ddof=ddof)
    sxx = np.empty_like(xx)
    sxy = np.empty_like(xy)
    for c in range(4):
        d = np.diag(xx[c])
        sxx[c] = np.sqrt(np.outer(d, d))
    for c, (cx, sx, cy, sy) in O.XTY_CLASS_COMBO.items():
        dx = np.diag(xx[O.xtx_class(cx, sx)])
        dy = np.diag(yy[O.xtx_class(cy, sy)])
        sxy[c] = np.sqrt(np.outer(dx, dy))
    return xx, xy, sxx, sxy


def entrywise_error(got, ref, scale):
    """Largest entry-wise error (see the module docstring); entries whose
    scale is 0 must match exactly (else +inf)."""
    got = np.asarray(got, dtype=np.float64)
    diff = np.abs(got - ref)
    zero = scale == 0
    if np.any(diff[zero] != 0):
        return float("inf")
    if np.all(zero):
        return 0.0
    return float(np.max(diff[~zero] / scale[~zero]))


def frobenius_error(got, ref):
    """Relative Frobenius error of the sampled block."""
    got = np.asarray(got, dtype=np.float64)
    nr = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref)) if nr == 0 else float(np.linalg.norm(got - ref) / nr)


def compare_block(gxx, gxy, ref):
    """Per class errors of sampled GPU blocks gxx[4][kx][kx] and gxy[8][kx][ky]
    against an oracle block ``ref = oracle_block(...)``:
    {"xtx": [(entrywise, frobenius)] * 4, "xty": [...] * 8}."""
    oxx, oxy, sxx, sxy = ref
    out = {"xtx": [], "xty": []}
    for c in range(4):
        out["xtx"].append((entrywise_error(gxx[c], oxx[c], sxx[c]),
                           frobenius_error(gxx[c], oxx[c])))
    for c in range(8 if oxy.shape[2] else 0):
        out["xty"].append((entrywise_error(gxy[c], oxy[c], sxy[c]),
                           frobenius_error(gxy[c], oxy[c])))
    return out


def compare_fold(gxx, gxy, Xs, Ys, fold, p, ddof=1):
    """compare_block against the oracle block of fold p."""
    return compare_block(gxx, gxy, oracle_block(Xs, Ys, fold, p, ddof))


def split_bf16_bound(X, Y, fold, p: int, ddof: int = 1):
    """Per-entry error bounds of fold p's split-bf16 (BF16X3) products, for
    problems whose sums are too short to average rounding out.

    Reading (the paper fixes no tolerance for reduced precision): a
    pivot-shifted value z = x - c is carried as hi + lo, hi = bf16(z),
    lo = bf16(z - hi); bf16 rounds to within 2^-9 relative, so
    |z - hi - lo| <= 2^-18 |z|.  The product (hi + lo)(hi' + lo') less the
    dropped lo lo' then errs by at most 3 2^-18 |z z'|, and the FP32 sum
    over the |T| training rows adds at most |T| 2^-24 sum |z z'|.  The pivot
    is a mean of the column's values, so |z| is at most the column's range
    R (over all rows) and sum_T |z_i z_j| <= |T| R_i R_j.  Undoing the shift
    and centring run in FP64 on FP64 statistics and add nothing at this
    scale; a scaled class divides by the training deviations.
    Returns ([4 X^T X bounds], [8 X^T Y bounds])."""
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    T = np.asarray(fold) != p
    nT = int(T.sum())
    eps = 3.0 * 2.0 ** -18 + nT * 2.0 ** -24

    def col_range(A):
        if A.shape[1] == 0:
            return np.zeros(0)
        # slack for a pivot rounded to FP32
        return A.max(axis=0) - A.min(axis=0) + 2.0 ** -20 * np.abs(A).max(axis=0)

    def deviations(A):
        if A.shape[1] == 0:
            return np.zeros(0)
        At = A[T]
        s = At.std(axis=0, ddof=ddof)
        const = (At == At[0]).all(axis=0)
        return np.where(const | (s == 0.0), 1.0, s)

    Rx, Ry = col_range(X), col_range(Y)
    sx, sy = deviations(X), deviations(Y)
    bxx, bxy = [], []
    for _c, (_cx, scx, _cy, _sy) in O.XTX_CLASS_COMBO.items():
        b = eps * nT * np.outer(Rx, Rx)
        bxx.append(b / np.outer(sx, sx) if scx else b)
    for _c, (_cx, scx, _cy, scy) in O.XTY_CLASS_COMBO.items():
        b = eps * nT * np.outer(Rx, Ry)
        if scx:
            b = b / sx[:, None]
        if scy:
            b = b / sy[None, :]
        bxy.append(b)
    return bxx, bxy
