"""FP64 CPU oracle for per-fold training-partition X^T X and X^T Y.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import this module; the product path (the HIP
library and its Python binding) never does, and shares no code with it.

What it computes is the paper's *baseline* definition, not its fast method:
for every fold p it materialises the training rows T_p = R minus V_p
(Definition 1), takes their column means (Definition 2) and sample standard
deviations (Definition 4), centres and/or scales (Definitions 3 and 5) and
multiplies (Algorithm 6, steps 4-12, generalised to every centering/scaling
combination of Section 6 and Table 1).  The fast algorithm reaches exactly the
same result (Propositions 1, 9 and 17), so this plain definition is the
reference it must match.

Readings where the paper is silent or only implicit:
  * fold labels are 0-based ints; label p is the paper's partition p+1, and
    P = max(label)+1 with every label in [0, P) used and 2 <= P <= N
    (Definition 1);
  * the deviation divisor is |T| - ddof with ddof in {0, 1}; ddof = 1 is the
    paper's Bessel correction (Definition 4).  Scaling needs |T| - ddof >= 1
    for every fold (Definition 6 generalised);
  * the rule that a zero deviation becomes 1 (Algorithm 6 step 10, Algorithm 7
    step 24) is read as: column j is constant over T.  Such a column keeps
    deviation 1, and its mean is the constant itself, so a centred constant
    column is exactly zero;
  * scaling without centering divides the raw training columns by the
    deviation about the training mean (the remark after Proposition 16,
    Table 1 first column);
  * X's preprocessing is the same in both products (Section 6), which leaves
    4 distinct X^T X and 8 distinct X^T Y; their class numbering is given by
    ``xtx_class`` and ``xty_class``.

Precision: all arithmetic in FP64 (FP32 inputs are widened exactly first).

Two leaky comparison modes (``leaky_global_fold``, ``leaky_lindgren_fold``)
compute what Section 4.1 shows to be wrong, for numerical demonstrations of
the leak; they are never the default.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "COMBOS", "xtx_class", "xty_class", "XTX_CLASS_COMBO", "XTY_CLASS_COMBO",
    "validation_partitions", "bookkeeping", "training_rows", "column_stats",
    "preprocess", "fold_products", "fold_all_classes", "fold_entries",
    "fold_train_stats", "leaky_global_fold", "leaky_lindgren_fold", "ridge_fold", "OracleError",
]


class OracleError(ValueError):
    pass


# (center_x, scale_x, center_y, scale_y) for all 16 combinations (Section 6)
COMBOS = [(cx, sx, cy, sy) for cx in (0, 1) for sx in (0, 1) for cy in (0, 1) for sy in (0, 1)]


def xtx_class(cx: int, sx: int, cy: int = 0, sy: int = 0) -> int:
    """X^T X depends on X's preprocessing only: 0 raw, 1 scaled, 2 centred,
    3 centred and scaled."""
    return 2 * int(bool(cx)) + int(bool(sx))


def xty_class(cx: int, sx: int, cy: int, sy: int) -> int:
    """X^T Y depends on (centre X or Y, scale X, scale Y) (Lemma 9, Table 1):
    4*c + 2*sx + sy with c = cx or cy."""
    c = int(bool(cx) or bool(cy))
    return 4 * c + 2 * int(bool(sx)) + int(bool(sy))


# one representative combination per class
XTX_CLASS_COMBO = {0: (0, 0, 0, 0), 1: (0, 1, 0, 0), 2: (1, 0, 1, 0), 3: (1, 1, 1, 0)}
XTY_CLASS_COMBO = {c: ((c >> 2) & 1, (c >> 1) & 1, (c >> 2) & 1, c & 1) for c in range(8)}


# ---------------------------------------------------------------------------
# Algorithm 1: validation partitions
# ---------------------------------------------------------------------------

def validation_partitions(fold_id) -> list[list[int]]:
    """Algorithm 1: V[p] collects every row n with label p, visiting n in
    ascending order, so each V[p] is in ascending row order.  Checks
    Definition 1 (2 <= P <= N, labels in [0, P), no empty fold)."""
    labels = [int(v) for v in np.asarray(fold_id).ravel()]
    n = len(labels)
    if n == 0:
        raise OracleError("empty partitioning")
    lo, hi = min(labels), max(labels)
    if lo < 0:
        raise OracleError("negative fold label")
    p_count = hi + 1
    if p_count < 2 or p_count > n:
        raise OracleError("need 2 <= P <= N")
    V: list[list[int]] = [[] for _ in range(p_count)]
    for row, p in enumerate(labels):
        V[p].append(row)
    if any(len(v) == 0 for v in V):
        raise OracleError("a fold has no rows")
    return V


def bookkeeping(fold_id):
    """Flattened Algorithm 1: (P, counts[P], offsets[P+1], perm[N]) where
    perm[offsets[p]:offsets[p+1]] lists V_p in ascending row order."""
    V = validation_partitions(fold_id)
    counts = np.array([len(v) for v in V], dtype=np.int64)
    offsets = np.zeros(len(V) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    perm = np.array([r for v in V for r in v], dtype=np.int32)
    return len(V), counts, offsets, perm


def training_rows(fold_id, p: int) -> np.ndarray:
    """T_p = R minus V_p, ascending (Definition 1)."""
    f = np.asarray(fold_id).ravel()
    return np.nonzero(f != p)[0]


# ---------------------------------------------------------------------------
# Definitions 2-5 on a materialised block
# ---------------------------------------------------------------------------

def column_stats(A: np.ndarray, ddof: int):
    """Column mean (Definition 2) and deviation (Definition 4 with divisor
    |S| - ddof), computed two-pass in FP64, plus the constant-column mask.
    A constant column gets mean = its value and deviation 1."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    const = np.all(A == A[:1, :], axis=0) if n > 0 else np.ones(A.shape[1], bool)
    mean = A.sum(axis=0) / n
    mean = np.where(const, A[0, :] if n > 0 else 0.0, mean)
    dev = A - mean[None, :]
    if n - ddof >= 1:
        var = (dev * dev).sum(axis=0) / (n - ddof)
        std = np.sqrt(var)
    else:
        std = np.full(A.shape[1], np.nan)
    std = np.where(const, 1.0, std)
    return mean, std, const


def preprocess(A: np.ndarray, center: bool, scale: bool, ddof: int) -> np.ndarray:
    """Definitions 3 and 5: subtract the column means if ``center``; divide by
    the column deviations if ``scale`` (both over the rows of A)."""
    A = np.asarray(A, dtype=np.float64)
    if scale and A.shape[0] - ddof < 1:
        raise OracleError("scaling needs |T| - ddof >= 1")
    mean, std, _ = column_stats(A, ddof)
    out = A.copy()
    if center:
        out = out - mean[None, :]
    if scale:
        out = out / std[None, :]
    return out


# ---------------------------------------------------------------------------
# per-fold products (Algorithm 6 generalised)
# ---------------------------------------------------------------------------

def _check_scalable(fold_id, ddof: int, scaling: bool):
    V = validation_partitions(fold_id)
    n = len(np.asarray(fold_id).ravel())
    if ddof not in (0, 1):
        raise OracleError("ddof must be 0 or 1")
    if scaling:
        for v in V:
            if n - len(v) - ddof < 1:
                raise OracleError("partitioning is not scalable (Definition 6)")
    return V


def fold_products(X, Y, fold_id, p: int, cx: int, sx: int, cy: int, sy: int, ddof: int = 1):
    """Preprocessed training products for fold p and one combination:
    materialise X_T, Y_T; centre/scale with training statistics; multiply."""
    _check_scalable(fold_id, ddof, bool(sx or sy))
    T = training_rows(fold_id, p)
    XT = np.asarray(X, dtype=np.float64)[T]
    YT = np.asarray(Y, dtype=np.float64)[T]
    Xp = preprocess(XT, bool(cx), bool(sx), ddof)
    Yp = preprocess(YT, bool(cy), bool(sy), ddof)
    return Xp.T @ Xp, Xp.T @ Yp


def fold_all_classes(X, Y, fold_id, p: int, ddof: int = 1, scaling: bool = True):
    """All distinct products of fold p: XtX[4, K, K] indexed by ``xtx_class``
    and XtY[8, K, M] indexed by ``xty_class``.  With ``scaling`` False only the
    unscaled classes are filled (the rest are NaN)."""
    _check_scalable(fold_id, ddof, scaling)
    T = training_rows(fold_id, p)
    XT = np.asarray(X, dtype=np.float64)[T]
    YT = np.asarray(Y, dtype=np.float64)[T]
    K, M = XT.shape[1], YT.shape[1]
    xtx = np.full((4, K, K), np.nan)
    xty = np.full((8, K, M), np.nan)
    for c, (cx, sx, _, _) in XTX_CLASS_COMBO.items():
        if sx and not scaling:
            continue
        Xp = preprocess(XT, bool(cx), bool(sx), ddof)
        xtx[c] = Xp.T @ Xp
    for c, (cx, sx, cy, sy) in XTY_CLASS_COMBO.items():
        if (sx or sy) and not scaling:
            continue
        Xp = preprocess(XT, bool(cx), bool(sx), ddof)
        Yp = preprocess(YT, bool(cy), bool(sy), ddof)
        xty[c] = Xp.T @ Yp
    return xtx, xty


def fold_entries(X, Y, fold_id, p: int, cx: int, sx: int, cy: int, sy: int, ddof: int,
                 xx_pairs, xy_pairs):
    """Selected entries of fold p's products, each from the definition using
    only the columns it needs.  ``xx_pairs``/``xy_pairs`` are sequences of
    (i, j); returns two FP64 arrays of the same lengths."""
    _check_scalable(fold_id, ddof, bool(sx or sy))
    T = training_rows(fold_id, p)
    X = np.asarray(X)
    Y = np.asarray(Y)
    cache_x: dict[int, np.ndarray] = {}
    cache_y: dict[int, np.ndarray] = {}

    def xcol(i):
        if i not in cache_x:
            col = np.asarray(X[T, i], dtype=np.float64)[:, None]
            cache_x[i] = preprocess(col, bool(cx), bool(sx), ddof)[:, 0]
        return cache_x[i]

    def ycol(j):
        if j not in cache_y:
            col = np.asarray(Y[T, j], dtype=np.float64)[:, None]
            cache_y[j] = preprocess(col, bool(cy), bool(sy), ddof)[:, 0]
        return cache_y[j]

    xx = np.array([float(xcol(i) @ xcol(j)) for i, j in xx_pairs], dtype=np.float64)
    xy = np.array([float(xcol(i) @ ycol(j)) for i, j in xy_pairs], dtype=np.float64)
    return xx, xy


def fold_train_stats(X, Y, fold_id, p: int, ddof: int = 1):
    """Training-partition means and deviations of fold p (Definitions 2 and 4,
    deviation 1 for a column constant over T)."""
    T = training_rows(fold_id, p)
    mx, sx, _ = column_stats(np.asarray(X, dtype=np.float64)[T], ddof)
    my, sy, _ = column_stats(np.asarray(Y, dtype=np.float64)[T], ddof)
    return mx, sx, my, sy


# ---------------------------------------------------------------------------
# leaky comparison modes (Section 4.1): NOT training-partition preprocessing
# ---------------------------------------------------------------------------

def leaky_global_fold(X, Y, fold_id, p: int, cx: int, sx: int, cy: int, sy: int, ddof: int = 1):
    """Fold p's training products when X and Y are centred and/or scaled once
    with the statistics of ALL rows (the "centred and scaled over the entire
    data set initially" approach the paper's introduction warns about): the
    validation rows leak into the preprocessing.  Centering and scaling of X
    and of Y are independent here (Lemma 9's equivalence needs statistics of
    the same rows as the product).  A column constant over all rows gets
    deviation 1 and a centred column of exact zeros, as in ``column_stats``."""
    validation_partitions(fold_id)
    if ddof not in (0, 1):
        raise OracleError("ddof must be 0 or 1")
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    if (sx or sy) and X.shape[0] - ddof < 1:
        raise OracleError("scaling needs N - ddof >= 1")
    Xg = preprocess(X, bool(cx), bool(sx), ddof)
    Yg = preprocess(Y, bool(cy), bool(sy), ddof)
    T = training_rows(fold_id, p)
    return Xg[T].T @ Xg[T], Xg[T].T @ Yg[T]


def leaky_lindgren_fold(X, Y, fold_id, p: int):
    """Lindgren et al.'s centred training products for fold p, their
    Equation (20) as restated in the proof of Lemma 11:
        (X^T X)_ij - (X_V^T X_V)_ij - xbar_i sum_V X_nj - xbar_j sum_V X_ni
        + (N / P) xbar_i xbar_j
    with xbar the mean over ALL rows (leaks, Lemma 11).  X^T Y is read the same
    way with Y's mean and validation sums on the Y side."""
    V = validation_partitions(fold_id)
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    N, P = X.shape[0], len(V)
    v = np.asarray(V[p], dtype=np.int64)
    xbar = X.sum(axis=0) / N
    ybar = Y.sum(axis=0) / N if Y.shape[1] else np.zeros(0)
    sx_v = X[v].sum(axis=0)
    sy_v = Y[v].sum(axis=0)
    xtx = (X.T @ X - X[v].T @ X[v] - np.outer(xbar, sx_v) - np.outer(sx_v, xbar)
           + (N / P) * np.outer(xbar, xbar))
    xty = (X.T @ Y - X[v].T @ Y[v] - np.outer(xbar, sy_v) - np.outer(sx_v, ybar)
           + (N / P) * np.outer(xbar, ybar))
    return xtx, xty


# ---------------------------------------------------------------------------
# a consumer of the products: ridge regression per fold (Section 1 names RR
# and OLS among the models that use X^T X and X^T Y)
# ---------------------------------------------------------------------------

def ridge_fold(X, Y, fold_id, p: int, cx: int, sx: int, cy: int, sy: int, ddof: int, lam: float):
    """B = (X^T X_T + lam I)^{-1} X^T Y_T for fold p and one combination, from
    the definitional products (``fold_products``) and a dense solve."""
    xtx, xty = fold_products(X, Y, fold_id, p, cx, sx, cy, sy, ddof)
    return np.linalg.solve(xtx + lam * np.eye(xtx.shape[0]), xty)
