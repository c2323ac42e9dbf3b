"""Planted mistakes in the oracle, on the CPU.

Each mutation below is a plausible slip in writing the paper's definitions
down: a wrong divisor, a variance used as a deviation, the constant-column
rule dropped, statistics or products over the wrong rows, a wrong sign, a
dropped centering term, an index reversed, an unstable row order.  The pin
battery is made of facts that do not come from the oracle's own formulas:
exact brute force in rationals (tests/exact_ref.py), the hand-derived worked
example (tests/golden/hand_worked.json), numpy's covariance and correlation,
the plain training-row product, and the bookkeeping as a stable sort.  The
battery must accept the oracle as written and reject every mutation.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

from oracle import cv_oracle as O
from tests.exact_ref import exact_fold

HERE = os.path.dirname(os.path.abspath(__file__))
COMBOS = [(cx, sx, cy, sy) for cx in (0, 1) for sx in (0, 1) for cy in (0, 1) for sy in (0, 1)]


def _close(a, b, tol=1e-12):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.shape != b.shape or not np.all(np.isfinite(a)):
        return False
    return bool(np.max(np.abs(a - b)) <= tol * max(1.0, float(np.max(np.abs(b)))))


def _eval_expr(e):
    # golden entries are closed-form expressions; 's' abbreviates sqrt(7/3)
    return float(eval(e, {"__builtins__": {}}, {"sqrt": math.sqrt, "s": math.sqrt(7.0 / 3.0)}))


def battery() -> list[str]:
    """Names of the pins that fail (an exception inside a check counts as a
    failure: a mutated oracle may also break outright)."""
    failed: list[str] = []

    def check(name, fn):
        try:
            if not fn():
                failed.append(name)
        except Exception:  # noqa: BLE001 - any breakage is a detection
            failed.append(name)

    # exact brute force: small integers, uneven folds, a column constant over
    # the training rows of fold 0 and one constant over every row
    X = [[1, 4, 7, 2], [3, 4, 1, 2], [2, 5, 0, 2], [5, 4, 3, 2], [0, 6, 2, 2], [4, 1, 5, 2],
         [6, 3, 1, 2], [1, 2, 8, 2], [2, 7, 4, 2], [3, 3, 3, 2]]
    Y = [[1, 0], [2, 1], [0, 3], [4, 1], [3, 2], [1, 5], [2, 2], [0, 1], [5, 0], [2, 3]]
    fold = np.array([0, 1, 1, 2, 0, 2, 1, 0, 2, 1], dtype=np.int32)
    X[0][1] = X[4][1] = X[7][1] = 9  # column 1 varies only inside fold 0's training rows

    def brute():
        for p in range(3):
            for ddof in (0, 1):
                for combo in COMBOS:
                    exx, exy = exact_fold(X, Y, fold.tolist(), p, *combo, ddof)
                    gxx, gxy = O.fold_products(X, Y, fold, p, *combo, ddof=ddof)
                    if not (_close(gxx, exx) and _close(gxy, exy)):
                        return False
        return True
    check("exact brute force", brute)

    # hand-derived worked example
    def golden():
        g = json.load(open(os.path.join(HERE, "golden", "hand_worked.json")))
        gf = np.array(g["fold_id"], np.int32)
        for p_str, f in g["folds"].items():
            xtx, xty = O.fold_all_classes(g["X"], g["Y"], gf, int(p_str), ddof=g["ddof"])
            ex = np.vectorize(_eval_expr)(np.array(f["xtx"], dtype=object)).astype(float)
            ey = np.vectorize(_eval_expr)(np.array(f["xty"], dtype=object)).astype(float)
            if not (_close(xtx, ex, 1e-13) and _close(xty, ey, 1e-13)):
                return False
        return True
    check("worked example", golden)

    # library special cases on real-valued data
    rng = np.random.default_rng(7)
    Xr = rng.normal(3.0, 2.0, size=(40, 5))
    Yr = rng.normal(-1.0, 1.5, size=(40, 3))
    fr = (np.arange(40) % 4).astype(np.int32)
    rng.shuffle(fr)

    def cov():
        for p in range(4):
            T = fr != p
            for ddof in (0, 1):
                xx, _ = O.fold_products(Xr, Yr, fr, p, 1, 0, 1, 0, ddof=ddof)
                if not _close(xx / (T.sum() - ddof), np.cov(Xr[T], rowvar=False, ddof=ddof)):
                    return False
        return True
    check("numpy covariance", cov)

    def corr():
        for p in range(4):
            T = fr != p
            xx, _ = O.fold_products(Xr, Yr, fr, p, 1, 1, 1, 1, ddof=1)
            if not _close(xx / (T.sum() - 1), np.corrcoef(Xr[T], rowvar=False)):
                return False
        return True
    check("numpy correlation", corr)

    def raw_and_scaled():
        for p in range(4):
            T = fr != p
            xx, xy = O.fold_products(Xr, Yr, fr, p, 0, 0, 0, 0, ddof=1)
            if not (_close(xx, Xr[T].T @ Xr[T]) and _close(xy, Xr[T].T @ Yr[T])):
                return False
            sxx, sxy = O.fold_products(Xr, Yr, fr, p, 0, 1, 0, 1, ddof=1)
            sx = Xr[T].std(axis=0, ddof=1)
            sy = Yr[T].std(axis=0, ddof=1)
            if not (_close(sxx, xx / np.outer(sx, sx)) and _close(sxy, xy / np.outer(sx, sy))):
                return False
        return True
    check("raw and scaled-only products", raw_and_scaled)

    def xty_centred():
        # centering X alone centres X^T Y: column sums of the centred
        # training rows vanish (Lemma 9), whatever Y is
        for p in range(4):
            T = fr != p
            _, xy = O.fold_products(Xr, Yr, fr, p, 1, 0, 0, 0, ddof=1)
            Xc = Xr[T] - Xr[T].mean(axis=0)
            if not _close(xy, Xc.T @ Yr[T]):
                return False
            _, xy2 = O.fold_products(Xr, Yr, fr, p, 0, 0, 1, 0, ddof=1)
            Yc = Yr[T] - Yr[T].mean(axis=0)
            if not _close(xy2, Xr[T].T @ Yc):
                return False
        return True
    check("centred cross products", xty_centred)

    def bookkeeping():
        P, counts, offsets, perm = O.bookkeeping(fr)
        return (P == 4 and np.array_equal(perm, np.argsort(fr, kind="stable"))
                and np.array_equal(counts, np.bincount(fr)))
    check("stable bookkeeping", bookkeeping)
    return failed


# ---------------------------------------------------------------------------
# mutations (each patches one oracle function for the duration of a test)
# ---------------------------------------------------------------------------

_orig_stats = O.column_stats
_orig_prep = O.preprocess
_orig_rows = O.training_rows
_orig_parts = O.validation_partitions


def _stats_ddof_ignored(A, ddof):
    return _orig_stats(A, 0)


def _stats_variance(A, ddof):
    mean, std, const = _orig_stats(A, ddof)
    return mean, np.where(const, 1.0, std * std), const


def _stats_no_constant_rule(A, ddof):
    mean, std, const = _orig_stats(A, ddof)
    A = np.asarray(A, dtype=np.float64)
    plain = np.sqrt(((A - A.mean(axis=0)) ** 2).sum(axis=0) / (A.shape[0] - ddof))
    return mean, plain, const


def _stats_mean_divisor(A, ddof):
    mean, std, const = _orig_stats(A, ddof)
    A = np.asarray(A, dtype=np.float64)
    return np.where(const, mean, A.sum(axis=0) / (A.shape[0] - 1)), std, const


def _rows_all(fold_id, p):
    return np.arange(np.asarray(fold_id).size)


def _rows_validation(fold_id, p):
    return np.nonzero(np.asarray(fold_id).ravel() == p)[0]


def _prep_wrong_sign(A, center, scale, ddof):
    A = np.asarray(A, dtype=np.float64)
    mean, std, _ = O.column_stats(A, ddof)
    out = A + mean[None, :] if center else A.copy()
    return out / std[None, :] if scale else out


def _prep_no_centering(A, center, scale, ddof):
    return _orig_prep(A, False, scale, ddof)


def _prep_reversed_columns(A, center, scale, ddof):
    out = _orig_prep(A, center, scale, ddof)
    A = np.asarray(A, dtype=np.float64)
    if A.shape[1] > 1 and scale:
        # deviations of the columns in reverse order (an index slip)
        _, std, _ = O.column_stats(A, ddof)
        out = out * std[None, :] / std[None, ::-1]
    return out


def _parts_reversed(fold_id):
    return [list(reversed(v)) for v in _orig_parts(fold_id)]


MUTATIONS = {
    "ddof ignored": ("column_stats", _stats_ddof_ignored),
    "variance used as deviation": ("column_stats", _stats_variance),
    "constant-column rule dropped": ("column_stats", _stats_no_constant_rule),
    "mean divided by n - 1": ("column_stats", _stats_mean_divisor),
    "statistics and products over all rows": ("training_rows", _rows_all),
    "validation rows used as training rows": ("training_rows", _rows_validation),
    "mean added instead of subtracted": ("preprocess", _prep_wrong_sign),
    "centering dropped": ("preprocess", _prep_no_centering),
    "deviations of the wrong columns": ("preprocess", _prep_reversed_columns),
    "unstable row order in the bookkeeping": ("validation_partitions", _parts_reversed),
}


def test_battery_accepts_the_oracle():
    assert battery() == []


@pytest.mark.filterwarnings("ignore::RuntimeWarning")  # some mutations divide by zero
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_battery_rejects_mutation(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(O, attr, fn)
    failed = battery()
    assert failed, f"mutation '{name}' passed every pin"
