"""Pins of the FP64 oracle against facts fixed by the paper and by
mathematics, not against itself.

* exact brute force on tiny integer inputs (every fold, all 16
  combinations, ddof 0 and 1, constant columns included);
* a hand-derived worked example (tests/golden/hand_worked.json);
* library special cases: the centred product over |T|-ddof is numpy's
  covariance, the centred-and-scaled one is (|T|-ddof) times numpy's
  correlation;
* the paper's claims: Lemma 9 / Section 6 (16 combinations -> 4 distinct
  X^T X, 8 distinct X^T Y, 12 distinct pairs), Lemma 11 (Lindgren's
  centering leaks: it differs from training-partition centering by
  N * xbar_i * xbar_j * (2 - 1/P) when the training columns are centred);
* invariants: symmetry, zero column sums of centred training data, unit
  diagonal of the correlation form, metamorphic shifts/scalings, fold
  bookkeeping equal to a stable sort.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

from oracle import cv_oracle as O
from oracle import fast_cpu
from tests.exact_ref import exact_fold, exact_stats

HERE = os.path.dirname(os.path.abspath(__file__))


def _close(a, b, rtol=1e-12):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = max(1.0, float(np.max(np.abs(b))) if b.size else 1.0)
    return np.allclose(a, b, rtol=rtol, atol=rtol * scale)


# ---------------------------------------------------------------------------
# exact brute force
# ---------------------------------------------------------------------------

def _tiny_cases():
    rng = np.random.default_rng(20240113)
    cases = []
    for trial in range(36):
        n = int(rng.integers(4, 11))
        k = int(rng.integers(1, 5))
        m = int(rng.integers(1, 4))
        p = int(rng.integers(2, max(3, n - 1)))
        X = rng.integers(-6, 7, size=(n, k))
        Y = rng.integers(-6, 7, size=(n, m))
        if trial % 3 == 0:
            X[:, 0] = 3                      # constant everywhere
        if trial % 4 == 1 and k > 1:
            X[: n // 2, k - 1] = -2          # constant over some training sets
        fold = np.concatenate([np.arange(p), rng.integers(0, p, size=n - p)])
        rng.shuffle(fold)
        cases.append((X.tolist(), Y.tolist(), fold.astype(np.int32)))
    return cases


@pytest.mark.parametrize("case", range(36))
def test_oracle_matches_exact_bruteforce(case):
    X, Y, fold = _tiny_cases()[case]
    n = len(fold)
    P = int(fold.max()) + 1
    sizes = np.bincount(fold, minlength=P)
    for ddof in (0, 1):
        scalable = all(n - s - ddof >= 1 for s in sizes)
        for combo in O.COMBOS:
            cx, sx, cy, sy = combo
            if (sx or sy) and not scalable:
                with pytest.raises(O.OracleError):
                    O.fold_products(X, Y, fold, 0, *combo, ddof=ddof)
                continue
            for p in range(P):
                got_xx, got_xy = O.fold_products(X, Y, fold, p, *combo, ddof=ddof)
                ex_xx, ex_xy = exact_fold(X, Y, fold.tolist(), p, *combo, ddof)
                assert _close(got_xx, ex_xx, 1e-13), (case, combo, ddof, p)
                assert _close(got_xy, ex_xy, 1e-13), (case, combo, ddof, p)


def test_train_stats_match_exact():
    for X, Y, fold in _tiny_cases()[:12]:
        P = int(fold.max()) + 1
        for p in range(P):
            rows = [r for r in range(len(fold)) if fold[r] != p]
            if len(rows) < 2:
                continue
            mx, sx, my, sy = O.fold_train_stats(X, Y, fold, p, ddof=1)
            em, es = exact_stats(X, rows, 1)
            assert _close(mx, em) and _close(sx, es)
            em, es = exact_stats(Y, rows, 1)
            assert _close(my, em) and _close(sy, es)


# ---------------------------------------------------------------------------
# hand-derived worked example
# ---------------------------------------------------------------------------

def _eval_expr(expr: str) -> float:
    s = math.sqrt(7.0 / 3.0)
    return float(eval(expr, {"__builtins__": {}}, {"sqrt": math.sqrt, "s": s}))


def test_hand_worked_example():
    g = json.load(open(os.path.join(HERE, "golden", "hand_worked.json")))
    X, Y, fold, ddof = g["X"], g["Y"], np.array(g["fold_id"], np.int32), g["ddof"]
    for p_str, f in g["folds"].items():
        p = int(p_str)
        assert O.training_rows(fold, p).tolist() == f["training_rows"]
        xtx, xty = O.fold_all_classes(X, Y, fold, p, ddof=ddof)
        exp_xtx = np.vectorize(_eval_expr)(np.array(f["xtx"], dtype=object)).astype(float)
        exp_xty = np.vectorize(_eval_expr)(np.array(f["xty"], dtype=object)).astype(float)
        assert _close(xtx, exp_xtx, 1e-14), p
        assert _close(xty, exp_xty, 1e-14), p
        mx, sx, my, sy = O.fold_train_stats(X, Y, fold, p, ddof)
        assert _close(mx, [_eval_expr(e) for e in f["mean_x"]])
        assert _close(sx, [_eval_expr(e) for e in f["std_x"]])
        assert _close(my, [_eval_expr(e) for e in f["mean_y"]])
        assert _close(sy, [_eval_expr(e) for e in f["std_y"]])


# ---------------------------------------------------------------------------
# library special cases and invariants on random float data
# ---------------------------------------------------------------------------

def _float_case(seed=7, n=120, k=9, m=4, P=6):
    rng = np.random.default_rng(seed)
    X = 3.0 + rng.standard_normal((n, k)) * rng.uniform(0.2, 3, size=k)
    Y = -2.0 + X[:, :m] * 0.5 + rng.standard_normal((n, m))
    fold = rng.integers(0, P, size=n).astype(np.int32)
    fold[:P] = np.arange(P)
    return X, Y, fold


@pytest.mark.parametrize("ddof", [0, 1])
def test_covariance_and_correlation_special_cases(ddof):
    X, Y, fold = _float_case()
    P = int(fold.max()) + 1
    for p in range(P):
        T = fold != p
        nt = int(T.sum())
        xtx, xty = O.fold_all_classes(X, Y, fold, p, ddof=ddof)
        Z = np.concatenate([X[T], Y[T]], axis=1)
        cov = np.cov(Z, rowvar=False, ddof=ddof)
        cor = np.corrcoef(Z, rowvar=False)
        K = X.shape[1]
        assert _close(xtx[2] / (nt - ddof), cov[:K, :K])
        assert _close(xty[4] / (nt - ddof), cov[:K, K:])
        assert _close(xtx[3] / (nt - ddof), cor[:K, :K])
        assert _close(xty[7] / (nt - ddof), cor[:K, K:])
        # raw product is the plain training product
        assert _close(xtx[0], X[T].T @ X[T]) and _close(xty[0], X[T].T @ Y[T])
        # scaled-only: the raw product over the outer product of deviations
        sdx = np.std(X[T], axis=0, ddof=ddof)
        sdy = np.std(Y[T], axis=0, ddof=ddof)
        assert _close(xtx[1], (X[T].T @ X[T]) / np.outer(sdx, sdx))
        assert _close(xty[1], (X[T].T @ Y[T]) / sdy[None, :])
        assert _close(xty[2], (X[T].T @ Y[T]) / sdx[:, None])


def test_invariants_symmetry_zero_sums_unit_diagonal():
    X, Y, fold = _float_case(seed=11)
    for p in range(int(fold.max()) + 1):
        T = O.training_rows(fold, p)
        xtx, _ = O.fold_all_classes(X, Y, fold, p, ddof=1)
        for c in range(4):
            assert np.array_equal(xtx[c], xtx[c].T) or _close(xtx[c], xtx[c].T, 1e-14)
        Xc = O.preprocess(X[T], True, False, 1)
        assert np.all(np.abs(Xc.sum(axis=0)) <= 64 * len(T) * 2.2e-16 * np.abs(X[T]).max())
        assert _close(np.diag(xtx[3]), np.full(X.shape[1], len(T) - 1.0))
        assert np.all(np.abs(xtx[3]) <= len(T) - 1 + 1e-9)


def test_16_combinations_give_12_distinct_pairs():
    """Section 6: X^T X has 4 distinct forms, X^T Y 8, the pairs 12; centering
    X, Y or both gives the same X^T Y (Lemma 9); centering only Y is not the
    same pair as centering both."""
    X, Y, fold = _float_case(seed=3, n=60, k=5, m=3, P=4)
    res = {c: O.fold_products(X, Y, fold, 1, *c, ddof=1) for c in O.COMBOS}

    def same(a, b):
        return _close(a, b, 1e-12)

    pair_classes: list[list[tuple]] = []
    for c in O.COMBOS:
        for cls in pair_classes:
            r = res[cls[0]]
            if same(r[0], res[c][0]) and same(r[1], res[c][1]):
                cls.append(c)
                break
        else:
            pair_classes.append([c])
    assert len(pair_classes) == 12
    xtx_classes = {O.xtx_class(*c) for c in O.COMBOS}
    xty_classes = {O.xty_class(*c) for c in O.COMBOS}
    assert len(xtx_classes) == 4 and len(xty_classes) == 8
    for cls in pair_classes:
        # members of one class share (xtx_class, xty_class)
        assert len({(O.xtx_class(*c), O.xty_class(*c)) for c in cls}) == 1
    for sx in (0, 1):
        for sy in (0, 1):
            a = res[(1, sx, 0, sy)]
            b = res[(1, sx, 1, sy)]
            assert same(a[0], b[0]) and same(a[1], b[1])
            c = res[(0, sx, 1, sy)]
            assert same(c[1], b[1]) and not same(c[0], b[0])


def test_lindgren_centering_leaks_lemma11():
    """Lemma 11: with balanced folds, if fold p's training columns are exactly
    centred but the full-data means are not zero, Lindgren et al.'s Eq. (20)
    differs from training-partition centering by N xbar_i xbar_j (2 - 1/P)."""
    P, per = 4, 6
    N = P * per
    rng = np.random.default_rng(5)
    K = 3
    fold = np.repeat(np.arange(P), per).astype(np.int32)
    X = rng.integers(-5, 6, size=(N, K)).astype(float)
    p = 2
    T = fold != p
    X[T] -= X[T].mean(axis=0)                     # centre the training rows
    X[~T] += 4.0 + np.arange(K)                   # keep the full mean nonzero
    xbar = X.mean(axis=0)
    assert np.all(np.abs(xbar) > 0.1)
    V = ~T
    xtx_full = X.T @ X
    xtx_v = X[V].T @ X[V]
    sumV = X[V].sum(axis=0)
    lind = xtx_full - xtx_v - np.outer(xbar, sumV) - np.outer(sumV, xbar) + (N / P) * np.outer(xbar, xbar)
    ours = O.fold_products(X, np.zeros((N, 1)), fold, p, 1, 0, 1, 0, ddof=1)[0]
    assert _close(ours, X[T].T @ X[T])            # training columns already centred
    assert _close(lind - ours, -N * np.outer(xbar, xbar) * (2 - 1 / P))
    assert np.max(np.abs(lind - ours)) > 1.0
    # centering with full-data statistics is also not the training-partition result
    glob = (X[T] - xbar).T @ (X[T] - xbar)
    assert not _close(glob, ours, 1e-6)


def test_metamorphic_shift_scale_permute_relabel():
    X, Y, fold = _float_case(seed=21, n=90, k=6, m=2, P=5)
    rng = np.random.default_rng(1)
    shift = rng.uniform(-50, 50, size=X.shape[1])
    scale = rng.uniform(0.1, 10, size=X.shape[1])
    for p in (0, 3):
        base = O.fold_all_classes(X, Y, fold, p, ddof=1)
        sh = O.fold_all_classes(X + shift, Y, fold, p, ddof=1)
        for c in (2, 3):
            assert _close(sh[0][c], base[0][c], 1e-10)
        for c in (4, 5, 6, 7):
            assert _close(sh[1][c], base[1][c], 1e-10)
        sc = O.fold_all_classes(X * scale, Y, fold, p, ddof=1)
        assert _close(sc[0][3], base[0][3], 1e-12) and _close(sc[1][7], base[1][7], 1e-12)
        assert _close(sc[0][1], base[0][1], 1e-12)
        # row permutation (labels travel with rows) changes nothing
        perm = rng.permutation(len(fold))
        pr = O.fold_all_classes(X[perm], Y[perm], fold[perm], p, ddof=1)
        assert _close(pr[0], base[0], 1e-12) and _close(pr[1], base[1], 1e-12)
        # duplicated column -> duplicated row and column
        X2 = np.concatenate([X, X[:, :1]], axis=1)
        d = O.fold_all_classes(X2, Y, fold, p, ddof=1)
        assert _close(d[0][:, -1, :-1], base[0][:, 0, :], 1e-12)
        assert _close(d[0][:, :-1, :-1], base[0], 1e-12)
    # relabelling folds permutes the per-fold results
    relabel = np.array([4, 2, 0, 1, 3], dtype=np.int32)
    f2 = relabel[fold]
    for p in range(5):
        a = O.fold_all_classes(X, Y, fold, p, ddof=1)
        b = O.fold_all_classes(X, Y, f2, int(relabel[p]), ddof=1)
        assert _close(a[0], b[0], 0) and _close(a[1], b[1], 0)


def test_leave_one_out_single_row_validation():
    """P = N: the validation product of fold p is the outer product of row p
    (Lemma 2 with |V| = 1)."""
    rng = np.random.default_rng(2)
    N, K = 7, 3
    X = rng.standard_normal((N, K))
    Y = rng.standard_normal((N, 2))
    fold = np.arange(N, dtype=np.int32)
    for p in range(N):
        xtx, xty = O.fold_products(X, Y, fold, p, 0, 0, 0, 0, ddof=1)
        assert _close(X.T @ X - xtx, np.outer(X[p], X[p]))
        assert _close(X.T @ Y - xty, np.outer(X[p], Y[p]))


# ---------------------------------------------------------------------------
# Algorithm 1 bookkeeping and Definition 1 errors
# ---------------------------------------------------------------------------

def test_bookkeeping_is_a_stable_sort():
    rng = np.random.default_rng(9)
    for n, P in ((10, 2), (1000, 7), (5000, 300), (64, 64)):
        fold = np.concatenate([np.arange(P), rng.integers(0, P, size=n - P)]).astype(np.int32)
        rng.shuffle(fold)
        Pn, counts, offsets, perm = O.bookkeeping(fold)
        assert Pn == P
        assert np.array_equal(perm, np.argsort(fold, kind="stable").astype(np.int32))
        assert np.array_equal(counts, np.bincount(fold, minlength=P))
        assert offsets[-1] == n and counts.sum() == n
        assert (n * (P - 1)) == sum(n - c for c in counts)        # Lemma 6
        for p in range(P):                                       # Lemma 1
            seg = perm[offsets[p]:offsets[p + 1]]
            assert np.all(fold[seg] == p) and np.all(np.diff(seg) > 0)


@pytest.mark.parametrize("bad", [
    [0, 0, 0],            # P = 1
    [0, 2, 2, 0],         # label 1 unused
    [0, -1, 1],           # negative label
    [0, 1, 2, 3, 4, 9],   # P > N
])
def test_definition1_violations_raise(bad):
    with pytest.raises(O.OracleError):
        O.bookkeeping(np.array(bad, dtype=np.int32))


def test_non_scalable_partitioning_raises_only_when_scaling():
    X = np.arange(8, dtype=float).reshape(4, 2)
    Y = np.ones((4, 1))
    fold = np.array([0, 0, 0, 1], dtype=np.int32)     # |T_0| = 1
    O.fold_products(X, Y, fold, 0, 1, 0, 1, 0, ddof=1)  # centering only: fine
    with pytest.raises(O.OracleError):
        O.fold_products(X, Y, fold, 0, 1, 1, 1, 1, ddof=1)
    O.fold_products(X, Y, fold, 0, 1, 1, 1, 1, ddof=0)  # |T| - ddof = 1


# ---------------------------------------------------------------------------
# the fast CPU algorithm agrees with the oracle (Proposition 17)
# ---------------------------------------------------------------------------

def test_fast_cpu_matches_oracle_small_workload():
    from synth import generators as G
    shape, (X, Y, fold) = G.workload(1)
    for ddof in (0, 1):
        for p, xtx, xty in fast_cpu.fast_all_folds(X, Y, fold, ddof=ddof):
            oxx, oxy = O.fold_all_classes(X, Y, fold, p, ddof=ddof)
            for c in range(4):
                err = np.linalg.norm(xtx[c] - oxx[c]) / np.linalg.norm(oxx[c])
                assert err < 1e-10, (p, c, err)
            for c in range(8):
                err = np.linalg.norm(xty[c] - oxy[c]) / np.linalg.norm(oxy[c])
                assert err < 1e-10, (p, c, err)


def test_fold_entries_match_full_products():
    X, Y, fold = _float_case(seed=4, n=80, k=7, m=3, P=4)
    pairs_xx = [(0, 0), (1, 5), (6, 2), (3, 3)]
    pairs_xy = [(0, 0), (6, 2), (4, 1)]
    for combo in O.COMBOS:
        xx, xy = O.fold_products(X, Y, fold, 2, *combo, ddof=1)
        ex, ey = O.fold_entries(X, Y, fold, 2, *combo, 1, pairs_xx, pairs_xy)
        assert _close(ex, [xx[i, j] for i, j in pairs_xx], 1e-12)
        assert _close(ey, [xy[i, j] for i, j in pairs_xy], 1e-12)


# ---------------------------------------------------------------------------
# leaky comparison modes (Section 4.1)
# ---------------------------------------------------------------------------

def test_leaky_lindgren_matches_lemma11_closed_form():
    """The oracle's Eq. (20) form equals Lemma 11's simplified form
    (X_T^T X_T)_ij - N xbar_i xbar_j (2 - 1/P) + |T| xbar_i xbarT_j
    + |T| xbar_j xbarT_i on uneven folds, and both leak."""
    rng = np.random.default_rng(17)
    N, K, M, P = 37, 4, 2, 5
    X = rng.normal(3.0, 1.5, size=(N, K))
    Y = rng.normal(-2.0, 0.7, size=(N, M))
    fold = rng.integers(0, P, size=N).astype(np.int32)
    fold[:P] = np.arange(P)
    for p in range(P):
        lx, ly = O.leaky_lindgren_fold(X, Y, fold, p)
        T = fold != p
        nt = int(T.sum())
        xbar, ybar = X.mean(axis=0), Y.mean(axis=0)
        xbt, ybt = X[T].mean(axis=0), Y[T].mean(axis=0)
        lemma_xx = (X[T].T @ X[T] - N * np.outer(xbar, xbar) * (2 - 1 / P)
                    + nt * np.outer(xbar, xbt) + nt * np.outer(xbt, xbar))
        lemma_xy = (X[T].T @ Y[T] - N * np.outer(xbar, ybar) * (2 - 1 / P)
                    + nt * np.outer(xbar, ybt) + nt * np.outer(xbt, ybar))
        assert _close(lx, lemma_xx) and _close(ly, lemma_xy)
        ours = O.fold_products(X, Y, fold, p, 1, 0, 1, 0, ddof=1)
        assert not _close(lx, ours[0], 1e-6)


def test_leaky_global_parallel_axis_identity():
    """Centering the training rows with the all-row mean xbar instead of
    their own mean xbarT adds |T| (xbarT - xbar)(xbarT - xbar)^T (and the
    matching cross term for X^T Y): the textbook parallel-axis identity.
    Scaling with all-row deviations divides by their outer product."""
    rng = np.random.default_rng(23)
    N, K, M, P = 29, 3, 2, 4
    X = rng.normal(1.0, 2.0, size=(N, K))
    Y = rng.normal(0.5, 1.0, size=(N, M))
    fold = np.arange(N, dtype=np.int32) % P
    for p in range(P):
        T = fold != p
        nt = int(T.sum())
        dx = X[T].mean(axis=0) - X.mean(axis=0)
        dy = Y[T].mean(axis=0) - Y.mean(axis=0)
        gx, gy = O.leaky_global_fold(X, Y, fold, p, 1, 0, 1, 0, ddof=1)
        tx, ty = O.fold_products(X, Y, fold, p, 1, 0, 1, 0, ddof=1)
        assert _close(gx, tx + nt * np.outer(dx, dx))
        assert _close(gy, ty + nt * np.outer(dx, dy))
        # X centred only: (X_T - xbar)^T Y_T = X_T^T Y_T - xbar sumT(Y)
        gx1, gy1 = O.leaky_global_fold(X, Y, fold, p, 1, 0, 0, 0, ddof=1)
        assert _close(gy1, X[T].T @ Y[T] - np.outer(X.mean(axis=0), Y[T].sum(axis=0)))
        # scaled with all-row deviations
        sx = X.std(axis=0, ddof=1)
        sy = Y.std(axis=0, ddof=1)
        gxs, gys = O.leaky_global_fold(X, Y, fold, p, 1, 1, 1, 1, ddof=1)
        assert _close(gxs, gx / np.outer(sx, sx)) and _close(gys, gy / np.outer(sx, sy))
        assert not _close(gxs, O.fold_products(X, Y, fold, p, 1, 1, 1, 1, ddof=1)[0], 1e-6)


def test_leaky_global_constant_column():
    """A column constant over all rows: deviation 1, centred column exactly 0."""
    rng = np.random.default_rng(3)
    N, P = 20, 4
    X = rng.normal(size=(N, 3))
    X[:, 1] = 7.25
    Y = rng.normal(size=(N, 1))
    fold = np.arange(N, dtype=np.int32) % P
    gx, gy = O.leaky_global_fold(X, Y, fold, 0, 1, 1, 1, 1, ddof=1)
    assert np.all(gx[1] == 0.0) and np.all(gx[:, 1] == 0.0) and np.all(gy[1] == 0.0)
    gx, _ = O.leaky_global_fold(X, Y, fold, 0, 0, 1, 0, 0, ddof=1)
    T = fold != 0
    assert _close(gx[1, 1], (X[T, 1] ** 2).sum())


# ---------------------------------------------------------------------------
# ridge regression consumer
# ---------------------------------------------------------------------------

def test_ridge_fold_equals_augmented_least_squares():
    """Ridge is least squares on the training rows stacked over sqrt(lam) I
    (a textbook identity), solved here by the SVD-based lstsq on the
    preprocessed training data, not through the products; lam = 0 is OLS."""
    rng = np.random.default_rng(31)
    N, K, M, P = 60, 5, 2, 4
    X = rng.normal(2.0, 1.0, size=(N, K))
    Y = X @ rng.normal(size=(K, M)) + rng.normal(0, 0.3, size=(N, M))
    fold = np.arange(N, dtype=np.int32) % P
    for combo in [(0, 0, 0, 0), (1, 0, 1, 0), (1, 1, 1, 1), (0, 1, 0, 1)]:
        for p in range(P):
            T = O.training_rows(fold, p)
            Xt = O.preprocess(X[T], bool(combo[0]), bool(combo[1]), 1)
            Yt = O.preprocess(Y[T], bool(combo[2]), bool(combo[3]), 1)
            for lam in (0.0, 0.5, 7.0):
                B = O.ridge_fold(X, Y, fold, p, *combo, 1, lam)
                Xa = np.vstack([Xt, np.sqrt(lam) * np.eye(K)])
                Ya = np.vstack([Yt, np.zeros((K, M))])
                ref = np.linalg.lstsq(Xa, Ya, rcond=None)[0]
                assert _close(B, ref, 1e-9), (combo, p, lam)
