"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bars: fold bookkeeping bit-exact; FP64-mode products within 1e-10 relative
Frobenius error per fold x class x output; training statistics within 1e-12;
X^T X bit-symmetric; equivalent combinations bit-identical; repeated runs
bit-identical.
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


def _dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    return torch.device("cuda:0")


def _t(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(_dev())


def _relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


def _check_all_folds(X, Y, fold, ddof, mode="fp64", tol=FP64_TOL, folds=None, label=""):
    print(f"[parity] {label} N={X.shape[0]} K={X.shape[1]} M={Y.shape[1]} ddof={ddof} mode={mode}",
          flush=True)
    Xd, Yd = _t(X), (_t(Y) if Y.shape[1] else None)
    fd = _t(fold.astype(np.int32))
    h = cv.cvgram_create(Xd, Yd, fd, 1, 1, 1, 1, ddof=ddof, mode=mode)
    P = cv.cvgram_num_folds(h)
    assert P == int(fold.max()) + 1
    if mode == "fp64":
        # FP32 input keeps FP32 panels up to K = 2048, FP64 panels otherwise
        f32_panels = X.dtype == np.float32 and X.shape[1] <= 2048
        assert cv.cvgram_plan_info(h)["panel_bytes"] == (4 if f32_panels else 8), label
    xx, xy = cv.cvgram_folds_all(h, 0, P)
    torch.cuda.synchronize()
    xx = xx.cpu().numpy()
    xy = xy.cpu().numpy() if xy is not None else np.zeros((P, 8, X.shape[1], 0))
    worst = 0.0
    for p in (range(P) if folds is None else folds):
        oxx, oxy = O.fold_all_classes(X, Y, fold, p, ddof=ddof)
        for c in range(4):
            e = _relerr(xx[p, c], oxx[c])
            worst = max(worst, e)
            assert e <= tol, (label, "XtX", p, c, e)
            assert np.array_equal(xx[p, c], xx[p, c].T), (label, "asymmetric", p, c)
        for c in range(8):
            if Y.shape[1] == 0:
                continue
            e = _relerr(xy[p, c], oxy[c])
            worst = max(worst, e)
            assert e <= tol, (label, "XtY", p, c, e)
    cv.cvgram_destroy(h)
    return worst


# ---------------------------------------------------------------------------
# fold bookkeeping (Algorithm 1) -- bit-exact
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,P,kind", [
    (10, 2, "random"), (1000, 5, "random"), (4097, 256, "random"), (4097, 257, "random"),
    (20000, 3000, "random"), (70000, 70000, "loo"), (5000, 7, "venetian"),
    (5000, 9, "contiguous"), (100003, 100, "dirichlet"),
])
def test_partition_bit_exact(n, P, kind):
    print(f"[partition] n={n} P={P} {kind}", flush=True)
    rng = np.random.default_rng(n + P)
    if kind == "random":
        fold = np.concatenate([np.arange(P), rng.integers(0, P, n - P)]).astype(np.int32)
        rng.shuffle(fold)
    elif kind == "loo":
        fold = rng.permutation(n).astype(np.int32)
    elif kind == "venetian":
        fold = G.folds_venetian(n, P)
    elif kind == "contiguous":
        fold = G.folds_contiguous(n, P)
    else:
        fold = G.folds_dirichlet(n, P, rng)
    X = rng.standard_normal((n, 1))
    h = cv.cvgram_create(_t(X), None, _t(fold), mode="fp64")
    perm, offs = cv.cvgram_partition(h)
    torch.cuda.synchronize()
    Pn, counts, offsets, operm = O.bookkeeping(fold)
    assert cv.cvgram_num_folds(h) == Pn
    assert np.array_equal(perm.cpu().numpy(), operm)
    assert np.array_equal(offs.cpu().numpy(), offsets)
    cv.cvgram_destroy(h)


# ---------------------------------------------------------------------------
# FP64 mode against the oracle, all folds and all 12 distinct classes
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ddof", [1, 0])
def test_fp64_gaussian_workload_all_classes(ddof):
    shape, (X, Y, fold) = G.workload(1)
    worst = _check_all_folds(X, Y, fold, ddof, label="gaussian N=1000 K=50 M=2 P=5")
    print(f"worst rel err {worst:.3e}")


@pytest.mark.parametrize("n,k,m,p,values,dtype", [
    (3001, 130, 5, 7, "spectra", "f64"),      # ragged in rows, tiles and folds
    (2500, 64, 16, 4, "offset", "f64"),       # exact tile multiple, large offsets
    (20000, 100, 3, 9, "offset", "f32"),      # FP32 input, FP64 arithmetic
    (777, 1, 1, 3, "gaussian", "f64"),        # K = 1
    (900, 33, 0, 6, "gaussian", "f64"),       # no Y
    (5000, 200, 40, 12, "spectra", "f64"),    # several XtY tiles
    (4000, 150, 24, 6, "spectra", "f64"),     # 16 < M <= 32: two XtY blocks per diagonal row
    (1500, 2100, 3, 3, "spectra", "f64"),     # 17 tile columns: tiles in 8 x 8 groups, dealt
                                              # round-robin over the XCDs; ragged last group
    (1500, 2048, 3, 3, "offset", "f32"),      # FP32 input: FP32 panels up to K = 2048 ...
    (1500, 2049, 3, 3, "offset", "f32"),      # ... FP64 panels beyond (pack, allocation and
                                              # Gram agree on the element type)
])
def test_fp64_ragged_shapes(n, k, m, p, values, dtype):
    shape = G.Shape(f"{values} N={n} K={k} M={m} P={p}", n, k, m, p, dtype, values, "dirichlet")
    X, Y, fold = G.make(shape, 900 + k, 0)
    _check_all_folds(X, Y, fold, 1, label=shape.name)


@pytest.mark.parametrize("n,k,m,p", [
    (4, 1, 1, 2),       # two folds of two rows: each training partition is two rows
    (5, 3, 2, 2),       # folds of 3 and 2 rows
    (9, 2, 1, 3),
    (65, 17, 3, 13),    # thirteen folds of five rows: the fold sums formed per fold
])
@pytest.mark.parametrize("ddof", [1, 0])
@pytest.mark.parametrize("mode", ["fp64", "bf16x3"])
def test_smallest_problems(n, k, m, p, ddof, mode):
    shape = G.Shape(f"gaussian N={n} K={k} M={m} P={p}", n, k, m, p, "f64", "gaussian",
                    "near_equal")
    X, Y, fold = G.make(shape, 950 + n, 0)
    if mode == "fp64":
        _check_all_folds(X, Y, fold, ddof, label=shape.name)
        return
    # BF16X3: a sum over a few rows does not average the split's rounding
    # out, so every entry is held to the split arithmetic's own bound
    # (tests/sampling.py: split_bf16_bound) instead of the relative
    # Frobenius bar of long sums
    from tests import sampling as S
    print(f"[parity] {shape.name} bf16x3 ddof={ddof}", flush=True)
    h = cv.cvgram_create(_t(X), _t(Y), _t(fold.astype(np.int32)), 1, 1, 1, 1, ddof=ddof,
                         mode=mode)
    xx, xy = cv.cvgram_folds_all(h, 0, p)
    torch.cuda.synchronize()
    xx, xy = xx.cpu().numpy(), xy.cpu().numpy()
    for q in range(p):
        oxx, oxy = O.fold_all_classes(X, Y, fold, q, ddof=ddof)
        bxx, bxy = S.split_bf16_bound(X, Y, fold, q, ddof=ddof)
        for c in range(4):
            assert np.all(np.abs(xx[q, c] - oxx[c]) <= bxx[c]), (shape.name, q, "XtX", c)
            assert np.array_equal(xx[q, c], xx[q, c].T)
        for c in range(8):
            assert np.all(np.abs(xy[q, c] - oxy[c]) <= bxy[c]), (shape.name, q, "XtY", c)
    cv.cvgram_destroy(h)


def test_fp64_constant_columns():
    rng = np.random.default_rng(3)
    n, k, m, P = 600, 70, 3, 5
    X = rng.standard_normal((n, k)) + 4.0
    Y = rng.standard_normal((n, m))
    fold = G.folds_near_equal(n, P, rng)
    X[:, 3] = 2.5                          # constant everywhere
    X[fold != 1, 10] = -7.0                # constant over T_1 only
    Y[:, 1] = 0.1                          # constant response
    Y[fold == 2, 2] = 1e3                  # wild values inside one fold only
    _check_all_folds(X, Y, fold, 1, label="constant columns")
    # centred products of a constant column are exactly zero
    h = cv.cvgram_create(_t(X), _t(Y), _t(fold), mode="fp64")
    xx, xy = cv.cvgram_folds_all(h, 0, P)
    xx = xx.cpu().numpy()
    xy = xy.cpu().numpy()
    assert np.all(xx[:, 2:, 3, :] == 0) and np.all(xx[:, 2:, :, 3] == 0)
    assert np.all(xx[1, 2:, 10, :] == 0)
    assert np.all(xy[:, 4:, :, 1] == 0)
    mx, sx, my, sy = cv.cvgram_fold_stats(h, 1)
    assert sx[3].item() == 1.0 and sx[10].item() == 1.0 and mx[10].item() == -7.0
    assert sy[1].item() == 1.0
    cv.cvgram_destroy(h)


def test_every_combination_and_equivalences_bit_identical():
    shape, (X, Y, fold) = G.workload(1)
    h = cv.cvgram_create(_t(X), _t(Y), _t(fold), 1, 1, 1, 1, ddof=1, mode="fp64")
    xx_all, xy_all = cv.cvgram_folds_all(h, 0, 5)
    for p in (0, 4):
        for combo in O.COMBOS:
            a, b = cv.cvgram_fold_combo(h, p, *combo)
            assert torch.equal(a, xx_all[p, O.xtx_class(*combo)])
            assert torch.equal(b, xy_all[p, O.xty_class(*combo)])
        a, b = cv.cvgram_fold(h, p)
        assert torch.equal(a, xx_all[p, 3]) and torch.equal(b, xy_all[p, 7])
    cv.cvgram_destroy(h)


def test_training_statistics_match_oracle():
    shape, (X, Y, fold) = G.workload(1)
    for ddof in (0, 1):
        h = cv.cvgram_create(_t(X), _t(Y), _t(fold), ddof=ddof, mode="fp64")
        for p in range(5):
            got = [t.cpu().numpy() for t in cv.cvgram_fold_stats(h, p)]
            ref = O.fold_train_stats(X, Y, fold, p, ddof)
            for g, r in zip(got, ref):
                assert np.allclose(g, r, rtol=1e-12, atol=0), (p, ddof)
        cv.cvgram_destroy(h)


def test_deterministic_repeat():
    shape, (X, Y, fold) = G.workload(2, n=20000)
    Xd, Yd, fd = _t(X), _t(Y), _t(fold)
    outs = []
    for _ in range(2):
        h = cv.cvgram_create(Xd, Yd, fd, 1, 1, 1, 1, mode="fp64")
        xx, xy = cv.cvgram_folds_all(h, 0, cv.cvgram_num_folds(h))
        torch.cuda.synchronize()
        outs.append((xx.cpu(), xy.cpu()))
        cv.cvgram_destroy(h)
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


# ---------------------------------------------------------------------------
# full spectra workload (N=100000, K=512, M=8, P=10): sampled entries
# ---------------------------------------------------------------------------

def test_fp64_spectra_full_size_sampled():
    shape, (X, Y, fold) = G.workload(2)
    print(f"[parity] {shape.name}", flush=True)
    h = cv.cvgram_create(_t(X), _t(Y), _t(fold), 1, 1, 1, 1, ddof=1, mode="fp64")
    P = cv.cvgram_num_folds(h)
    xx, xy = cv.cvgram_folds_all(h, 0, P)
    torch.cuda.synchronize()
    xx = xx.cpu().numpy()
    xy = xy.cpu().numpy()
    rng = np.random.default_rng(0)
    K, M = X.shape[1], Y.shape[1]
    sizes = np.bincount(fold, minlength=P)
    for p in sorted({0, 3, P - 1, int(np.argmin(sizes)), int(np.argmax(sizes))}):
        # every entry among 16 X and 4 Y columns, against its Cauchy-Schwarz
        # scale (tests/sampling.py)
        xcols = S.pick_columns(K, 16, rng)
        ycols = S.pick_columns(M, 4, rng)
        res = S.compare_fold(xx[p][:, xcols][:, :, xcols], xy[p][:, xcols][:, :, ycols],
                             X[:, xcols], Y[:, ycols], fold, p)
        for kind in ("xtx", "xty"):
            for c, (ew, fe) in enumerate(res[kind]):
                assert ew <= FP64_TOL and fe <= FP64_TOL, (p, kind, c, ew, fe)
        # properties that hold at any size
        nt = int((fold != p).sum())
        assert np.array_equal(xx[p, 3], xx[p, 3].T)
        assert np.allclose(np.diag(xx[p, 3]), nt - 1, rtol=1e-12)
        assert np.all(np.abs(xx[p, 3]) <= (nt - 1) * (1 + 1e-12))
    # one whole fold against the oracle's full product
    oxx, oxy = O.fold_all_classes(X, Y, fold, 1, ddof=1)
    for c in range(4):
        assert _relerr(xx[1, c], oxx[c]) <= FP64_TOL
    for c in range(8):
        assert _relerr(xy[1, c], oxy[c]) <= FP64_TOL
    cv.cvgram_destroy(h)


@pytest.mark.parametrize("mode", ["fp64", "bf16x3"])
def test_not_scalable_partition_writes_nan_only_where_undefined(mode):
    """Definition 6 fails: fold 0 holds all rows but one, so its training
    partition has one row and no deviation with ddof = 1.  cvgram_folds_all
    writes every class: fold 0's scaled classes are NaN, its unscaled ones
    and every class of fold 1 are the oracle's.  The single-combination call
    with scaling reports CVGRAM_ENOTSCALABLE."""
    n, k, m = 40, 9, 2
    rng = np.random.default_rng(66)
    X = rng.normal(3.0, 1.0, (n, k))
    Y = X[:, :m] + rng.normal(0, 0.2, (n, m))
    fold = np.zeros(n, np.int32)
    fold[17] = 1
    # a handle asked for a scaled combination is refused (Definition 6)
    with pytest.raises(cv.CVGramError) as ei:
        cv.cvgram_create(_t(X), _t(Y), _t(fold), 1, 1, 1, 1, ddof=1, mode=mode)
    assert ei.value.name == "CVGRAM_ENOTSCALABLE"
    h = cv.cvgram_create(_t(X), _t(Y), _t(fold), 1, 0, 1, 0, ddof=1, mode=mode)
    xx, xy = cv.cvgram_folds_all(h, 0, 2)
    torch.cuda.synchronize()
    xx = xx.double().cpu().numpy()
    xy = xy.double().cpu().numpy()
    tol = FP64_TOL if mode == "fp64" else 2e-5
    scaled_xx, scaled_xy = (1, 3), (1, 2, 3, 5, 6, 7)
    for c in scaled_xx:
        assert np.all(np.isnan(xx[0, c])), c
    for c in scaled_xy:
        assert np.all(np.isnan(xy[0, c])), c
    # fold 0's unscaled classes (the oracle without scaling)
    oxx, oxy = O.fold_all_classes(X, Y, fold, 0, ddof=1, scaling=False)
    for c in (0, 2):
        assert _relerr(xx[0, c], oxx[c]) <= tol, c
    for c in (0, 4):
        assert _relerr(xy[0, c], oxy[c]) <= tol, c
    # fold 1 (39 training rows): every class.  Its training rows are those of
    # fold 0 of a scalable relabelling (row 17 alone, the rest split in two),
    # so the oracle computes them there.
    relab = np.where(np.arange(n) % 2 == 0, 1, 2).astype(np.int32)
    relab[17] = 0
    oxx, oxy = O.fold_all_classes(X, Y, relab, 0, ddof=1)
    for c in range(4):
        assert _relerr(xx[1, c], oxx[c]) <= tol, c
    for c in range(8):
        assert _relerr(xy[1, c], oxy[c]) <= tol, c
    with pytest.raises(cv.CVGramError) as ei:
        cv.cvgram_fold_combo(h, 1, 1, 1, 1, 1)
    assert ei.value.name == "CVGRAM_ENOTSCALABLE"
    cv.cvgram_destroy(h)


# ---------------------------------------------------------------------------
# error paths that need device-resident labels
# ---------------------------------------------------------------------------

def test_error_statuses():
    rng = np.random.default_rng(1)
    X = _t(rng.standard_normal((10, 2)))
    Y = _t(rng.standard_normal((10, 1)))

    def status(fold, **kw):
        try:
            h = cv.cvgram_create(X, Y, _t(np.array(fold, np.int32)), **kw)
        except cv.CVGramError as e:
            return e.status
        cv.cvgram_destroy(h)
        return 0

    # more labels than the one-pass label count covers: the sort's own check
    n = 6000
    big = np.arange(n, dtype=np.int32) % 5001
    big[big == 4321] = 0                                         # fold 4321 empty
    Xb = _t(rng.standard_normal((n, 2)))
    Yb = _t(rng.standard_normal((n, 1)))
    with pytest.raises(cv.CVGramError) as ei:
        cv.cvgram_create(Xb, Yb, _t(big))
    assert ei.value.status == 2
    big[0] = 4321                                                # every fold non-empty
    cv.cvgram_destroy(cv.cvgram_create(Xb, Yb, _t(big)))

    assert status([0] * 10) == 2                                 # P = 1
    assert status([0, 1, 3, 3, 0, 1, 3, 0, 1, 3]) == 2           # fold 2 empty
    assert status([0, 1, -1, 0, 1, 0, 1, 0, 1, 0]) == 2          # negative label
    assert status([0, 1, 2, 3, 4, 5, 6, 7, 8, 11]) == 2          # P > N
    nonscal = [0] * 9 + [1]                                      # |T_0| = 1
    assert status(nonscal, scale_x=1) == 3
    assert status(nonscal, center_x=1) == 0
    assert status(nonscal, scale_x=1, ddof=0) == 0
    h = cv.cvgram_create(X, Y, _t(np.array(nonscal, np.int32)), center_x=1)
    with pytest.raises(cv.CVGramError) as ei:
        cv.cvgram_fold_combo(h, 0, 1, 1, 1, 1)
    assert ei.value.status == 3
    with pytest.raises(cv.CVGramError) as ei:
        cv.cvgram_fold(h, 2)
    assert ei.value.status == 6
    cv.cvgram_destroy(h)


@pytest.mark.parametrize("n,k,m,p,dtype,mode", [
    (3001, 130, 5, 7, "f64", "fp64"), (1500, 2048, 3, 3, "f32", "fp64"),
    (1500, 2049, 3, 3, "f32", "fp64"), (6000, 300, 40, 5, "f32", "bf16x3"),
    (20000, 64, 4, 20000, "f64", "fp64"), (9000, 100, 2, 9, "f32", "fp32"),
])
def test_plan_query_matches_created_plan(n, k, m, p, dtype, mode):
    """cvgram_plan_query (host only) returns the plan cvgram_create makes."""
    values = "gaussian" if dtype == "f64" else "offset"
    kind = "dirichlet" if p < n else "near_equal"   # p = n: leave-one-out
    shape = G.Shape(f"plan N={n} K={k}", n, k, m, p, dtype, values, kind)
    X, Y, fold = G.make(shape, 17 + k, 0)
    sizes = np.bincount(fold, minlength=int(fold.max()) + 1)
    q = cv.cvgram_plan_query(n, k, m, sizes, dtype, mode)
    h = cv.cvgram_create(_t(X), _t(Y), _t(fold.astype(np.int32)), 1, 1, 1, 1, ddof=1, mode=mode)
    info = cv.cvgram_plan_info(h)
    cv.cvgram_destroy(h)
    print(f"[plan] {shape.name} {mode}: {info}", flush=True)
    for key in ("tile", "items", "slabs", "fused", "panel_bytes"):
        assert q[key] == info[key], (key, q, info)
