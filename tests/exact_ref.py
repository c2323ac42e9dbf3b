"""Exact brute-force reference for tiny inputs (test helper, independent of
the oracle: it shares no code with it and uses no floating point until the
final rounding).

Rows, means and sums are Python ``Fraction``s.  A scaled entry is
(exact rational) / sqrt(var_i * var_j) with var rational, evaluated in
``decimal`` at 60 significant digits, then rounded once to a float.
"""
from __future__ import annotations

from decimal import Decimal, getcontext
from fractions import Fraction

getcontext().prec = 60


def _dec(q: Fraction) -> Decimal:
    return Decimal(q.numerator) / Decimal(q.denominator)


def _column(rows, j):
    return [Fraction(r[j]) for r in rows]


def _prep(vals, center, ddof):
    """Centred (or raw) exact column, its exact variance about the training
    mean, and whether it is constant."""
    n = len(vals)
    mu = sum(vals, Fraction(0)) / n
    const = all(v == vals[0] for v in vals)
    ss = sum(((v - mu) ** 2 for v in vals), Fraction(0))
    var = ss / (n - ddof) if n - ddof >= 1 else None
    out = [v - mu for v in vals] if center else list(vals)
    return out, var, const, mu


def exact_fold(X, Y, fold_id, p, cx, sx, cy, sy, ddof):
    """(XtX, XtY) of fold p as nested lists of floats, by brute force."""
    T = [n for n in range(len(fold_id)) if fold_id[n] != p]
    XT = [X[n] for n in T]
    YT = [Y[n] for n in T]
    K = len(X[0])
    M = len(Y[0])
    xs = [_prep(_column(XT, j), cx, ddof) for j in range(K)]
    ys = [_prep(_column(YT, j), cy, ddof) for j in range(M)]

    def scale_of(entry, scale):
        _, var, const, _ = entry
        if not scale or const:
            return Fraction(1)
        return var  # squared scale

    def value(a, b, sa, sb):
        num = sum((u * v for u, v in zip(a[0], b[0])), Fraction(0))
        den2 = scale_of(a, sa) * scale_of(b, sb)
        if den2 == 1:
            return float(num)
        return float(_dec(num) / _dec(den2).sqrt())

    xtx = [[value(xs[i], xs[j], sx, sx) for j in range(K)] for i in range(K)]
    xty = [[value(xs[i], ys[j], sx, sy) for j in range(M)] for i in range(K)]
    return xtx, xty


def exact_stats(A, rows, ddof):
    """Exact training mean and deviation (1 for a constant column) of the
    columns of A over ``rows``, rounded to floats."""
    out_m, out_s = [], []
    for j in range(len(A[0])):
        vals = [Fraction(A[n][j]) for n in rows]
        _, var, const, mu = _prep(vals, False, ddof)
        out_m.append(float(mu))
        out_s.append(1.0 if const else float(_dec(var).sqrt()))
    return out_m, out_s
