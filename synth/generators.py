"""Seeded synthetic inputs for the fold-independent cross-validation Gram path.

This module only draws data: row-major X (N x K), Y (N x M) and an int32 fold
label per row.  It holds none of the method's arithmetic (no Gram products, no
means or deviations of the data); both the FP64 oracle and the GPU path read
the same arrays from here.

Randomness: every array is drawn from numpy's PCG64 seeded by a SeedSequence
whose entropy is (13185, workload, problem, stream, chunk).  Rows are drawn in
fixed-size chunks with one generator per chunk, so any row range can be
regenerated on its own and the result does not depend on how many threads
drew it.  Values are drawn in FP64 and cast to the requested dtype at the end.

Workloads (shapes follow the paper's benchmark setting in Section 7; the value
models are these):
  * ``gaussian``   -- per-column Gaussian X, column mean ~ N(5, 2^2), column
                      std ~ LogNormal(0, 0.5); Y = X W + N(0, 0.1^2).
  * ``spectra``    -- smooth spectra: per row a baseline ~ U(0.5, 2) plus five
                      Gaussian bumps (centre ~ U(0,1), width ~ U(0.01, 0.1),
                      amplitude ~ U(0.1, 1)) on t_k = k/(K-1), plus N(0, 1e-3^2)
                      noise; Y = X W / sqrt(K) + N(0, 0.1^2).
  * ``offset``     -- precision stress: column mean ~ U(1e3, 1e4), column std
                      ~ U(0.1, 1); Y has the same offset model and depends
                      linearly on the standardised X.
Fold labels are 0-based (label p is the paper's partition p+1 of Definition 1).
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

ROOT_SEED = 13185
CHUNK_ROWS = 32768

# stream tags inside one problem
_S_PARAMS = 1
_S_X = 2
_S_Y = 3
_S_FOLDS = 4


def _rng(workload: int, problem: int, stream: int, chunk: int = 0) -> np.random.Generator:
    ss = np.random.SeedSequence([ROOT_SEED, workload, problem, stream, chunk])
    return np.random.Generator(np.random.PCG64(ss))


def _chunks(n: int):
    for c, start in enumerate(range(0, n, CHUNK_ROWS)):
        yield c, start, min(n, start + CHUNK_ROWS)


def _fill_rows(n: int, width: int, fn, threads: int | None = None) -> np.ndarray:
    """Allocate an (n, width) FP64 array and fill it chunk by chunk with
    ``fn(chunk_index, start, stop) -> array``; chunks are independent."""
    out = np.empty((n, width), dtype=np.float64)
    jobs = list(_chunks(n))

    def run(job):
        c, a, b = job
        out[a:b] = fn(c, a, b)

    if threads is None:
        threads = min(16, max(1, (len(jobs) + 3) // 4))
    if threads <= 1 or len(jobs) <= 1:
        for j in jobs:
            run(j)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(run, jobs))
    return out


# ---------------------------------------------------------------------------
# fold labels
# ---------------------------------------------------------------------------

def folds_near_equal(n: int, p: int, rng: np.random.Generator) -> np.ndarray:
    """Random permutation split into p near-equal parts (the first n mod p
    folds get one extra row)."""
    if not 1 <= p <= n:
        raise ValueError("need 1 <= P <= N")
    perm = rng.permutation(n)
    base, extra = divmod(n, p)
    sizes = np.full(p, base, dtype=np.int64)
    sizes[:extra] += 1
    fold = np.empty(n, dtype=np.int32)
    start = 0
    for f in range(p):
        fold[perm[start:start + sizes[f]]] = f
        start += sizes[f]
    return fold


def dirichlet_sizes(n: int, p: int, rng: np.random.Generator, alpha: float = 2.0) -> np.ndarray:
    """Uneven fold sizes from Dirichlet(alpha) proportions: floor(w*n), the
    remainder to the largest fractional parts (ties to the lower fold), then
    every empty fold takes one row from the currently largest fold."""
    if not 1 <= p <= n:
        raise ValueError("need 1 <= P <= N")
    w = rng.dirichlet(np.full(p, alpha))
    raw = w * n
    sizes = np.floor(raw).astype(np.int64)
    rem = n - int(sizes.sum())
    frac = raw - sizes
    order = np.argsort(-frac, kind="stable")
    sizes[order[:rem]] += 1
    for f in range(p):
        if sizes[f] == 0:
            big = int(np.argmax(sizes))
            sizes[big] -= 1
            sizes[f] += 1
    assert int(sizes.sum()) == n and sizes.min() >= 1
    return sizes


def folds_from_sizes(sizes: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    n = int(np.sum(sizes))
    perm = rng.permutation(n)
    fold = np.empty(n, dtype=np.int32)
    start = 0
    for f, s in enumerate(sizes):
        fold[perm[start:start + int(s)]] = f
        start += int(s)
    return fold


def folds_dirichlet(n: int, p: int, rng: np.random.Generator, alpha: float = 2.0) -> np.ndarray:
    return folds_from_sizes(dirichlet_sizes(n, p, rng, alpha), rng)


def folds_venetian(n: int, p: int) -> np.ndarray:
    """Every p-th row in the same fold (venetian blinds, Definition 1)."""
    return (np.arange(n) % p).astype(np.int32)


def folds_contiguous(n: int, p: int) -> np.ndarray:
    """p contiguous blocks of near-equal size: row n goes to floor(n*p/N)."""
    return ((np.arange(n, dtype=np.int64) * p) // n).astype(np.int32)


# ---------------------------------------------------------------------------
# value models
# ---------------------------------------------------------------------------

def gaussian_xy(n: int, k: int, m: int, workload: int, problem: int = 0):
    """Gaussian columns with mean ~ N(5, 2^2), std ~ LogNormal(0, 0.5);
    Y = X W + N(0, 0.1^2) with W ~ N(0, 1)^{K x M}."""
    pr = _rng(workload, problem, _S_PARAMS)
    mu = pr.normal(5.0, 2.0, size=k)
    sd = pr.lognormal(0.0, 0.5, size=k)
    W = pr.standard_normal((k, m))

    def xfn(c, a, b):
        r = _rng(workload, problem, _S_X, c)
        return mu + sd * r.standard_normal((b - a, k))

    X = _fill_rows(n, k, xfn)

    def yfn(c, a, b):
        r = _rng(workload, problem, _S_Y, c)
        return X[a:b] @ W + r.normal(0.0, 0.1, size=(b - a, m))

    Y = _fill_rows(n, m, yfn)
    return X, Y


def spectra_xy(n: int, k: int, m: int, workload: int, problem: int = 0):
    """Smooth spectra (baseline + 5 Gaussian bumps + small noise)."""
    pr = _rng(workload, problem, _S_PARAMS)
    W = pr.standard_normal((k, m)) / math.sqrt(k)
    t = np.arange(k, dtype=np.float64) / max(1, k - 1)

    def xfn(c, a, b):
        r = _rng(workload, problem, _S_X, c)
        rows = b - a
        base = r.uniform(0.5, 2.0, size=(rows, 1))
        centre = r.uniform(0.0, 1.0, size=(rows, 5))
        width = r.uniform(0.01, 0.1, size=(rows, 5))
        amp = r.uniform(0.1, 1.0, size=(rows, 5))
        out = np.repeat(base, k, axis=1)
        for j in range(5):
            z = (t[None, :] - centre[:, j:j + 1]) / width[:, j:j + 1]
            out += amp[:, j:j + 1] * np.exp(-0.5 * z * z)
        out += r.normal(0.0, 1e-3, size=(rows, k))
        return out

    X = _fill_rows(n, k, xfn)

    def yfn(c, a, b):
        r = _rng(workload, problem, _S_Y, c)
        return X[a:b] @ W + r.normal(0.0, 0.1, size=(b - a, m))

    Y = _fill_rows(n, m, yfn)
    return X, Y


def offset_xy(n: int, k: int, m: int, workload: int, problem: int = 0):
    """Large column offsets: mean ~ U(1e3, 1e4), std ~ U(0.1, 1) for X and Y;
    Y's fluctuation is a linear map of the standardised X plus noise."""
    pr = _rng(workload, problem, _S_PARAMS)
    mu = pr.uniform(1e3, 1e4, size=k)
    sd = pr.uniform(0.1, 1.0, size=k)
    ymu = pr.uniform(1e3, 1e4, size=m)
    ysd = pr.uniform(0.1, 1.0, size=m)
    W = pr.standard_normal((k, m)) / math.sqrt(k)

    def zfn(c, a, b):
        r = _rng(workload, problem, _S_X, c)
        return r.standard_normal((b - a, k))

    Z = _fill_rows(n, k, zfn)

    def yfn(c, a, b):
        r = _rng(workload, problem, _S_Y, c)
        f = Z[a:b] @ W + r.normal(0.0, 0.1, size=(b - a, m))
        return ymu + ysd * f

    Y = _fill_rows(n, m, yfn)
    # X = mu + sd * Z, in place, chunk by chunk
    for _, a, b in _chunks(n):
        Z[a:b] *= sd
        Z[a:b] += mu
    return Z, Y


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Shape:
    name: str
    n: int
    k: int
    m: int
    p: int
    dtype: str          # storage dtype of X and Y: "f64" or "f32"
    values: str         # "gaussian" | "spectra" | "offset"
    folds: str          # "near_equal" | "dirichlet"


WORKLOADS = {
    1: Shape("gaussian N=1000 K=50 M=2 P=5 fp64", 1000, 50, 2, 5, "f64", "gaussian", "near_equal"),
    2: Shape("spectra N=100000 K=512 M=8 P=10 fp64", 100_000, 512, 8, 10, "f64", "spectra", "dirichlet"),
    3: Shape("offset N=1000000 K=1024 M=16 P=100 fp32", 1_000_000, 1024, 16, 100, "f32", "offset", "near_equal"),
    5: Shape("spectra N=2000000 K=4096 M=64 P=64 fp32", 2_000_000, 4096, 64, 64, "f32", "spectra", "dirichlet"),
}

_VALUES = {"gaussian": gaussian_xy, "spectra": spectra_xy, "offset": offset_xy}
_DT = {"f64": np.float64, "f32": np.float32}


def make(shape: Shape, workload: int, problem: int = 0):
    """Draw (X, Y, fold_id) for ``shape``; ``workload``/``problem`` key the seeds."""
    X, Y = _VALUES[shape.values](shape.n, shape.k, shape.m, workload, problem)
    fr = _rng(workload, problem, _S_FOLDS)
    if shape.folds == "near_equal":
        fold = folds_near_equal(shape.n, shape.p, fr)
    elif shape.folds == "dirichlet":
        fold = folds_dirichlet(shape.n, shape.p, fr)
    elif shape.folds == "venetian":
        fold = folds_venetian(shape.n, shape.p)
    elif shape.folds == "contiguous":
        fold = folds_contiguous(shape.n, shape.p)
    else:
        raise ValueError(shape.folds)
    dt = _DT[shape.dtype]
    if dt is not np.float64:
        X = X.astype(dt)
        Y = Y.astype(dt)
    return np.ascontiguousarray(X), np.ascontiguousarray(Y), fold


def workload(wid: int, problem: int = 0, **override):
    """The named workload ``wid`` (optionally with fields overridden, e.g. a
    smaller N for a parity case of the same family)."""
    shape = WORKLOADS[wid]
    if override:
        shape = Shape(**{**shape.__dict__, **override})
    return shape, make(shape, wid, problem)


# ---------------------------------------------------------------------------
# batched workload: many independent problems of different shapes
# ---------------------------------------------------------------------------

BATCH_WORKLOAD = 4


def batch_shapes(count: int = 256, n_lo: int = 1000, n_hi: int = 200_000,
                 ks=(64, 128, 256, 512), m_max: int = 16, p_lo: int = 3, p_hi: int = 20):
    """Shapes of ``count`` independent problems: N ~ log-uniform[n_lo, n_hi],
    K uniform over ``ks``, M ~ U{1..m_max}, P ~ U{p_lo..p_hi}, uneven folds."""
    r = _rng(BATCH_WORKLOAD, 0, _S_PARAMS)
    out = []
    for i in range(count):
        n = int(round(math.exp(r.uniform(math.log(n_lo), math.log(n_hi)))))
        k = int(ks[r.integers(0, len(ks))])
        m = int(r.integers(1, m_max + 1))
        p = int(r.integers(p_lo, p_hi + 1))
        out.append(Shape(f"batch[{i}] N={n} K={k} M={m} P={p} fp32", n, k, m, p,
                         "f32", "spectra", "dirichlet"))
    return out


def batch_problem(shape: Shape, index: int):
    return make(shape, BATCH_WORKLOAD, index + 1)


# ---------------------------------------------------------------------------
# device-side drawing of the same value models (large workloads only)
# ---------------------------------------------------------------------------

def spectra_xy_torch(n: int, k: int, m: int, seed: int, device, dtype=None,
                     chunk_rows: int = 65536):
    """The spectra value model of ``spectra_xy`` drawn with torch's generator
    on ``device`` (a different random stream from the NumPy path: used where
    drawing gigabytes on the host would dominate, never by the oracle tests).
    Returns (X, Y) of ``dtype`` (default float32)."""
    import torch
    dtype = dtype or torch.float32
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = dict(dtype=torch.float64, device=device)
    W = torch.randn(k, m, generator=g, **f64) / math.sqrt(k)
    t = torch.arange(k, **f64) / max(1, k - 1)
    X = torch.empty(n, k, dtype=dtype, device=device)
    Y = torch.empty(n, m, dtype=dtype, device=device)
    for a in range(0, n, chunk_rows):
        b = min(n, a + chunk_rows)
        rows = b - a
        base = 0.5 + 1.5 * torch.rand(rows, 1, generator=g, **f64)
        centre = torch.rand(rows, 5, generator=g, **f64)
        width = 0.01 + 0.09 * torch.rand(rows, 5, generator=g, **f64)
        amp = 0.1 + 0.9 * torch.rand(rows, 5, generator=g, **f64)
        out = base.expand(rows, k).clone()
        for j in range(5):
            z = (t[None, :] - centre[:, j:j + 1]) / width[:, j:j + 1]
            out += amp[:, j:j + 1] * torch.exp(-0.5 * z * z)
        out += 1e-3 * torch.randn(rows, k, generator=g, **f64)
        X[a:b] = out.to(dtype)
        Y[a:b] = (out @ W + 0.1 * torch.randn(rows, m, generator=g, **f64)).to(dtype)
    return X, Y


def batch_problem_device(shape: Shape, index: int, device):
    """A problem of the batched workload with values drawn on ``device``
    (spectra model) and fold labels drawn on the host (Dirichlet(2) sizes)."""
    import torch
    X, Y = spectra_xy_torch(shape.n, shape.k, shape.m, ROOT_SEED * 1000 + index, device)
    fold = folds_dirichlet(shape.n, shape.p, _rng(BATCH_WORKLOAD, index + 1, _S_FOLDS))
    return X, Y, torch.from_numpy(fold).to(device)
