"""Stream-ordered release and stream changes, on the GPU.

cvgram_destroy returns a handle's workspace to the cache without waiting:
the blocks carry an event recorded on the handle's stream.  A handle created
on another stream right after takes the same blocks and must wait for that
event; cvgram_set_stream must order the new stream's work behind the old
stream's.  The first case delays the first stream with a bounded spin kernel
so that a missing wait would let the two handles' work overlap in the same
memory; the second reads a Gram still running on the old stream.  The
results must equal, bit for bit, a reference computed with full
synchronisation (which the oracle anchors on one fold).
"""
from __future__ import annotations

import numpy as np
import pytest

import paper_2401_13185_amd as cv
from oracle import cv_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N, K, M, P = 20000, 96, 4, 5
DELAY_CYCLES = 50_000_000  # a few tens of milliseconds of spinning


def _dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    return torch.device("cuda:0")


def _data(n=N, k=K):
    rng = np.random.default_rng(21)
    X = rng.normal(3.0, 1.5, size=(n, k))
    Y = X[:, :M] * 0.5 + rng.normal(0.0, 0.2, size=(n, M))
    fold = rng.integers(0, P, size=n).astype(np.int32)
    fold[:P] = np.arange(P)
    dev = _dev()
    return X, Y, fold, torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev), \
        torch.from_numpy(fold).to(dev)


def _outputs(dev, k=K):
    return (torch.empty(P, 4, k, k, dtype=torch.float64, device=dev),
            torch.empty(P, 8, k, M, dtype=torch.float64, device=dev))


def _reference(Xd, Yd, fd):
    xx, xy = _outputs(Xd.device, Xd.shape[1])
    h = cv.cvgram_create(Xd, Yd, fd, 1, 1, 1, 1, ddof=1)
    cv.cvgram_folds_all(h, 0, P, xx, xy)
    torch.cuda.synchronize()
    cv.cvgram_destroy(h)
    torch.cuda.synchronize()
    return xx, xy


def test_release_then_reuse_on_another_stream():
    X, Y, fold, Xd, Yd, fd = _data()
    ref_xx, ref_xy = _reference(Xd, Yd, fd)
    oxx, oxy = O.fold_all_classes(X, Y, fold, 0, ddof=1)
    for c in range(4):
        assert np.linalg.norm(ref_xx[0, c].cpu().numpy() - oxx[c]) <= 1e-10 * np.linalg.norm(oxx[c])
    for c in range(8):
        assert np.linalg.norm(ref_xy[0, c].cpu().numpy() - oxy[c]) <= 1e-10 * np.linalg.norm(oxy[c])

    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()

    def run(stream, delay):
        with torch.cuda.stream(stream):
            xx, xy = _outputs(Xd.device)
            h = cv.cvgram_create(Xd, Yd, fd, 1, 1, 1, 1, ddof=1, stream=stream)
            if delay:
                # the corrections, which read the handle's workspace, wait
                # behind the spin
                torch.cuda._sleep(delay)
            cv.cvgram_folds_all(h, 0, P, xx, xy)
            cv.cvgram_destroy(h)  # returns at once: the work is still queued
        return xx, xy

    outs = []
    for it in range(3):
        print(f"[streams] round {it}", flush=True)
        outs.append(run(s1, DELAY_CYCLES))  # still running when the next handle is made
        outs.append(run(s2, 0))
    torch.cuda.synchronize()
    for xx, xy in outs:
        assert torch.equal(xx, ref_xx)
        assert torch.equal(xy, ref_xy)


def test_set_stream_orders_the_new_stream_behind_the_old():
    # a problem whose Gram takes milliseconds: still running on s1 when
    # create returns and the corrections are queued on s2
    n, k = 400_000, 512
    X, Y, fold, Xd, Yd, fd = _data(n, k)
    ref_xx, ref_xy = _reference(Xd, Yd, fd)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for it in range(2):
        print(f"[streams] set_stream round {it}", flush=True)
        with torch.cuda.stream(s1):
            h = cv.cvgram_create(Xd, Yd, fd, 1, 1, 1, 1, ddof=1, stream=s1)
        with torch.cuda.stream(s2):
            xx, xy = _outputs(Xd.device, k)
        cv.cvgram_set_stream(h, s2)
        # the corrections on s2 read the Gram still running on s1
        cv.cvgram_folds_all(h, 0, P, xx, xy)
        cv.cvgram_destroy(h)
        torch.cuda.synchronize()
        assert torch.equal(xx, ref_xx)
        assert torch.equal(xy, ref_xy)
