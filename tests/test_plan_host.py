"""Host tests of the planner through cvgram_plan_query (no device needed):
tile and panel rules, work-list sizes against closed-form tile counts, the
fused / grouped choice, the XCD balance and the workspace size, and the
argument errors."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import paper_2401_13185_amd as cv
from synth import generators as G


def _dirichlet_sizes(n, p, seed=0):
    lab = G.folds_dirichlet(n, p, np.random.default_rng(seed))
    return np.bincount(lab, minlength=p)


def _x_tiles(K, M, tile):
    """Output tiles per fold row range: the upper triangle of X^T X in
    128-wide (or 64-wide) tiles plus the X^T Y tiles when M > 32; for
    256 x 128 tiles the pairs (ti, tj >= 2 ti)."""
    tb = 128 if tile == 256 else tile
    kp = -(-K // tile) * tile
    nt = kp // tb
    nyt = 0 if M <= 32 else -(-M // tb)
    if tile == 256:
        na = kp // 256
        return sum(nt - 2 * ti for ti in range(na)) + na * nyt
    return nt * (nt + 1) // 2 + nt * nyt


def test_large_problem_plans():
    sizes = _dirichlet_sizes(2_000_000, 64)
    q = cv.cvgram_plan_query(2_000_000, 4096, 64, sizes, "f32", "fp64")
    assert (q["tile"], q["panel_bytes"], q["fused"], q["slabs"]) == (128, 8, False, 64)
    assert q["items"] == 64 * _x_tiles(4096, 64, 128) == 35840
    # the XCDs get whole tile groups of near-equal cost
    assert 1 <= q["xcd_items_min"] <= q["xcd_items_max"] <= 1.25 * q["xcd_items_min"]
    b = cv.cvgram_plan_query(2_000_000, 4096, 64, sizes, "f32", "bf16x3")
    assert (b["tile"], b["panel_bytes"], b["slabs"]) == (256, 2, 64)
    assert b["items"] == 64 * _x_tiles(4096, 64, 256) == 18432
    # FP64 panels: 2e6 rows in 64 folds padded to 32-row panels x 4224 columns x 8 bytes
    np_rows = int(sum(-(-int(s) // 32) * 32 for s in sizes))
    assert q["workspace_bytes"] >= np_rows * (4096 + 128) * 8
    assert b["workspace_bytes"] >= 2 * np_rows * (4096 + 128) * 2


@pytest.mark.parametrize("K,dtype,mode,expect", [
    (2048, "f32", "fp64", 4), (2049, "f32", "fp64", 8), (512, "f64", "fp64", 8),
    (512, "f32", "fp32", 4), (512, "f64", "fp32", 4), (512, "f32", "bf16x3", 2),
])
def test_panel_element_rule(K, dtype, mode, expect):
    q = cv.cvgram_plan_query(1500, K, 3, [500, 500, 500], dtype, mode)
    assert q["panel_bytes"] == expect


@pytest.mark.parametrize("K,mode,tile", [
    (64, "fp64", 64), (65, "fp64", 128), (4096, "fp64", 128), (64, "bf16x3", 64),
    (128, "bf16x3", 128), (129, "bf16x3", 256), (64, "fp32", 64), (1000, "fp32", 128),
])
def test_tile_rule(K, mode, tile):
    assert cv.cvgram_plan_query(4000, K, 2, [1000] * 4, "f32", mode)["tile"] == tile


def test_fused_for_many_small_folds_grouped_otherwise():
    loo = cv.cvgram_plan_query(100_000, 512, 8, [1] * 100_000, "f64", "fp64")
    assert loo["fused"]
    grouped = cv.cvgram_plan_query(100_000, 512, 8, [10_000] * 10, "f64", "fp64")
    assert not grouped["fused"]
    # the fused path splits the whole row range, the grouped one each fold
    assert grouped["slabs"] >= 10 and grouped["items"] == grouped["slabs"] * _x_tiles(512, 8, 128)
    assert loo["items"] == loo["slabs"] * _x_tiles(512, 8, 128)


def test_row_splits_fill_the_chip_and_workspace_grows_with_rows():
    small = cv.cvgram_plan_query(20_000, 512, 8, [2000] * 10, "f64", "fp64")
    large = cv.cvgram_plan_query(200_000, 512, 8, [20_000] * 10, "f64", "fp64")
    # few tiles per fold: the folds are split along rows into several slabs
    assert small["slabs"] > 10 and large["slabs"] > 10
    assert large["workspace_bytes"] > small["workspace_bytes"]
    # panels + slabs lower-bound the workspace
    for q, n in ((small, 20_000), (large, 200_000)):
        assert q["workspace_bytes"] >= n * (512 + 32) * 8 + q["slabs"] * 512 * 520 * 8


def test_plan_query_errors():
    with pytest.raises(cv.CVGramError) as ei:
        cv.cvgram_plan_query(10, 4, 1, [5, 0, 5], "f32", "fp64")   # empty fold
    assert ei.value.status == 2
    with pytest.raises(cv.CVGramError) as ei:
        cv.cvgram_plan_query(10, 4, 1, [5, 4], "f32", "fp64")      # sizes sum to 9
    assert ei.value.status == 1
    with pytest.raises(cv.CVGramError) as ei:
        cv.cvgram_plan_query(1, 4, 1, [1], "f32", "fp64")          # N < 2
    assert ei.value.status == 1
    lib = cv.load()
    info = (ctypes.c_int64 * 8)()
    sizes = (ctypes.c_int64 * 2)(5, 5)
    assert lib.cvgram_plan_query(10, 4, 1, sizes, 2, 0, 9, info, 8) == 1    # bad mode
    assert lib.cvgram_plan_query(10, 4, 1, sizes, 2, 3, 0, info, 8) == 1    # bad dtype
    assert lib.cvgram_plan_query(10, 4, 1, None, 2, 0, 0, info, 8) == 1     # no sizes
