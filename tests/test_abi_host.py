"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function that include/cvgram.h declares, and rejects bad arguments
before touching the device."""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys

import pytest

import paper_2401_13185_amd as cv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    declared = cv.header_symbols()
    assert "cvgram_create" in declared and "cvgram_fold" in declared
    lib = cv.load()
    missing = [s for s in declared if not hasattr(lib, s)]
    assert not missing, missing
    # the binding exposes the same names
    for s in declared:
        assert hasattr(cv, s), s


def test_status_strings_and_version():
    assert cv.cvgram_version() >= 100
    for st in range(8):
        assert cv.cvgram_status_string(st)
    assert cv.cvgram_status_string(99) == "unknown status"


def _create_raw(X=None, Y=None, fold=None, N=10, K=3, M=1, dtype=1, flags=(0, 0, 0, 0), ddof=1,
                mode=0):
    lib = cv.load()
    out = ctypes.c_void_p(123)
    st = lib.cvgram_create(X, Y, fold, N, K, M, dtype, *flags, ddof, mode, None, ctypes.byref(out))
    return st, out.value


FAKE = 0x1000  # never dereferenced: every case below fails before device work


@pytest.mark.parametrize("kw,status", [
    (dict(X=None, fold=FAKE), 1),
    (dict(X=FAKE, fold=None), 1),
    (dict(X=FAKE, fold=FAKE, Y=None, M=2), 1),
    (dict(X=FAKE, fold=FAKE, Y=FAKE, N=1), 1),
    (dict(X=FAKE, fold=FAKE, Y=FAKE, K=0), 1),
    (dict(X=FAKE, fold=FAKE, Y=FAKE, M=-1), 1),
    (dict(X=FAKE, fold=FAKE, Y=FAKE, dtype=7), 1),
    (dict(X=FAKE, fold=FAKE, Y=FAKE, mode=9), 1),
    (dict(X=FAKE, fold=FAKE, Y=FAKE, flags=(2, 0, 0, 0)), 1),
    (dict(X=FAKE, fold=FAKE, Y=FAKE, ddof=2), 1),
    (dict(X=FAKE, fold=FAKE, Y=FAKE, N=2**31), 1),
])
def test_create_rejects_bad_arguments_before_device_work(kw, status):
    st, h = _create_raw(**kw)
    assert st == status
    assert h is None
    assert cv.cvgram_last_error_message()


def test_null_handle_calls():
    lib = cv.load()
    assert lib.cvgram_num_folds(None) == -1
    assert lib.cvgram_fold(None, 0, None, None) == 1
    assert lib.cvgram_fold_combo(None, 0, 0, 0, 0, 0, None, None) == 1
    assert lib.cvgram_fold_leaky(None, 0, 1, None, None) == 1
    assert lib.cvgram_ridge(None, 0, 1, None, 1, None) == 1
    assert lib.cvgram_folds_all(None, 0, 1, None, None) == 1
    assert lib.cvgram_fold_stats(None, 0, None, None, None, None) == 1
    assert lib.cvgram_partition(None, None, None) == 1
    assert lib.cvgram_set_stream(None, None) == 1
    assert lib.cvgram_destroy(None) == 0


def test_batch_and_autotune_reject_bad_arguments():
    lib = cv.load()
    out = ctypes.c_void_p(1)
    assert lib.cvgram_batch_create(None, 1, 1, 1, 0, None, ctypes.byref(out)) == 1
    assert out.value is None
    probs = (cv._Problem * 1)()
    probs[0] = cv._Problem(FAKE, FAKE, FAKE, 10, 3, 1, None, None)
    assert lib.cvgram_batch_create(probs, 0, 1, 1, 0, None, ctypes.byref(out)) == 1
    assert lib.cvgram_batch_create(probs, 1, 5, 1, 0, None, ctypes.byref(out)) == 1
    assert lib.cvgram_batch_create(probs, 1, 1, 3, 0, None, ctypes.byref(out)) == 1
    probs[0] = cv._Problem(FAKE, None, FAKE, 10, 3, 2, None, None)   # Y NULL with M > 0
    assert lib.cvgram_batch_create(probs, 1, 1, 1, 0, None, ctypes.byref(out)) == 1
    assert "problem 0" in cv.cvgram_last_error_message()
    assert lib.cvgram_batch_run(None) == 1
    assert lib.cvgram_batch_run_eager(None) == 1
    assert lib.cvgram_batch_destroy(None) == 0
    t, i = ctypes.c_int32(), ctypes.c_int32()
    assert lib.cvgram_autotune(None, None, FAKE, 10, 3, 0, 1, 0, None, ctypes.byref(t),
                               ctypes.byref(i)) == 1
    # the batch tuner validates before any device work
    w, ms = ctypes.c_int32(), ctypes.c_double()
    outs = (ctypes.byref(t), ctypes.byref(w), ctypes.byref(i), ctypes.byref(ms))
    probs[0] = cv._Problem(FAKE, FAKE, FAKE, 10, 3, 1, None, None)
    assert lib.cvgram_batch_autotune(None, 1, 1, 0, None, *outs) == 1
    assert lib.cvgram_batch_autotune(probs, 0, 1, 0, None, *outs) == 1
    assert lib.cvgram_batch_autotune(probs, 1, 5, 0, None, *outs) == 1
    assert lib.cvgram_batch_autotune(probs, 1, 1, 7, None, *outs) == 1
    probs[0] = cv._Problem(FAKE, None, FAKE, 10, 3, 2, None, None)   # Y NULL with M > 0
    assert lib.cvgram_batch_autotune(probs, 1, 1, 0, None, *outs) == 1
    assert "problem 0" in cv.cvgram_last_error_message()


def test_product_path_has_no_oracle_or_cpu_fallback():
    """The package and its native sources never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_2401_13185_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.replace("oracle/", ""), f
                assert "import numpy" not in text, f


def test_binding_fails_loudly_without_library(tmp_path):
    """With the shared library absent, the binding raises instead of falling
    back to anything else."""
    code = (
        "import paper_2401_13185_amd as cv, os\n"
        "cv.lib_path = lambda: os.path.join(%r, 'missing.so')\n"
        "try:\n    cv.load()\nexcept RuntimeError as e:\n    print('raised', e)\n" % str(tmp_path)
    )
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT)
    assert "raised" in r.stdout, r.stdout + r.stderr


def _header_enum(prefix):
    import re
    text = open(cv.HEADER).read()
    return {m.group(1): int(m.group(2))
            for m in re.finditer(r"\b(" + prefix + r"[A-Z0-9_]+)\s*=\s*(\d+)", text)}


def test_mode_numbering_matches_header_and_binding():
    """The arithmetic modes are numbered FP64 = 0, BF16X3 = 1, FP32 = 2 in the
    header, and the binding passes the same numbers."""
    modes = _header_enum("CVGRAM_MODE_")
    assert modes == {"CVGRAM_MODE_FP64": 0, "CVGRAM_MODE_BF16X3": 1, "CVGRAM_MODE_FP32": 2}
    assert cv.MODES == {"fp64": 0, "bf16x3": 1, "fp32": 2}
    status = _header_enum("CVGRAM_E")
    status["CVGRAM_OK"] = 0
    assert {v: k for k, v in status.items()} == cv.STATUS


def test_num_folds_returns_int32_and_minus_one_for_null():
    lib = cv.load()
    assert lib.cvgram_num_folds.restype is ctypes.c_int32
    assert lib.cvgram_num_folds(None) == -1
    assert "NULL" in cv.cvgram_last_error_message()
