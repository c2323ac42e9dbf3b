"""Python binding of libcvgram: fold-independent cross-validation Gram
products on MI355X (gfx950).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libcvgram.so``; torch supplies device memory and the stream.
The functions mirror the C ABI of ``include/cvgram.h`` (same names, same
meaning); tensors are passed as device pointers.  There is no CPU path: if the
library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import re

__all__ = [
    "CVGramError", "lib_path", "load", "exported_symbols", "header_symbols",
    "cvgram_create", "cvgram_num_folds", "cvgram_plan_info", "cvgram_plan_query",
    "cvgram_partition", "cvgram_fold",
    "cvgram_fold_combo", "cvgram_fold_leaky", "LEAK_KINDS", "cvgram_ridge", "cvgram_folds_all",
    "cvgram_folds_all_noalloc", "cvgram_fold_stats", "cvgram_set_stream",
    "cvgram_destroy", "cvgram_status_string", "cvgram_last_error_message", "cvgram_version",
    "cvgram_set_stage_timing", "cvgram_stage_times", "cvgram_trim_cache",
    "cvgram_batch_create", "cvgram_batch_run", "cvgram_batch_run_eager",
    "cvgram_batch_problem_info", "cvgram_batch_destroy", "cvgram_autotune",
    "cvgram_batch_autotune", "Batch",
    "CVGram", "MODES", "XTX_CLASSES", "XTY_CLASSES",
]

_PKG = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_PKG)
HEADER = os.path.join(_ROOT, "include", "cvgram.h")
MODES = {"fp64": 0, "bf16x3": 1, "fp32": 2}
# leakage comparison kinds of cvgram_fold_leaky (never training-partition results)
LEAK_KINDS = {"global": 1, "lindgren": 2}
XTX_CLASSES = 4
XTY_CLASSES = 8

STATUS = {0: "CVGRAM_OK", 1: "CVGRAM_EINVAL", 2: "CVGRAM_EFOLDS", 3: "CVGRAM_ENOTSCALABLE",
          4: "CVGRAM_ENOMEM", 5: "CVGRAM_EDEVICE", 6: "CVGRAM_ERANGE", 7: "CVGRAM_ESINGULAR"}


class CVGramError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{self.name}: {message}")


def lib_path() -> str:
    return os.path.join(_PKG, "libcvgram.so")


_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_int = ctypes.c_int

_SIGS = {
    "cvgram_create": (_int, [_vp, _vp, _vp, _i64, _i64, _i64, _int, _int, _int, _int, _int, _int,
                             _int, _vp, ctypes.POINTER(_vp)]),
    "cvgram_num_folds": (_i32, [_vp]),
    "cvgram_plan_info": (_int, [_vp, ctypes.POINTER(_i64), _i32]),
    "cvgram_plan_query": (_int, [_i64, _i64, _i64, ctypes.POINTER(_i64), _i32, _int, _int,
                                 ctypes.POINTER(_i64), _i32]),
    "cvgram_partition": (_int, [_vp, _vp, _vp]),
    "cvgram_fold": (_int, [_vp, _i32, _vp, _vp]),
    "cvgram_fold_combo": (_int, [_vp, _i32, _int, _int, _int, _int, _vp, _vp]),
    "cvgram_fold_leaky": (_int, [_vp, _i32, _int, _vp, _vp]),
    "cvgram_ridge": (_int, [_vp, _i32, _i32, ctypes.POINTER(ctypes.c_double), _i32, _vp]),
    "cvgram_folds_all": (_int, [_vp, _i32, _i32, _vp, _vp]),
    "cvgram_folds_all_noalloc": (_int, [_vp, _vp, _vp, _i64, _i64, _i64, _int, _int, _int, _i32,
                                        _vp, _vp, _vp]),
    "cvgram_fold_stats": (_int, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "cvgram_set_stream": (_int, [_vp, _vp]),
    "cvgram_destroy": (_int, [_vp]),
    "cvgram_status_string": (ctypes.c_char_p, [_int]),
    "cvgram_last_error_message": (ctypes.c_char_p, []),
    "cvgram_version": (_i32, []),
    "cvgram_set_stage_timing": (_int, [_int]),
    "cvgram_batch_create": (_int, [_vp, _i32, _int, _int, _int, _vp, ctypes.POINTER(_vp)]),
    "cvgram_batch_run": (_int, [_vp]),
    "cvgram_batch_run_eager": (_int, [_vp]),
    "cvgram_batch_problem_info": (_int, [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "cvgram_batch_destroy": (_int, [_vp]),
    "cvgram_autotune": (_int, [_vp, _vp, _vp, _i64, _i64, _i64, _int, _int, _vp,
                               ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "cvgram_batch_autotune": (_int, [_vp, _i32, _int, _int, _vp, ctypes.POINTER(_i32),
                                     ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                     ctypes.POINTER(ctypes.c_double)]),
    "cvgram_stage_times": (_int, [_vp, ctypes.POINTER(ctypes.c_double), _i32]),
    "cvgram_trim_cache": (_int, []),
}


def load():
    """Load libcvgram.so (built by ``python -m paper_2401_13185_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2401_13185_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def header_symbols() -> list[str]:
    """Function names declared in include/cvgram.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cvgram_[a-z_0-9]+)\s*\(", text)))


def exported_symbols() -> list[str]:
    lib = load()
    return [s for s in header_symbols() if hasattr(lib, s)]


def _check(st: int):
    if st != 0:
        msg = load().cvgram_last_error_message().decode()
        raise CVGramError(st, msg or load().cvgram_status_string(st).decode())


def _torch():
    import torch
    return torch


def _ptr(t, what: str, dtype=None, numel=None):
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous (row-major)")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{what} must have dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what} must have {numel} elements, got {t.numel()}")
    return t.data_ptr()


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


class Handle:
    """Owns a cvgram_t; keeps the input tensors alive while work may use them."""

    def __init__(self, ptr, X, Y, fold_id, N, K, M, mode, stream):
        self.ptr = ptr
        self._keep = (X, Y, fold_id)
        self.N, self.K, self.M = N, K, M
        self.mode = mode
        self.stream = stream
        self.out_dtype = _torch().float64 if mode == "fp64" else _torch().float32
        self.device = X.device

    def __del__(self):
        try:
            if self.ptr:
                cvgram_destroy(self)
        except Exception:
            pass


def cvgram_create(X, Y, fold_id, center_x=0, scale_x=0, center_y=0, scale_y=0, ddof=1,
                  mode="fp64", stream=None) -> Handle:
    torch = _torch()
    lib = load()
    if X.dim() != 2:
        raise ValueError("X must be N x K")
    N, K = X.shape
    if Y is None:
        M = 0
    else:
        if Y.dim() != 2 or Y.shape[0] != N:
            raise ValueError("Y must be N x M")
        M = Y.shape[1]
        if Y.dtype != X.dtype:
            raise TypeError("X and Y must have the same dtype")
    if X.dtype == torch.float64:
        dt = 1
    elif X.dtype == torch.float32:
        dt = 0
    else:
        raise TypeError("X must be float32 or float64")
    if mode not in MODES:
        raise ValueError(f"mode must be one of {sorted(MODES)}")
    xp = _ptr(X, "X")
    yp = _ptr(Y, "Y") if M > 0 else None
    fp = _ptr(fold_id, "fold_id", torch.int32, N)
    s = _stream_ptr(stream)
    out = _vp()
    _check(lib.cvgram_create(xp, yp, fp, N, K, M, dt, int(center_x), int(scale_x), int(center_y),
                             int(scale_y), int(ddof), MODES[mode], s, ctypes.byref(out)))
    return Handle(out.value, X, Y, fold_id, N, K, M, mode, s)


def cvgram_num_folds(h: Handle) -> int:
    P = int(load().cvgram_num_folds(h.ptr))
    if P < 0:
        raise CVGramError(1, cvgram_last_error_message() or "NULL handle")
    return P


def cvgram_plan_info(h: Handle) -> dict:
    """The plan the handle's launch used: tile edge, Gram work items, slabs,
    whether the fused fold path was taken, and the packed panels' bytes per
    element."""
    info = (_i64 * 5)()
    _check(load().cvgram_plan_info(h.ptr, info, 5))
    return {"tile": info[0], "items": info[1], "slabs": info[2], "fused": bool(info[3]),
            "panel_bytes": info[4]}


def cvgram_plan_query(N, K, M, fold_sizes, dtype="f32", mode="fp64") -> dict:
    """The plan cvgram_create would make for this shape and these fold sizes,
    computed on the host (no device work): the cvgram_plan_info fields, the
    device workspace bytes, and the most and fewest Gram items per XCD."""
    if mode not in MODES:
        raise ValueError(f"mode must be one of {sorted(MODES)}")
    if dtype not in ("f32", "f64"):
        raise ValueError("dtype must be 'f32' or 'f64'")
    sizes = (_i64 * len(fold_sizes))(*[int(v) for v in fold_sizes])
    info = (_i64 * 8)()
    _check(load().cvgram_plan_query(N, K, M, sizes, len(fold_sizes), 1 if dtype == "f64" else 0,
                                    MODES[mode], info, 8))
    return {"tile": info[0], "items": info[1], "slabs": info[2], "fused": bool(info[3]),
            "panel_bytes": info[4], "workspace_bytes": info[5], "xcd_items_max": info[6],
            "xcd_items_min": info[7]}


def cvgram_partition(h: Handle, perm=None, offsets=None):
    torch = _torch()
    P = cvgram_num_folds(h)
    if perm is None:
        perm = torch.empty(h.N, dtype=torch.int32, device=h.device)
    if offsets is None:
        offsets = torch.empty(P + 1, dtype=torch.int64, device=h.device)
    _check(load().cvgram_partition(h.ptr, _ptr(perm, "perm", torch.int32, h.N),
                                   _ptr(offsets, "offsets", torch.int64, P + 1)))
    return perm, offsets


def _outs(h: Handle, out_XtX, out_XtY, lead=()):
    torch = _torch()
    if out_XtX is None:
        out_XtX = torch.empty(*lead, h.K, h.K, dtype=h.out_dtype, device=h.device)
    if out_XtY is None and h.M > 0:
        out_XtY = torch.empty(*lead, h.K, h.M, dtype=h.out_dtype, device=h.device)
    n_lead = 1
    for v in lead:
        n_lead *= v
    xp = _ptr(out_XtX, "out_XtX", h.out_dtype, n_lead * h.K * h.K) if out_XtX is not False else None
    yp = (_ptr(out_XtY, "out_XtY", h.out_dtype, n_lead * h.K * h.M)
          if (out_XtY is not None and out_XtY is not False) else None)
    return out_XtX, out_XtY, xp, yp


def cvgram_fold(h: Handle, p: int, out_XtX=None, out_XtY=None):
    out_XtX, out_XtY, xp, yp = _outs(h, out_XtX, out_XtY)
    _check(load().cvgram_fold(h.ptr, int(p), xp, yp))
    return out_XtX, out_XtY


def cvgram_fold_combo(h: Handle, p: int, center_x, scale_x, center_y, scale_y, out_XtX=None,
                      out_XtY=None):
    out_XtX, out_XtY, xp, yp = _outs(h, out_XtX, out_XtY)
    _check(load().cvgram_fold_combo(h.ptr, int(p), int(center_x), int(scale_x), int(center_y),
                                    int(scale_y), xp, yp))
    return out_XtX, out_XtY


def cvgram_fold_leaky(h: Handle, p: int, kind: str, out_XtX=None, out_XtY=None):
    """Leakage comparison for fold p (kind "global" or "lindgren"); see
    include/cvgram.h.  Not training-partition preprocessing."""
    out_XtX, out_XtY, xp, yp = _outs(h, out_XtX, out_XtY)
    _check(load().cvgram_fold_leaky(h.ptr, int(p), LEAK_KINDS[kind], xp, yp))
    return out_XtX, out_XtY


def cvgram_ridge(h: Handle, p_begin: int, p_end: int, lambdas, out_B=None):
    """Ridge coefficients B[f][l] = (XtX_T + lambda_l I)^{-1} XtY_T for folds
    [p_begin, p_end) and the given penalties (FP64, on the device)."""
    torch = _torch()
    lam = [float(v) for v in lambdas]
    n = int(p_end) - int(p_begin)
    if out_B is None:
        out_B = torch.empty(max(n, 0), len(lam), h.K, h.M, dtype=torch.float64, device=h.device)
    bp = _ptr(out_B, "out_B", torch.float64, max(n, 0) * len(lam) * h.K * h.M)
    arr = (ctypes.c_double * max(1, len(lam)))(*lam)
    _check(load().cvgram_ridge(h.ptr, int(p_begin), int(p_end), arr, len(lam), bp))
    return out_B


def cvgram_folds_all(h: Handle, p_begin: int, p_end: int, out_XtX=None, out_XtY=None):
    torch = _torch()
    n = int(p_end) - int(p_begin)
    if out_XtX is None:
        out_XtX = torch.empty(n, XTX_CLASSES, h.K, h.K, dtype=h.out_dtype, device=h.device)
    if out_XtY is None and h.M > 0:
        out_XtY = torch.empty(n, XTY_CLASSES, h.K, h.M, dtype=h.out_dtype, device=h.device)
    xp = _ptr(out_XtX, "out_XtX", h.out_dtype, n * XTX_CLASSES * h.K * h.K) if out_XtX is not False else None
    yp = (_ptr(out_XtY, "out_XtY", h.out_dtype, n * XTY_CLASSES * h.K * h.M)
          if (out_XtY is not None and out_XtY is not False) else None)
    _check(load().cvgram_folds_all(h.ptr, int(p_begin), int(p_end), xp, yp))
    return out_XtX, out_XtY


def cvgram_folds_all_noalloc(X, Y, fold_id, P, out_XtX, out_XtY, ddof=1, mode="fp64",
                             stream=None):
    """Every fold's 12 classes into caller-owned outputs, with the library's
    fixed scratch as workspace (no device allocation by the library).
    out_XtX: [P][4][K][K], out_XtY: [P][8][K][M] (or None), FP64 in mode
    fp64 and FP32 otherwise."""
    torch = _torch()
    if X.dim() != 2:
        raise ValueError("X must be N x K")
    N, K = X.shape
    M = 0 if Y is None else Y.shape[1]
    if Y is not None and (Y.dim() != 2 or Y.shape[0] != N or Y.dtype != X.dtype):
        raise ValueError("Y must be N x M with X's dtype")
    if X.dtype not in (torch.float32, torch.float64):
        raise TypeError("X must be float32 or float64")
    if mode not in MODES:
        raise ValueError(f"mode must be one of {sorted(MODES)}")
    od = torch.float64 if mode == "fp64" else torch.float32
    xp = _ptr(out_XtX, "out_XtX", od, int(P) * XTX_CLASSES * K * K)
    yp = _ptr(out_XtY, "out_XtY", od, int(P) * XTY_CLASSES * K * M) if M > 0 else None
    _check(load().cvgram_folds_all_noalloc(
        _ptr(X, "X"), _ptr(Y, "Y") if M > 0 else None, _ptr(fold_id, "fold_id", torch.int32, N),
        N, K, M, 1 if X.dtype == torch.float64 else 0, int(ddof), MODES[mode], int(P),
        _stream_ptr(stream), xp, yp))
    return out_XtX, out_XtY


def cvgram_fold_stats(h: Handle, p: int):
    torch = _torch()
    f64 = dict(dtype=torch.float64, device=h.device)
    mx, sx = torch.empty(h.K, **f64), torch.empty(h.K, **f64)
    my, sy = torch.empty(h.M, **f64), torch.empty(h.M, **f64)
    _check(load().cvgram_fold_stats(h.ptr, int(p), mx.data_ptr(), sx.data_ptr(),
                                    my.data_ptr() if h.M else None,
                                    sy.data_ptr() if h.M else None))
    return mx, sx, my, sy


def cvgram_set_stream(h: Handle, stream):
    s = _stream_ptr(stream)
    _check(load().cvgram_set_stream(h.ptr, s))
    h.stream = s


def _record_on_stream(tensors, stream_ptr):
    """Mark tensors as in use on the stream `stream_ptr` (torch's allocator
    then keeps their memory until the work queued there has run)."""
    torch = _torch()
    for t in tensors:
        if t is None:
            continue
        st = (torch.cuda.default_stream(t.device) if not stream_ptr
              else torch.cuda.ExternalStream(stream_ptr, device=t.device))
        t.record_stream(st)


def cvgram_destroy(h: Handle):
    if h.ptr:
        ptr, h.ptr = h.ptr, None
        _check(load().cvgram_destroy(ptr))
        # the library does not wait for the handle's queued work: the inputs
        # stay reserved for that work in torch's allocator
        if h._keep is not None:
            _record_on_stream(h._keep, h.stream)
        h._keep = None


def cvgram_set_stage_timing(on: bool):
    _check(load().cvgram_set_stage_timing(1 if on else 0))


STAGES = ("partition", "stats", "gram", "reduce")


def cvgram_stage_times(h: Handle) -> dict:
    """Stage durations (ms) recorded by cvgram_create with timing enabled."""
    ms = (ctypes.c_double * 4)()
    _check(load().cvgram_stage_times(h.ptr, ms, 4))
    return dict(zip(STAGES, list(ms)))


def cvgram_trim_cache():
    _check(load().cvgram_trim_cache())


def cvgram_status_string(status: int) -> str:
    return load().cvgram_status_string(int(status)).decode()


def cvgram_last_error_message() -> str:
    return load().cvgram_last_error_message().decode()


def cvgram_version() -> int:
    return int(load().cvgram_version())


class _Problem(ctypes.Structure):
    _fields_ = [("X", _vp), ("Y", _vp), ("fold_id", _vp), ("N", _i64), ("K", _i64), ("M", _i64),
                ("out_XtX", _vp), ("out_XtY", _vp)]


class Batch:
    """Owns a cvgram_batch_t and the tensors it borrows."""

    def __init__(self, ptr, keep, outs, mode, stream):
        self.ptr = ptr
        self._keep = keep
        self.outs = outs
        self.mode = mode
        self.stream = stream

    def __del__(self):
        try:
            if self.ptr:
                cvgram_batch_destroy(self)
        except Exception:
            pass


def cvgram_batch_create(problems, ddof=1, mode="fp64", stream=None) -> Batch:
    """problems: sequence of (X, Y, fold_id) CUDA tensors (same dtype).  The
    outputs are allocated here: Batch.outs[i] = (XtX [P][4][K][K],
    XtY [P][8][K][M] or None)."""
    torch = _torch()
    lib = load()
    if not problems:
        raise ValueError("need at least one problem")
    dt = problems[0][0].dtype
    if dt not in (torch.float32, torch.float64):
        raise TypeError("X must be float32 or float64")
    if mode not in MODES:
        raise ValueError(f"mode must be one of {sorted(MODES)}")
    odt = torch.float64 if mode == "fp64" else torch.float32
    arr = (_Problem * len(problems))()
    keep, outs = [], []
    for i, (X, Y, f) in enumerate(problems):
        if X.dtype != dt or (Y is not None and Y.dtype != dt):
            raise TypeError("every X and Y of a batch must have the same dtype")
        N, K = X.shape
        M = 0 if Y is None else Y.shape[1]
        P = int(f.max().item()) + 1 if f.numel() else 0
        xx = torch.empty(max(P, 0), XTX_CLASSES, K, K, dtype=odt, device=X.device)
        xy = torch.empty(max(P, 0), XTY_CLASSES, K, M, dtype=odt, device=X.device) if M else None
        arr[i] = _Problem(_ptr(X, "X"), _ptr(Y, "Y") if M else None,
                          _ptr(f, "fold_id", torch.int32, N), N, K, M, xx.data_ptr(),
                          xy.data_ptr() if xy is not None else None)
        keep.append((X, Y, f))
        outs.append((xx, xy))
    s = _stream_ptr(stream)
    out = _vp()
    _check(lib.cvgram_batch_create(arr, len(problems), 1 if dt == torch.float64 else 0, int(ddof),
                                   MODES[mode], s, ctypes.byref(out)))
    return Batch(out.value, keep, outs, mode, s)


def cvgram_batch_autotune(problems, mode="fp64", stream=None):
    """Tune the Gram launches of a batch of (X, Y, fold_id) problems in the
    batch itself; returns (widest tile, smallest K on 256 x 128 tiles (0: the
    built-in rule), target items, Gram-stage ms).  A following
    cvgram_batch_create of these problems uses the choice."""
    torch = _torch()
    if not problems:
        raise ValueError("need at least one problem")
    dt = problems[0][0].dtype
    if dt not in (torch.float32, torch.float64):
        raise TypeError("X must be float32 or float64")
    if mode not in MODES:
        raise ValueError(f"mode must be one of {sorted(MODES)}")
    arr = (_Problem * len(problems))()
    for i, (X, Y, f) in enumerate(problems):
        N, K = X.shape
        M = 0 if Y is None else Y.shape[1]
        arr[i] = _Problem(_ptr(X, "X"), _ptr(Y, "Y") if M else None,
                          _ptr(f, "fold_id", torch.int32, N), N, K, M, None, None)
    tile, wide_k, items, ms = _i32(), _i32(), _i32(), ctypes.c_double()
    _check(load().cvgram_batch_autotune(arr, len(problems), 1 if dt == torch.float64 else 0,
                                        MODES[mode], _stream_ptr(stream), ctypes.byref(tile),
                                        ctypes.byref(wide_k), ctypes.byref(items),
                                        ctypes.byref(ms)))
    return tile.value, wide_k.value, items.value, ms.value


def cvgram_batch_run(b: Batch):
    _check(load().cvgram_batch_run(b.ptr))


def cvgram_batch_run_eager(b: Batch):
    _check(load().cvgram_batch_run_eager(b.ptr))


def cvgram_batch_problem_info(b: Batch, i: int):
    P, sc = _i32(), _i32()
    _check(load().cvgram_batch_problem_info(b.ptr, int(i), ctypes.byref(P), ctypes.byref(sc)))
    return P.value, bool(sc.value)


def cvgram_batch_destroy(b: Batch):
    if b.ptr:
        ptr, b.ptr = b.ptr, None
        _check(load().cvgram_batch_destroy(ptr))
        b._keep = None


def cvgram_autotune(X, Y, fold_id, mode="fp64", stream=None):
    """Tune the grouped Gram launch on this problem; returns (tile, target_items)."""
    torch = _torch()
    N, K = X.shape
    M = 0 if Y is None else Y.shape[1]
    tile, items = _i32(), _i32()
    _check(load().cvgram_autotune(_ptr(X, "X"), _ptr(Y, "Y") if M else None,
                                  _ptr(fold_id, "fold_id", torch.int32, N), N, K, M,
                                  1 if X.dtype == torch.float64 else 0, MODES[mode],
                                  _stream_ptr(stream), ctypes.byref(tile), ctypes.byref(items)))
    return tile.value, items.value


class CVGram:
    """Convenience wrapper: ``with CVGram(X, Y, folds, center_x=1, ...) as cv:
    XtX, XtY = cv.fold(p)``."""

    def __init__(self, X, Y, fold_id, **kw):
        self.h = cvgram_create(X, Y, fold_id, **kw)
        self.P = cvgram_num_folds(self.h)

    def fold(self, p, **kw):
        return cvgram_fold(self.h, p, **kw)

    def fold_combo(self, p, cx, sx, cy, sy, **kw):
        return cvgram_fold_combo(self.h, p, cx, sx, cy, sy, **kw)

    def folds_all(self, p_begin=0, p_end=None, **kw):
        return cvgram_folds_all(self.h, p_begin, self.P if p_end is None else p_end, **kw)

    def stats(self, p):
        return cvgram_fold_stats(self.h, p)

    def partition(self):
        return cvgram_partition(self.h)

    def close(self):
        cvgram_destroy(self.h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
