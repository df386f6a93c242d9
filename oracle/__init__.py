"""CPU oracles for the direct 2D convolution and the hotspot stencil — TEST
INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The HIP library never calls it, and the
two share no code: the only common module is ``datagen`` (seeded inputs, no
convolution arithmetic).

* ``conv2d_f64`` / ``conv2d_points_f64`` / ``conv2d_rows_f64``: the plain FP64
  definition of the convolution (see ``conv2d_oracle.c``), parallel over rows.
* ``hotspot_f64``: the hotspot thermal stencil (see ``hotspot_oracle.c``), FP64
  explicit steps from FP32 inputs.
* ``oracle.tuning``: the tuner's statistics (tuning impact, median, top-k,
  application efficiency, performance portability), written from their
  definitions in the paper's Section 4.
* ``oracle.space``: the search space and its restriction, by plain enumeration.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "conv2d_oracle.c"), os.path.join(_HERE, "hotspot_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle_conv2d.so")

CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-std=c11", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc; returns the library path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", *CFLAGS, *_SRCS, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(p) for p in _SRCS):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        fp, dp, lp = (ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double),
                      ctypes.POINTER(ctypes.c_long))
        L = ctypes.c_long
        lib.oracle_conv2d_f64.argtypes = [fp, fp, L, L, L, L, dp, dp]
        lib.oracle_conv2d_points_f64.argtypes = [fp, fp, L, L, L, L, lp, lp, L, dp, dp]
        lib.oracle_conv2d_rows_f64.argtypes = [fp, fp, L, L, L, L, L, L, dp, dp]
        for fn in (lib.oracle_conv2d_f64, lib.oracle_conv2d_points_f64, lib.oracle_conv2d_rows_f64):
            fn.restype = ctypes.c_int
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_num_threads.restype = None
        D = ctypes.c_double
        lib.oracle_hotspot_f64.argtypes = [fp, fp, L, L, L, D, D, D, D, D, dp]
        lib.oracle_hotspot_f64.restype = ctypes.c_int
        _lib = lib
    return _lib


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _dptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(inp, filt):
    inp = np.ascontiguousarray(inp, dtype=np.float32)
    filt = np.ascontiguousarray(filt, dtype=np.float32)
    if inp.ndim != 2 or filt.ndim != 2:
        raise ValueError("input and filter must be 2-D")
    fh, fw = filt.shape
    out_h, out_w = inp.shape[0] - fh + 1, inp.shape[1] - fw + 1
    if out_h < 0 or out_w < 0:
        raise ValueError("filter larger than input")
    return inp, filt, out_h, out_w, fh, fw


def conv2d_f64(inp, filt, with_abs: bool = True):
    """Full FP64 oracle. Returns (out, S) (S is None unless ``with_abs``)."""
    inp, filt, H, W, fh, fw = _check(inp, filt)
    out = np.empty((H, W), np.float64)
    s = np.empty((H, W), np.float64) if with_abs else None
    rc = _load().oracle_conv2d_f64(_fptr(inp), _fptr(filt), H, W, fh, fw, _dptr(out), _dptr(s))
    if rc != 0:
        raise ValueError("oracle_conv2d_f64 rejected its arguments")
    return out, s


def conv2d_points_f64(inp, filt, ys, xs):
    """FP64 oracle at points (ys[k], xs[k]). Returns (values, S)."""
    inp, filt, H, W, fh, fw = _check(inp, filt)
    ys = np.ascontiguousarray(ys, dtype=np.int64)
    xs = np.ascontiguousarray(xs, dtype=np.int64)
    n = ys.size
    out = np.empty(n, np.float64)
    s = np.empty(n, np.float64)
    rc = _load().oracle_conv2d_points_f64(_fptr(inp), _fptr(filt), H, W, fh, fw,
                                          ys.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                                          xs.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                                          n, _dptr(out), _dptr(s))
    if rc != 0:
        raise ValueError("oracle_conv2d_points_f64 rejected its arguments")
    return out, s


def conv2d_rows_f64(inp, filt, y0: int, y1: int):
    """FP64 oracle for output rows [y0, y1). Returns (out, S) of shape (y1-y0, W)."""
    inp, filt, H, W, fh, fw = _check(inp, filt)
    out = np.empty((y1 - y0, W), np.float64)
    s = np.empty((y1 - y0, W), np.float64)
    rc = _load().oracle_conv2d_rows_f64(_fptr(inp), _fptr(filt), H, W, fh, fw, y0, y1,
                                        _dptr(out), _dptr(s))
    if rc != 0:
        raise ValueError("oracle_conv2d_rows_f64 rejected its arguments")
    return out, s


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of later oracle calls (timing only; results do not change)."""
    _load().oracle_set_num_threads(int(n))


def normalized_error(gpu, ref, abs_sum):
    """Per-point normalised error max |gpu - ref| / S, with S = sum |f||in|.

    Where S == 0 the exact result is 0 and the GPU value must be exactly 0
    (reported as +inf otherwise)."""
    gpu = np.asarray(gpu, np.float64)
    diff = np.abs(gpu - ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(abs_sum > 0, diff / np.where(abs_sum > 0, abs_sum, 1.0),
                     np.where(diff == 0, 0.0, np.inf))
    if not np.all(np.isfinite(gpu)):
        return float("inf")
    return float(e.max()) if e.size else 0.0


def time_conv2d(inp, filt, repeats: int = 1):
    """Wall time (s, best of ``repeats``) of the full oracle on this host."""
    best = float("inf")
    for _ in range(repeats):
        t0 = time.perf_counter()
        conv2d_f64(inp, filt, with_abs=False)
        best = min(best, time.perf_counter() - t0)
    return best


def hotspot_f64(temp, power, steps: int, cc: float, gx: float, gy: float, gz: float, t_amb: float):
    """The hotspot grid after ``steps`` explicit steps (FP64 result) from FP32
    ``temp`` and ``power`` (rows x cols); coefficients as in hotspot_oracle.c."""
    temp = np.ascontiguousarray(temp, dtype=np.float32)
    power = np.ascontiguousarray(power, dtype=np.float32)
    if temp.ndim != 2 or temp.shape != power.shape:
        raise ValueError("temp and power must be 2-D arrays of one shape")
    rows, cols = temp.shape
    out = np.empty((rows, cols), np.float64)
    rc = _load().oracle_hotspot_f64(_fptr(temp), _fptr(power), rows, cols, int(steps), float(cc), float(gx),
                                    float(gy), float(gz), float(t_amb), _dptr(out))
    if rc != 0:
        raise ValueError("oracle_hotspot_f64 rejected its arguments")
    return out
