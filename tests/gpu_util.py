"""Helpers for the GPU tests: device buffers from seeded host arrays, runs
through the C ABI, and comparison against the FP64 oracle."""
from __future__ import annotations

import concurrent.futures as cf
import sys

import numpy as np

TOL = 1e-5  # max |gpu - oracle| / sum |f||in|, per output point


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test without a GPU")
    return torch


def to_dev(a):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def nan_like(h, w):
    torch = torch_cuda()
    return torch.full((h, w), float("nan"), dtype=torch.float32, device="cuda")


def run_config(C, inp, filt, cfg, out=None):
    """Runs one configuration through conv2d_plan/conv2d_run on NaN-prefilled output."""
    torch = torch_cuda()
    fh, fw = filt.shape
    H, W = inp.shape[0] - fh + 1, inp.shape[1] - fw + 1
    s = C.shape(H, W, fh, fw)
    plan = C.conv2d_plan(s, cfg)
    try:
        if out is None:
            out = nan_like(H, W)
        C.conv2d_run(plan, inp.data_ptr(), filt.data_ptr(), out.data_ptr(),
                     torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
    finally:
        C.conv2d_destroy(plan)
    return out


def precompile(C, shape, cfgs, vin, vout, threads=16):
    """Compiles configurations in parallel (ctypes releases the GIL) so that the
    plans of a test hit the code-object cache."""
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda c: C.conv2d_compile(shape, c, vin, vout), cfgs))


VEC = 4   # load and store vector width of every plan (rows of any width)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def hip_runtime():
    """The HIP runtime this process already uses (the one torch loaded)."""
    import ctypes
    with open("/proc/self/maps") as fh:
        paths = sorted({ln.split()[-1] for ln in fh if "libamdhip64" in ln})
    assert len(paths) == 1, paths
    hip = ctypes.CDLL(paths[0])
    hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    hip.hipFree.argtypes = [ctypes.c_void_p]
    return hip


def hip_malloc(nbytes):
    """A device allocation of exactly `nbytes` (torch's caching allocator
    would hand out a slice of a larger segment); free with hip_free."""
    import ctypes
    torch_cuda().cuda.synchronize()
    p = ctypes.c_void_p()
    assert hip_runtime().hipMalloc(ctypes.byref(p), nbytes) == 0
    return p.value


def hip_free(ptr):
    hip_runtime().hipFree(ptr)
