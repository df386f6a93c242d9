"""Planted mistakes in the oracle (on the CPU): each mutant of conv2d_oracle.c
must fail at least one pin, so a plausible slip in the oracle cannot pass
unnoticed. The mutants are textual edits of the real source, compiled to a
temporary library with the same flags."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "conv2d_oracle.c")

MUTANTS = {
    # filter flip (true convolution instead of correlation)
    "flip": ("double w = (double)frow[j];", "double w = (double)f[(fh - 1 - i) * fw + (fw - 1 - j)];"),
    # input pitch from the wrong axis (transposed operand)
    "pitch_axis": ("const long pitch = out_w + fw - 1;\n#pragma omp parallel for schedule(static)\n    for (long y = 0; y < out_h; ++y) {\n        for (long x = 0; x < out_w; ++x) {\n            double v, a;\n            one_point(in, f, pitch, fh, fw, y, x, &v, &a);\n            out[y * out_w + x] = v;",
                   "const long pitch = out_h + fh - 1;\n#pragma omp parallel for schedule(static)\n    for (long y = 0; y < out_h; ++y) {\n        for (long x = 0; x < out_w; ++x) {\n            double v, a;\n            one_point(in, f, pitch, fh, fw, y, x, &v, &a);\n            out[y * out_w + x] = v;"),
    # dropped first filter column
    "dropped_tap": ("for (long j = 0; j < fw; ++j) {", "for (long j = 1; j < fw; ++j) {"),
    # filter row stride from the wrong dimension
    "filter_stride": ("const float *frow = f + i * fw;", "const float *frow = f + i * fh;"),
    # sign lost in the absolute sum
    "abs_sum_sign": ("a += fabs(v) * fabs(w);", "a += v * w;"),
    # input row offset uses x and y swapped
    "xy_swap": ("const float *row = in + (y + i) * pitch + x;", "const float *row = in + (x + i) * pitch + y;"),
    # single precision accumulation
    "fp32_acc": ("double s = 0.0, a = 0.0;", "float s = 0.0f; double a = 0.0;"),
}


def _compile_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of {name} not unique"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", *oracle.CFLAGS, str(path), "-o", str(lib), "-lm"], check=True)
    return ctypes.CDLL(str(lib))


def _wrap(lib):
    fp, dp, L = ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double), ctypes.c_long
    lib.oracle_conv2d_f64.argtypes = [fp, fp, L, L, L, L, dp, dp]

    def conv(inp, filt):
        inp = np.ascontiguousarray(inp, np.float32)
        filt = np.ascontiguousarray(filt, np.float32)
        fh, fw = filt.shape
        H, W = inp.shape[0] - fh + 1, inp.shape[1] - fw + 1
        out = np.zeros((H, W))
        s = np.zeros((H, W))
        lib.oracle_conv2d_f64(inp.ctypes.data_as(fp), filt.ctypes.data_as(fp), H, W, fh, fw,
                              out.ctypes.data_as(dp), s.ctypes.data_as(dp))
        return out, s
    return conv


def test_real_oracle_passes_every_pin():
    assert pins.run_battery(oracle.conv2d_f64) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    conv = _wrap(_compile_mutant(tmp_path, name, old, new))
    failed = pins.run_battery(conv)
    assert failed, f"mutant {name} passed every pin"
