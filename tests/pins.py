"""Pins for the FP64 convolution oracle: checks against facts that do not come
from the oracle itself (a hand-worked example, closed forms, algebraic
invariants, and library routines that compute the same thing by another
route). ``run_battery(conv)`` applies all of them to any function
``conv(inp, filt) -> (out, S)`` and returns the names of the pins that fail,
so the mutation tests can show that a planted mistake in the oracle is caught.
"""
from __future__ import annotations

import json
import os

import numpy as np
import scipy.signal

import datagen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def pin_worked_example(conv):
    """Hand-worked 3x4 (*) 2x2 example, exact."""
    with open(os.path.join(GOLDEN, "worked_3x4_2x2.json")) as fh:
        g = json.load(fh)
    out, s = conv(np.array(g["input"], np.float32), np.array(g["filter"], np.float32))
    return np.array_equal(out, np.array(g["output"], np.float64)) and \
        np.array_equal(s, np.array(g["abs_sum"], np.float64))


def pin_offcentre_delta(conv):
    """f[a][b] = 1, else 0  =>  out[y][x] = in[y+a][x+b] exactly (indexing, no flip, pitch)."""
    for (H, W, fh, fw, a, b) in [(7, 5, 3, 4, 0, 3), (6, 9, 5, 2, 4, 1), (4, 4, 1, 3, 0, 2),
                                 (5, 3, 3, 1, 2, 0), (3, 8, 4, 5, 1, 3)]:
        inp = datagen.uniform_pm1(11, (H + fh - 1) * (W + fw - 1)).reshape(H + fh - 1, W + fw - 1)
        f = np.zeros((fh, fw), np.float32)
        f[a, b] = 1.0
        out, s = conv(inp, f)
        want = inp[a:a + H, b:b + W].astype(np.float64)
        if out.shape != (H, W) or not np.array_equal(out, want) or not np.array_equal(s, np.abs(want)):
            return False
    return True


def pin_box_constant(conv):
    """Constant image c under a box filter of ones: out = c*fh*fw, S = |c|*fh*fw."""
    for (H, W, fh, fw, c) in [(5, 6, 3, 3, 0.5), (4, 7, 2, 5, -1.25), (3, 3, 4, 1, 2.0)]:
        inp = np.full((H + fh - 1, W + fw - 1), c, np.float32)
        out, s = conv(inp, np.ones((fh, fw), np.float32))
        if not np.array_equal(out, np.full((H, W), c * fh * fw)):
            return False
        if not np.array_equal(s, np.full((H, W), abs(c) * fh * fw)):
            return False
    return True


def pin_box_mean(conv):
    """Box filter 1/(fh*fw) on a constant image returns the constant (to rounding)."""
    inp = np.full((12, 11), 0.75, np.float32)
    out, _ = conv(inp, np.full((5, 4), np.float32(1.0 / 20.0), np.float32))
    return np.allclose(out, 0.75 * 20 * np.float64(np.float32(1.0 / 20.0)), rtol=1e-14, atol=0)


def pin_linearity(conv):
    """conv(p*a + q*b, f) = p conv(a, f) + q conv(b, f), and the same in f."""
    H, W, fh, fw = 9, 7, 4, 3
    n = (H + fh - 1) * (W + fw - 1)
    a = datagen.small_ints(21, n).reshape(H + fh - 1, W + fw - 1)
    b = datagen.small_ints(22, n).reshape(H + fh - 1, W + fw - 1)
    f = datagen.small_ints(23, fh * fw).reshape(fh, fw)
    g = datagen.small_ints(24, fh * fw).reshape(fh, fw)
    p, q = 3.0, -2.0
    lhs, _ = conv((p * a + q * b).astype(np.float32), f)
    ra, _ = conv(a, f)
    rb, _ = conv(b, f)
    if not np.array_equal(lhs, p * ra + q * rb):
        return False
    lhs2, _ = conv(a, (p * f + q * g).astype(np.float32))
    rg, _ = conv(a, g)
    return np.array_equal(lhs2, p * ra + q * rg)


def pin_separable(conv):
    """A rank-1 filter u v^T equals a 1-D pass along rows with v, then along
    columns with u (each 1-D pass by numpy.correlate, 'valid')."""
    H, W, fh, fw = 10, 13, 5, 3
    inp = datagen.small_ints(31, (H + fh - 1) * (W + fw - 1)).reshape(H + fh - 1, W + fw - 1)
    u = np.array([1, -2, 3, 0, 1], np.float32)
    v = np.array([2, 1, -1], np.float32)
    out, _ = conv(inp, np.outer(u, v).astype(np.float32))
    rows = np.stack([np.correlate(r.astype(np.float64), v.astype(np.float64), "valid") for r in inp])
    cols = np.stack([np.correlate(c, u.astype(np.float64), "valid") for c in rows.T]).T
    return np.array_equal(out, cols)


def pin_scipy_correlate(conv):
    """scipy.signal.correlate2d(mode='valid') computes the same cross-correlation:
    exact on integer data, and to FP64 rounding on uniform data; convolve2d with
    the flipped filter gives it too."""
    for (H, W, fh, fw) in [(1, 1, 1, 1), (1, 9, 3, 2), (8, 1, 2, 3), (6, 6, 4, 4), (5, 7, 3, 2),
                           (11, 4, 1, 5), (3, 12, 6, 1), (1, 1, 6, 5)]:
        ih, iw = H + fh - 1, W + fw - 1
        inp = datagen.small_ints(41 + H, ih * iw, m=8).reshape(ih, iw)
        f = datagen.small_ints(42 + W, fh * fw, m=8).reshape(fh, fw)
        out, _ = conv(inp, f)
        want = scipy.signal.correlate2d(inp.astype(np.int64), f.astype(np.int64), mode="valid")
        if out.shape != want.shape or not np.array_equal(out, want.astype(np.float64)):
            return False
        want2 = scipy.signal.convolve2d(inp.astype(np.int64), f[::-1, ::-1].astype(np.int64), mode="valid")
        if not np.array_equal(out, want2.astype(np.float64)):
            return False
    inp, f = datagen.conv_problem(23, 19, 7, 5)
    out, s = conv(inp, f)
    want = scipy.signal.correlate2d(inp.astype(np.float64), f.astype(np.float64), mode="valid")
    abs_want = scipy.signal.correlate2d(np.abs(inp.astype(np.float64)), np.abs(f.astype(np.float64)),
                                        mode="valid")
    return bool(np.all(np.abs(out - want) <= 1e-13 * abs_want) and
                np.all(np.abs(s - abs_want) <= 1e-13 * abs_want))


def pin_abs_sum_bound(conv):
    """|out| <= S everywhere, and S is the correlation of |in| with |f|."""
    inp, f = datagen.conv_problem(17, 21, 6, 3, seed_in=51, seed_f=52)
    out, s = conv(inp, f)
    out_abs, _ = conv(np.abs(inp), np.abs(f))
    return bool(np.all(np.abs(out) <= s * (1 + 1e-15)) and np.allclose(s, out_abs, rtol=1e-15, atol=0))


BATTERY = {
    "worked_example": pin_worked_example,
    "offcentre_delta": pin_offcentre_delta,
    "box_constant": pin_box_constant,
    "box_mean": pin_box_mean,
    "linearity": pin_linearity,
    "separable": pin_separable,
    "scipy_correlate": pin_scipy_correlate,
    "abs_sum_bound": pin_abs_sum_bound,
}


def run_battery(conv):
    """Names of the pins that ``conv`` fails (an exception counts as a failure)."""
    failed = []
    for name, pin in BATTERY.items():
        try:
            ok = pin(conv)
        except Exception:  # a crash or shape error is a failed pin
            ok = False
        if not ok:
            failed.append(name)
    return failed
