"""Pins for the FP64 hotspot oracle: facts that do not come from the oracle
itself (a hand-worked step, the closed form of a uniform grid, conservation of
heat, the cosine eigenmodes of the reflecting-boundary Laplacian, the maximum
principle, superposition). ``run_battery(hs)`` applies them to any function
``hs(temp, power, steps, cc, gx, gy, gz, t_amb) -> grid`` and returns the names
of the pins that fail, so planted mistakes in the oracle can be shown caught.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

import datagen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def pin_worked_step(hs):
    """Hand-worked single step on a 2x3 grid (gx != gy, every edge case)."""
    with open(os.path.join(GOLDEN, "hotspot_2x3_one_step.json")) as fh:
        g = json.load(fh)
    got = hs(np.array(g["temp"], np.float32), np.array(g["power"], np.float32), g["steps"], g["cc"], g["gx"],
             g["gy"], g["gz"], g["t_amb"])
    return np.array_equal(got, np.array(g["result"], np.float64))


def pin_ambient_equilibrium(hs):
    """Every cell at the ambient temperature and no power: nothing changes."""
    t = np.full((9, 13), 318.5, np.float32)
    got = hs(t, np.zeros_like(t), 25, 0.2, 0.7, 0.4, 0.05, 318.5)
    return np.array_equal(got, t.astype(np.float64))


def pin_uniform_closed_form(hs):
    """A uniform grid stays uniform (no lateral flow) and follows the linear
    recurrence T <- a T + b, a = 1 - cc gz, b = cc (p + gz t_amb), whose n-th
    term is a^n T0 + b (1 - a^n) / (1 - a)."""
    for (rows, cols, t0, p, cc, gz, amb, n) in [(6, 11, 300.0, 2.5, 0.1, 0.3, 280.0, 17),
                                                (1, 5, 10.0, 0.0, 0.5, 1.0, 20.0, 4),
                                                (7, 1, -3.0, 1.0, 0.25, 0.5, 0.0, 9)]:
        t = np.full((rows, cols), t0, np.float32)
        pw = np.full((rows, cols), p, np.float32)
        got = hs(t, pw, n, cc, 0.9, 0.6, gz, amb)
        a, b = 1.0 - cc * gz, cc * (p + gz * amb)
        want = a ** n * t0 + b * (1.0 - a ** n) / (1.0 - a)
        if got.shape != (rows, cols) or np.max(np.abs(got - want)) > 1e-12 * max(1.0, abs(want)):
            return False
    return True


def pin_heat_conservation(hs):
    """No vertical sink (gz = 0): the lateral fluxes cancel in pairs (no heat
    crosses the chip's sides), so the total rises by cc * sum(P) per step."""
    for (rows, cols, n) in [(8, 5, 6), (3, 16, 11), (1, 9, 4), (12, 1, 5)]:
        t = 300.0 + 40.0 * datagen.unit_float(21, rows * cols).reshape(rows, cols).astype(np.float32)
        pw = datagen.unit_float(22, rows * cols).reshape(rows, cols).astype(np.float32)
        t = t.astype(np.float32)
        cc = 0.15
        got = hs(t, pw, n, cc, 0.8, 0.5, 0.0, 280.0)
        want = float(np.sum(t.astype(np.float64))) + n * cc * float(np.sum(pw.astype(np.float64)))
        if abs(float(np.sum(got)) - want) > 1e-10 * abs(want):
            return False
    return True


def pin_cosine_modes(hs):
    """With the reflecting boundary (outside neighbour = the cell itself), the
    grid cos(pi k (r + 1/2) / rows) cos(pi m (c + 1/2) / cols) is an
    eigenvector of the step with P = gz = 0: one step multiplies it by
    1 - 4 cc (gy sin^2(pi k / 2 rows) + gx sin^2(pi m / 2 cols)). A constant
    offset is unchanged. Rectangular grid and gx != gy tell rows from columns."""
    rows, cols, cc, gx, gy, n = 10, 7, 0.1, 1.0, 0.45, 5
    r = (np.arange(rows) + 0.5)[:, None]
    c = (np.arange(cols) + 0.5)[None, :]
    for (k, m) in [(1, 0), (0, 2), (3, 1), (2, 5)]:
        mode = np.cos(math.pi * k * r / rows) * np.cos(math.pi * m * c / cols)
        t = (50.0 + 8.0 * mode).astype(np.float32)
        lam = 1.0 - 4.0 * cc * (gy * math.sin(math.pi * k / (2 * rows)) ** 2 +
                                gx * math.sin(math.pi * m / (2 * cols)) ** 2)
        got = hs(t, np.zeros_like(t), n, cc, gx, gy, 0.0, 0.0)
        t64 = t.astype(np.float64)
        want = 50.0 + (t64 - 50.0) * lam ** n   # the FP32 input is the mode up to rounding of each cell
        # the rounding of the FP32 input is not an eigenvector: allow its own evolution (bounded by its size)
        if np.max(np.abs(got - want)) > 1e-5:
            return False
    return True


def pin_maximum_principle(hs):
    """No power and no sink, stable step (cc (2 gx + 2 gy) <= 1): every new
    value is a convex combination of old ones, so the maximum never rises and
    the minimum never falls."""
    t = datagen.uniform_pm1(31, 11 * 14).reshape(11, 14).astype(np.float32) * 50.0
    t = t.astype(np.float32)
    hi, lo = float(t.max()), float(t.min())
    for n in (1, 3, 10):
        got = hs(t, np.zeros_like(t), n, 0.2, 1.0, 1.5, 0.0, 0.0)
        if got.max() > hi or got.min() < lo:
            return False
    return True


def pin_superposition(hs):
    """The step is affine, linear in (T, P, t_amb) together: the result for
    the sums of two inputs is the sum of the results (small integers, so the
    FP32 sums are exact)."""
    rows, cols = 6, 9
    t1 = datagen.small_ints(41, rows * cols).reshape(rows, cols)
    t2 = datagen.small_ints(42, rows * cols).reshape(rows, cols)
    p1 = datagen.small_ints(43, rows * cols).reshape(rows, cols)
    p2 = datagen.small_ints(44, rows * cols).reshape(rows, cols)
    a = hs(t1, p1, 7, 0.125, 0.5, 0.75, 0.25, 3.0)
    b = hs(t2, p2, 7, 0.125, 0.5, 0.75, 0.25, -1.0)
    ab = hs((t1 + t2).astype(np.float32), (p1 + p2).astype(np.float32), 7, 0.125, 0.5, 0.75, 0.25, 2.0)
    return np.max(np.abs(ab - (a + b))) <= 1e-12 * max(1.0, float(np.max(np.abs(ab))))


PINS = {
    "worked_step": pin_worked_step,
    "ambient_equilibrium": pin_ambient_equilibrium,
    "uniform_closed_form": pin_uniform_closed_form,
    "heat_conservation": pin_heat_conservation,
    "cosine_modes": pin_cosine_modes,
    "maximum_principle": pin_maximum_principle,
    "superposition": pin_superposition,
}


def run_battery(hs):
    return [name for name, pin in PINS.items() if not pin(hs)]
