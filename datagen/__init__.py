"""Seeded synthetic inputs for the direct 2D convolution workloads.

This module is shared by the tests, the benchmark and the CPU oracle checks.
It holds no convolution arithmetic: only counter-based random numbers and the
problem recipes (shapes, halo, value distributions, arrival traces) built on
them.

Generator
---------
SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), used in its counter form: the i-th output of the
stream seeded with ``seed`` is

    mix64(seed + (i + 1) * 0x9E3779B97F4A7C15)      (all arithmetic mod 2**64)

with the published finaliser

    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)

Every element is a pure function of (seed, index), so any element can be
regenerated on its own; the device-side generator of the serving path
implements the same definition independently.

Value maps
----------
* ``uniform_pm1``: k = top 24 bits of the hash, v = (k - 2**23) * 2**-23.
  v lies in [-1, 1 - 2**-23] and is exactly representable in FP32, so host and
  device see the same bits. ("uniform [-1, 1]" read as half-open.)
* ``small_ints``: v = (hash >> 32) mod (2m+1) - m, an integer in [-m, m]
  stored as FP32. With |in|, |f| <= 4 and at most 63*63 taps every partial sum
  of a convolution is an integer below 2**24, so FP32 sums are exact in any
  order.
* ``unit_float``: u = (hash >> 11) * 2**-53 in [0, 1), for shapes and traces.
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Seeds of the standard workloads: input and filter of the plain problem, and
# the per-problem offsets of the batched and served problems.
SEED_INPUT = 1
SEED_FILTER = 2
SEED_BATCH_SHAPES = 3
SEED_ARRIVALS = 4
SEED_SERVING_SAMPLE = 5
SEED_BATCH_INPUT_BASE = 1000
SEED_BATCH_FILTER_BASE = 2000

# Filter sizes drawn by the batched and served workloads.
BATCH_FILTERS = (3, 5, 9, 17)


def splitmix64(seed: int, index: np.ndarray) -> np.ndarray:
    """Return the SplitMix64 outputs number ``index`` (uint64 array) of ``seed``."""
    with np.errstate(over="ignore"):
        idx = np.asarray(index, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (idx + np.uint64(1)) * GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed: int, n: int, start: int = 0) -> np.ndarray:
    """``n`` FP32 values in [-1, 1 - 2**-23], elements ``start .. start+n-1``."""
    z = splitmix64(seed, np.arange(start, start + n, dtype=np.uint64))
    k = (z >> np.uint64(40)).astype(np.int64)
    return ((k - (1 << 23)).astype(np.float64) * 2.0 ** -23).astype(np.float32)


def small_ints(seed: int, n: int, m: int = 4) -> np.ndarray:
    """``n`` integers in [-m, m] as FP32 (exact-arithmetic test data)."""
    z = splitmix64(seed, np.arange(n, dtype=np.uint64))
    k = ((z >> np.uint64(32)) % np.uint64(2 * m + 1)).astype(np.int64) - m
    return k.astype(np.float32)


def unit_float(seed: int, n: int) -> np.ndarray:
    """``n`` float64 values in [0, 1)."""
    z = splitmix64(seed, np.arange(n, dtype=np.uint64))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def conv_problem(out_h: int, out_w: int, fh: int, fw: int, *, seed_in: int = SEED_INPUT,
                 seed_f: int = SEED_FILTER, kind: str = "uniform", zero_halo: bool = False):
    """Input (out_h+fh-1, out_w+fw-1) and filter (fh, fw) FP32 arrays, row-major.

    The input element at (r, c) is hash element r*(out_w+fw-1)+c of ``seed_in``.
    ``zero_halo`` zeroes the outer ring of half-filter width (the 1024x1024 /
    17x17 plain workload: a zero-padded "same" convolution in disguise).
    ``kind`` is "uniform" (U[-1,1)) or "int" (integers in [-4, 4]).
    """
    ih, iw = out_h + fh - 1, out_w + fw - 1
    if kind == "uniform":
        a = uniform_pm1(seed_in, ih * iw).reshape(ih, iw)
        f = uniform_pm1(seed_f, fh * fw).reshape(fh, fw)
    elif kind == "int":
        a = small_ints(seed_in, ih * iw).reshape(ih, iw)
        f = small_ints(seed_f, fh * fw).reshape(fh, fw)
    else:
        raise ValueError(f"unknown kind {kind!r}")
    if zero_halo:
        hy, hx = (fh - 1) // 2, (fw - 1) // 2
        a[:hy, :] = 0
        a[ih - (fh - 1 - hy):, :] = 0
        a[:, :hx] = 0
        a[:, iw - (fw - 1 - hx):] = 0
    return a, f


def log_uniform_sides(seed: int, n: int, lo: int, hi: int) -> np.ndarray:
    """``n`` integer sides round(exp(U[ln lo, ln hi))) (batched and served shapes)."""
    u = unit_float(seed, n)
    s = np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo))))
    return np.clip(s, lo, hi).astype(np.int64)


def filter_choices(seed: int, n: int, choices=BATCH_FILTERS) -> np.ndarray:
    """``n`` draws from ``choices`` using the top bits of the hash of ``seed``."""
    z = splitmix64(seed ^ 0x5A5A5A5A, np.arange(n, dtype=np.uint64))
    idx = ((z >> np.uint64(32)) % np.uint64(len(choices))).astype(np.int64)
    return np.asarray(choices, dtype=np.int64)[idx]


def batch_shapes(n: int = 64, lo: int = 256, hi: int = 2048, seed: int = SEED_BATCH_SHAPES):
    """The batched workload: ``n`` square outputs, sides log-uniform in [lo, hi],
    filters uniform from {3, 5, 9, 17}. Returns a list of (out_h, out_w, fh, fw)."""
    sides = log_uniform_sides(seed, n, lo, hi)
    fs = filter_choices(seed, n)
    return [(int(s), int(s), int(f), int(f)) for s, f in zip(sides, fs)]


def poisson_arrivals(rate_hz: float, duration_s: float, seed: int = SEED_ARRIVALS):
    """Arrival times (s) of a Poisson process of ``rate_hz`` over ``duration_s``:
    inter-arrival gaps -ln(1-u)/rate from the hash stream of ``seed``."""
    if rate_hz <= 0:
        return np.zeros(0)
    n_guess = int(rate_hz * duration_s * 1.5 + 64)
    while True:
        u = unit_float(seed, n_guess)
        t = np.cumsum(-np.log1p(-u) / rate_hz)
        if t[-1] >= duration_s:
            return t[t < duration_s]
        n_guess *= 2


def serving_requests(rate_hz: float, duration_s: float, lo: int = 128, hi: int = 4096,
                     seed: int = SEED_ARRIVALS):
    """The served workload: Poisson arrival times with square output sides
    log-uniform in [lo, hi] and filters from {3, 5, 9, 17}.
    Returns (arrival_s, list of (out_h, out_w, fh, fw))."""
    t = poisson_arrivals(rate_hz, duration_s, seed)
    sides = log_uniform_sides(seed + 7919, len(t), lo, hi)
    fs = filter_choices(seed + 7919, len(t))
    return t, [(int(s), int(s), int(f), int(f)) for s, f in zip(sides, fs)]


def serving_sample(n: int = 160, lo: int = 128, hi: int = 4096, seed: int = SEED_SERVING_SAMPLE):
    """``n`` request shapes drawn like the served workload's (square sides
    log-uniform in [lo, hi], filters from {3, 5, 9, 17}) from a seed of their
    own, so that tuning for serving does not see the served trace."""
    sides = log_uniform_sides(seed, n, lo, hi)
    fs = filter_choices(seed, n)
    return [(int(s), int(s), int(f), int(f)) for s, f in zip(sides, fs)]


# ---------------------------------------------------------------- hotspot workload
# A square silicon chip split into rows x cols cells (the compact thermal RC
# model's setting): side, thickness, conductivity and volumetric heat capacity
# of silicon, ambient, and a peak power density.
CHIP_SIDE_M = 0.016
CHIP_THICKNESS_M = 0.0005
K_SILICON = 100.0          # W / (m K)
CV_SILICON = 1.75e6        # J / (m^3 K)
T_AMBIENT_K = 318.15
PEAK_POWER_W_M2 = 3.0e6
SEED_HOTSPOT_TEMP = 71
SEED_HOTSPOT_POWER = 72


def hotspot_chip(rows: int, cols: int, stability: float = 0.25):
    """(cc, gx, gy, gz, t_amb, p_max) of the chip workload: conductances G =
    k A / d between neighbouring cell centres (A = thickness x cell side,
    d = the other side) and through the thickness to the ambient (A = cell
    area, d = thickness); the time step is `stability` times the explicit
    step's stability limit C / (2 gx + 2 gy + gz), so cc = dt / C =
    stability / (2 gx + 2 gy + gz); p_max is the peak power of one cell."""
    w, h, t = CHIP_SIDE_M / cols, CHIP_SIDE_M / rows, CHIP_THICKNESS_M
    gx = K_SILICON * t * h / w
    gy = K_SILICON * t * w / h
    gz = K_SILICON * w * h / t
    cc = stability / (2 * gx + 2 * gy + gz)
    return cc, gx, gy, gz, T_AMBIENT_K, PEAK_POWER_W_M2 * w * h


def hotspot_problem(rows: int, cols: int, seed_t: int = SEED_HOTSPOT_TEMP, seed_p: int = SEED_HOTSPOT_POWER):
    """FP32 (temp, power) grids and the FP32-rounded coefficients
    (cc, gx, gy, gz, t_amb) of the chip workload: temperatures
    t_amb + 30 K * u, powers p_max * u^2 (few hot cells), u uniform in [0, 1)."""
    cc, gx, gy, gz, t_amb, p_max = hotspot_chip(rows, cols)
    temp = (t_amb + 30.0 * unit_float(seed_t, rows * cols)).astype(np.float32).reshape(rows, cols)
    power = (p_max * unit_float(seed_p, rows * cols) ** 2).astype(np.float32).reshape(rows, cols)
    coeffs = tuple(float(np.float32(v)) for v in (cc, gx, gy, gz, t_amb))
    return temp, power, coeffs
