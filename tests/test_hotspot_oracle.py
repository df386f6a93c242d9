"""The hotspot oracle against its pins, and planted mistakes (on the CPU):
each textual mutant of hotspot_oracle.c must fail at least one pin."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests import hotspot_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "hotspot_oracle.c")

MUTANTS = {
    # the y-direction flow weighted by the x conductance
    "gy_as_gx": ("+ (north + south - 2.0 * t) * gy +", "+ (north + south - 2.0 * t) * gx +"),
    # mirror instead of clamp at the top edge
    "mirror_edge": ("const long rn = clampl(r - 1, 0, rows - 1)", "const long rn = clampl(r > 0 ? r - 1 : 1, 0, rows - 1)"),
    # heat flowing the wrong way through the vertical path
    "sink_sign": ("(t_amb - t) * gz", "(t - t_amb) * gz"),
    # power ignored
    "dropped_power": ("const double flow = (double)power[r * cols + c] +", "const double flow = 0.0 +"),
    # east neighbour two cells away
    "east_offset": ("ce = clampl(c + 1, 0, cols - 1)", "ce = clampl(c + 2, 0, cols - 1)"),
    # rows and columns swapped in the north/south reads
    "transposed": ("north = cur[rn * cols + c], south = cur[rs * cols + c]",
                   "north = cur[c * rows + rn], south = cur[c * rows + rs]"),
    # time step over capacity dropped
    "no_cc": ("nxt[r * cols + c] = t + cc * flow;", "nxt[r * cols + c] = t + flow;"),
    # one step too few
    "steps_off_by_one": ("for (long s = 0; s < steps; ++s) {", "for (long s = 1; s < steps; ++s) {"),
}


def _mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of {name} not unique"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    lib_path = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", *oracle.CFLAGS, str(path), "-o", str(lib_path), "-lm"], check=True)
    lib = ctypes.CDLL(str(lib_path))
    fp, dp, L, D = ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double), ctypes.c_long, ctypes.c_double
    lib.oracle_hotspot_f64.argtypes = [fp, fp, L, L, L, D, D, D, D, D, dp]

    def hs(temp, power, steps, cc, gx, gy, gz, t_amb):
        temp = np.ascontiguousarray(temp, np.float32)
        power = np.ascontiguousarray(power, np.float32)
        out = np.zeros(temp.shape)
        lib.oracle_hotspot_f64(temp.ctypes.data_as(fp), power.ctypes.data_as(fp), temp.shape[0], temp.shape[1],
                               steps, cc, gx, gy, gz, t_amb, out.ctypes.data_as(dp))
        return out
    return hs


def test_real_oracle_passes_every_pin():
    assert pins.run_battery(oracle.hotspot_f64) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    failed = pins.run_battery(_mutant(tmp_path, name, old, new))
    assert failed, f"mutant {name} passed every pin"


def test_argument_errors():
    t = np.zeros((3, 3), np.float32)
    with pytest.raises(ValueError):
        oracle.hotspot_f64(t, np.zeros((3, 4), np.float32), 1, 0.1, 0.1, 0.1, 0.1, 0.0)
    with pytest.raises(ValueError):
        oracle.hotspot_f64(t, t, -1, 0.1, 0.1, 0.1, 0.1, 0.0)
    assert np.array_equal(oracle.hotspot_f64(t + 1, t, 0, 0.1, 0.1, 0.1, 0.1, 0.0), np.ones((3, 3)))
