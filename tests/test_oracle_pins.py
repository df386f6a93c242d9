"""The FP64 oracle against its pins (no GPU)."""
import numpy as np
import pytest

import datagen
import oracle
from tests import pins


@pytest.mark.parametrize("name", sorted(pins.BATTERY))
def test_pin(name):
    assert pins.BATTERY[name](oracle.conv2d_f64), name


def test_points_and_rows_match_full():
    inp, f = datagen.conv_problem(37, 29, 9, 5, seed_in=61, seed_f=62)
    full, s = oracle.conv2d_f64(inp, f)
    ys = np.array([0, 36, 17, 5, 36, 0])
    xs = np.array([0, 28, 13, 27, 0, 28])
    v, sv = oracle.conv2d_points_f64(inp, f, ys, xs)
    assert np.array_equal(v, full[ys, xs]) and np.array_equal(sv, s[ys, xs])
    band, sb = oracle.conv2d_rows_f64(inp, f, 11, 30)
    assert np.array_equal(band, full[11:30]) and np.array_equal(sb, s[11:30])


def test_edge_shapes():
    # Filter as large as the input: a single output, the full dot product.
    inp = datagen.small_ints(71, 6 * 5).reshape(6, 5)
    f = datagen.small_ints(72, 6 * 5).reshape(6, 5)
    out, _ = oracle.conv2d_f64(inp, f)
    assert out.shape == (1, 1) and out[0, 0] == float(np.sum(inp.astype(np.int64) * f.astype(np.int64)))
    # Empty output rows are legal and produce an empty result.
    out, _ = oracle.conv2d_f64(np.zeros((2, 7), np.float32), np.ones((3, 2), np.float32))
    assert out.shape == (0, 6)


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.conv2d_f64(np.zeros((2, 2), np.float32), np.zeros((4, 4), np.float32))
    with pytest.raises(ValueError):
        oracle.conv2d_points_f64(np.zeros((4, 4), np.float32), np.ones((2, 2), np.float32), [3], [0])


def test_zero_halo_workload_is_same_convolution():
    """The 1024x1024/17x17 plain workload zeroes an 8-pixel ring of the input,
    which makes it a zero-padded 'same' correlation of the interior (checked
    on a small analogue against scipy's mode='same')."""
    inp, f = datagen.conv_problem(20, 24, 5, 5, zero_halo=True)
    assert np.all(inp[:2] == 0) and np.all(inp[-2:] == 0) and np.all(inp[:, :2] == 0) and np.all(inp[:, -2:] == 0)
    out, _ = oracle.conv2d_f64(inp, f)
    inner = inp[2:-2, 2:-2].astype(np.float64)
    import scipy.signal
    want = scipy.signal.correlate2d(inner, f.astype(np.float64), mode="same")
    assert np.allclose(out, want, rtol=0, atol=1e-12)


def test_normalized_error_definition():
    ref = np.array([1.0, 0.0, -2.0])
    s = np.array([4.0, 0.0, 2.0])
    assert oracle.normalized_error(np.array([1.5, 0.0, -2.0]), ref, s) == 0.125
    assert oracle.normalized_error(np.array([1.0, 1e-30, -2.0]), ref, s) == float("inf")
    assert oracle.normalized_error(np.array([np.nan, 0.0, -2.0]), ref, s) == float("inf")
