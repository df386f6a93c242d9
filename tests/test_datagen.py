"""The seeded input generator (no GPU)."""
import numpy as np

import datagen


def test_splitmix64_reference_values():
    # First outputs of SplitMix64 seeded with 0 and with 1234567, as printed by
    # the reference C implementation of the generator (Vigna, splitmix64.c):
    # next() adds the golden gamma to the state, then applies the finaliser.
    z = datagen.splitmix64(0, np.arange(3))
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    z = datagen.splitmix64(1234567, np.arange(5))
    assert [int(v) for v in z] == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                                   4593380528125082431, 16408922859458223821]


def test_uniform_range_and_exactness():
    v = datagen.uniform_pm1(1, 200000)
    assert v.dtype == np.float32
    assert v.min() >= -1.0 and v.max() <= 1.0 - 2.0 ** -23
    k = v.astype(np.float64) * 2 ** 23
    assert np.array_equal(k, np.round(k))          # multiples of 2^-23: exact in FP32
    assert abs(float(v.mean())) < 0.01 and abs(float(v.var()) - 1 / 3) < 0.01


def test_streams_are_positional():
    a = datagen.uniform_pm1(5, 100)
    b = datagen.uniform_pm1(5, 40, start=60)
    assert np.array_equal(a[60:], b)
    assert not np.array_equal(datagen.uniform_pm1(1, 100), datagen.uniform_pm1(2, 100))


def test_small_ints():
    v = datagen.small_ints(9, 10000)
    assert set(np.unique(v).tolist()) == set(range(-4, 5))


def test_batch_shapes_recipe():
    shapes = datagen.batch_shapes()
    assert len(shapes) == 64
    sides = np.array([s[0] for s in shapes])
    assert sides.min() >= 256 and sides.max() <= 2048
    assert {s[2] for s in shapes} <= {3, 5, 9, 17} and all(s[2] == s[3] for s in shapes)
    assert datagen.batch_shapes() == shapes          # deterministic


def test_poisson_trace():
    t, shapes = datagen.serving_requests(50.0, 20.0)
    assert np.all(np.diff(t) > 0) and t[-1] < 20.0
    assert abs(len(t) - 1000) < 150                  # ~ rate * duration
    assert all(128 <= s[0] <= 4096 for s in shapes)
