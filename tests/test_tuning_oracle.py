"""The tuner-statistics and search-space oracles against closed forms (no GPU)."""
import math

import pytest

from oracle import space, tuning


def test_space_counts():
    # 4 * 5 * 4 * 4 * 2 * 2 = 1280; block_x=128 with block_y=16 is the only
    # product over 1024 threads: 4*4*2*2 = 64 tuples removed.
    assert len(space.product()) == 1280
    assert len(space.restricted()) == 1280 - 64 == 1216
    assert all(c[0] * c[1] <= 1024 for c in space.restricted())
    assert len(set(space.restricted())) == 1216


def test_median_and_impact():
    assert tuning.median([3, 1, 2]) == 2
    assert tuning.median([4, 1, 3, 2]) == 2.5
    # impact = max / median (Table 3 caption): Table 3's MI250X conv numbers
    # give 11460 / 380 = 30.16, printed as 30.1x.
    assert math.floor(10 * 11460 / 380) / 10 == 30.1
    assert tuning.tuning_impact([380, 11460, 100]) == pytest.approx(11460 / 380)
    assert tuning.tuning_impact([1, 2, 3, 4, 100]) == pytest.approx(100 / 3)
    with pytest.raises(ValueError):
        tuning.median([])


def test_gflops_convention():
    # 4096^2 outputs, 17x17 taps, one multiply and one add per tap.
    assert tuning.gflops(4096, 4096, 17, 17, 1.0) == pytest.approx(9.697230848)


def test_winner_tie_break():
    t = {(64, 1, 2, 4, 0, 0): 1.000, (32, 1, 2, 4, 0, 0): 1.004, (16, 1, 1, 1, 0, 0): 1.2}
    assert tuning.pick_winner(t) == (32, 1, 2, 4, 0, 0)          # within 0.5 %: smaller tuple
    assert tuning.pick_winner(t, rel_tie=0.0) == (64, 1, 2, 4, 0, 0)
    assert tuning.top_k(t, 2) == [(64, 1, 2, 4, 0, 0), (32, 1, 2, 4, 0, 0)]


def test_efficiency_and_pp():
    assert tuning.efficiency(50, [10, 50, 100]) == 0.5
    # harmonic mean closed forms
    assert tuning.performance_portability([0.8, 0.8, 0.8]) == pytest.approx(0.8)
    assert tuning.performance_portability([1.0, 0.5]) == pytest.approx(2 / 3)
    assert tuning.performance_portability([1.0, 0.0]) == 0.0


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert tuning.percentile_nearest_rank(v, 50) == 50
    assert tuning.percentile_nearest_rank(v, 99) == 99
    assert tuning.percentile_nearest_rank([5.0], 99) == 5.0
    assert tuning.percentile_nearest_rank([3, 1, 2], 50) == 2


def test_local_search_effort_matches_the_replay():
    """analysis.local_search_effort runs the tuner's local search (synthetic
    cost) and reports, per seed, the evaluation at which the best time so far
    first came within p of the optimum; the oracle's plain replay of the same
    walk gives the same counts."""
    import numpy as np

    import paper_2407_11488_amd as C
    from paper_2407_11488_amd import analysis as A
    rng = np.random.default_rng(11)
    shape = (4096, 4096, 17, 17)
    legal = C.conv2d_space(C.shape(*shape), 1, 0)
    times = {c[:6]: float(rng.lognormal(0, 0.4)) for c in legal}
    ps, seeds, budget = (0.0, 0.05), (3, 4, 5), 300
    got = A.local_search_effort(times, shape, ps=ps, seeds=seeds, max_evals=budget)
    axes = [list(v) for _, v in space.AXES]
    best = min(times.values())
    for p in ps:
        want = []
        for seed in seeds:
            _, order = tuning.local_search({c: times[c[:6]] for c in legal}, legal, axes, budget, seed)
            run, first = float("inf"), None
            for k, c in enumerate(order, 1):
                run = min(run, times[c[:6]])
                if run <= (1 + p) * best:
                    first = k
                    break
            want.append(first)
        assert got[f"p{round(100 * p)}"]["per_seed"] == want
