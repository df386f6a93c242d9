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


def test_results_analysis_matches_the_statistics_oracle(tmp_path):
    """The product's results-database analysis (NEXT-1: impact, percentiles,
    application efficiency, performance portability and the most portable
    configuration over shapes) against the statistics oracle computed
    directly from the same synthetic times; failed points are ignored."""
    import json

    import numpy as np

    from paper_2407_11488_amd import analysis as A
    rng = np.random.default_rng(5)
    configs = [(bx, by, tx, 1, 0, 0, 1) for bx in (16, 32, 64, 128) for by in (1, 2, 4) for tx in (1, 2, 4, 8)]
    shapes = [(512, 512, 3, 3), (512, 512, 9, 9), (512, 512, 17, 17)]
    dbs, times = {}, {}
    for s in shapes:
        db = tmp_path / f"r_{s[2]}.jsonl"
        t = {c: float(rng.lognormal(0, 0.5)) for c in configs}
        failed = set(configs[3::11])
        with open(db, "w") as fh:
            for c in configs:
                st = "verify" if c in failed else "ok"
                fh.write(json.dumps({"arch": "gfx950", "src": "x", "shape": list(s), "config": list(c),
                                     "status": st, "ms": t[c] if st == "ok" else 0.0}) + "\n")
        dbs[s] = str(db)
        times[s] = {c: v for c, v in t.items() if c not in failed}
    for s in shapes:
        perf = {c: tuning.gflops(*s, ms * 1e-3) for c, ms in times[s].items()}
        assert A.impact(dbs[s], s) == pytest.approx(tuning.tuning_impact(list(perf.values())), rel=1e-12)
        best = max(perf.values())
        pc = A.percentiles(dbs[s], s)
        for q in (10, 25, 50, 75, 90):
            assert pc[f"p{q}"] == pytest.approx(tuning.percentile_nearest_rank(list(perf.values()), q) / best,
                                                abs=5e-5)
        c0 = next(iter(times[s]))
        e = A.efficiency_of(dbs[s], s, c0)["efficiency"]
        assert e == pytest.approx(tuning.efficiency(perf[c0], list(perf.values())), abs=5e-5)
    cfg, row = A.most_portable(dbs)
    common = set.intersection(*(set(times[s]) for s in shapes))

    def pp(c):
        effs = []
        for s in shapes:
            perf = {k: tuning.gflops(*s, ms * 1e-3) for k, ms in times[s].items()}
            effs.append(tuning.efficiency(perf[c], list(perf.values())))
        return tuning.performance_portability(effs)
    want = max(sorted(common), key=pp)
    assert cfg == want and row["pp"] == pytest.approx(pp(want), rel=1e-12)
