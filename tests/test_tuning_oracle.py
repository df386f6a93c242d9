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


# ------------------------------------------------ local search, worked by hand
#
# A 4 x 3 lattice (axes a in 0..3, b in 0..2; enumeration order (0,0), (0,1),
# ..., (3,2)); point (3,1) fails. Times:
#
#          b=0   b=1   b=2
#   a=0    5     4     6
#   a=1    7     3     8
#   a=2    9     2     7
#   a=3    1.5   fail  10
#
# Seed 1. Restart k starts at the idx-th unevaluated point in enumeration
# order, idx = splitmix64(1, k) mod count (the counter-form values are
# 0x910a2dec89025cc1, 0xbeeb8da1658eec67, 0xf893a2eefb32555e,
# 0x71c18690ee42c90b: mod 12 = 5, mod 3 = 1, mod 2 = 0, mod 1 = 0).
#
# restart 0: 12 fresh, idx 5 -> (1,2) = 8. Its neighbours, axis by axis,
#   lower value first: (0,2) = 6, (2,2) = 7, (1,1) = 3 (no (1,3)); the best,
#   (1,1), improves -> move.  (1,1): new neighbours (0,1) = 4, (2,1) = 2,
#   (1,0) = 7 ((1,2) already known); best (2,1) = 2 < 3 -> move.  (2,1): new
#   (3,1) fails, (2,0) = 9; known (1,1) = 3, (2,2) = 7; best 3 is not below 2
#   -> local minimum. 9 evaluations.
# restart 1: fresh (0,0), (3,0), (3,2); idx 1 -> (3,0) = 1.5. Neighbours
#   (2,0) = 9 and (3,1) failed: no move. 10 evaluations.
# restart 2: fresh (0,0), (3,2); idx 0 -> (0,0) = 5, then (0,1) = 4 -> (1,1)
#   -> (2,1), all known: no new evaluation. 11 evaluations.
# restart 3: fresh (3,2); idx 0 -> (3,2) = 10 -> (2,2) -> (2,1). 12, and no
#   fresh point is left.
#
# A first-improvement walk would leave (1,2) for (0,2), the first improving
# neighbour, and evaluate (0,0) sixth instead of (2,1).

HAND_AXES = [[0, 1, 2, 3], [0, 1, 2]]
HAND_LEGAL = [(a, b) for a in range(4) for b in range(3)]
HAND_TIMES = {(0, 0): 5.0, (0, 1): 4.0, (0, 2): 6.0, (1, 0): 7.0, (1, 1): 3.0, (1, 2): 8.0,
              (2, 0): 9.0, (2, 1): 2.0, (2, 2): 7.0, (3, 0): 1.5, (3, 1): None, (3, 2): 10.0}
HAND_ORDER = [(1, 2), (0, 2), (2, 2), (1, 1), (0, 1), (2, 1), (1, 0), (3, 1), (2, 0), (3, 0), (0, 0), (3, 2)]


def _hand_case_holds(local_search):
    """True when a local-search implementation reproduces every figure of the
    walk worked by hand above."""
    for budget, best in ((100, (3, 0)), (12, (3, 0)), (10, (3, 0)), (9, (2, 1)), (4, (1, 1)), (1, (1, 2))):
        got_best, order = local_search(HAND_TIMES, HAND_LEGAL, HAND_AXES, budget, 1)
        if order != HAND_ORDER[:budget] or got_best != best:
            return False
    return True


def test_splitmix_restart_indices_of_the_hand_case():
    import numpy as np

    from datagen import splitmix64
    z = [int(v) for v in splitmix64(1, np.arange(4, dtype=np.uint64))]
    assert z == [0x910a2dec89025cc1, 0xbeeb8da1658eec67, 0xf893a2eefb32555e, 0x71c18690ee42c90b]
    assert (z[0] % 12, z[1] % 3, z[2] % 2, z[3] % 1) == (5, 1, 0, 0)


def test_local_search_walk_worked_by_hand():
    assert _hand_case_holds(tuning.local_search)


def _mutant(old: str, new: str):
    """tuning.local_search with one line of its source replaced."""
    import inspect
    import textwrap
    src = textwrap.dedent(inspect.getsource(tuning.local_search))
    assert src.count(old) == 1, old
    ns = {"np": __import__("numpy")}
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    return ns["local_search"]


@pytest.mark.parametrize("old,new", [
    # first improvement: move to the first improving neighbour in order
    ("nxt = min(ok, key=lambda c: (state[c], c))",
     "nxt = next((n for n in ok if state[n] < state[cur]), cur)"),
    # restart index off by one
    ("np.array([restart], dtype=np.uint64)", "np.array([restart + 1], dtype=np.uint64)"),
    # start counted over every legal point instead of the unevaluated ones
    ("cur = fresh[z % len(fresh)]", "cur = legal[z % len(legal)]"),
    # neighbours higher value first
    ("for q in (pos - 1, pos + 1):", "for q in (pos + 1, pos - 1):"),
    # every restart from the stream's first value
    ("np.array([restart], dtype=np.uint64)", "np.array([0], dtype=np.uint64)"),
    # the last point evaluated reported instead of the best
    ("return min(ok, key=lambda c: (state[c], c)), order", "return order[-1], order"),
])
def test_local_search_mutants_fail_the_hand_case(old, new):
    assert not _hand_case_holds(_mutant(old, new))


# ------------------------------------------------ hotspot space, counted by hand
#
# Axes: block_x in {16, 32, 64, 128, 256}, block_y in {1, 2, 4, 8, 16},
# tile_x, tile_y in {1, 2, 4}, temporal in {1, 2, 3, 4, 6, 8}, and two on/off
# switches (step-loop unroll, power on chip) that no restriction reads (x4).
# Restrictions: 64 <= block_x*block_y <= 1024; the region of
# (block_y*tile_y) x (block_x*tile_x) cells larger than 2*temporal on both axes.
#
# Blocks with 64..1024 threads: 16 x {4, 8, 16}, 32 x {2, 4, 8, 16},
# 64 x {1, ..., 16}, 128 x {1, 2, 4, 8}, 256 x {1, 2, 4}: 19 pairs.
# Legal tile_y per (block_y, temporal), temporal 1, 2, 3, 4, 6, 8 (2t = 2, 4,
# 6, 8, 12, 16; rows = block_y*tile_y must exceed 2t):
#   block_y 1: rows 1, 2, 4           -> 1 0 0 0 0 0
#   block_y 2: rows 2, 4, 8           -> 2 1 1 0 0 0
#   block_y 4: rows 4, 8, 16          -> 3 2 2 1 1 0
#   block_y 8: rows 8, 16, 32         -> 3 3 3 2 2 1
#   block_y 16: rows 16, 32, 64       -> 3 3 3 3 3 2
# Legal tile_x per (block_x, temporal): block_x 16 gives columns 16, 32, 64
# -> 3 3 3 3 3 2; block_x >= 32 gives at least 32 columns -> 3 everywhere.
# Sum over blocks of tile_x count * tile_y count:
#   16 x 4: 27, 16 x 8: 41, 16 x 16: 49                      -> 117
#   32 x {2, 4, 8, 16}: 3 * (4 + 9 + 14 + 17)                -> 132
#   64 x {1, ..., 16}: 3 * (1 + 4 + 9 + 14 + 17)             -> 135
#   128 x {1, 2, 4, 8}: 3 * (1 + 4 + 9 + 14)                 -> 84
#   256 x {1, 2, 4}: 3 * (1 + 4 + 9)                         -> 42
# 510 (block, tile, temporal) points, x4 switches = 2,040.

HAND_TY = {1: [1, 0, 0, 0, 0, 0], 2: [2, 1, 1, 0, 0, 0], 4: [3, 2, 2, 1, 1, 0],
           8: [3, 3, 3, 2, 2, 1], 16: [3, 3, 3, 3, 3, 2]}
HAND_TX = {16: [3, 3, 3, 3, 3, 2], 32: [3] * 6, 64: [3] * 6, 128: [3] * 6, 256: [3] * 6}
HAND_BLOCKS = {16: (4, 8, 16), 32: (2, 4, 8, 16), 64: (1, 2, 4, 8, 16), 128: (1, 2, 4, 8), 256: (1, 2, 4)}
TEMPORAL = (1, 2, 3, 4, 6, 8)


def test_hotspot_space_count_by_hand():
    from collections import Counter
    got = Counter((c[0], c[1], c[4]) for c in space.hotspot_restricted())
    want = {}
    for bx, bys in HAND_BLOCKS.items():
        for by in bys:
            for k, t in enumerate(TEMPORAL):
                n = 4 * HAND_TX[bx][k] * HAND_TY[by][k]
                if n:
                    want[(bx, by, t)] = n
    assert dict(got) == want
    assert sum(want.values()) == 2040 == len(space.hotspot_restricted())
    assert [sum(4 * HAND_TX[bx][k] * HAND_TY[by][k] for by in bys for k in range(6))
            for bx, bys in HAND_BLOCKS.items()] == [4 * 117, 4 * 132, 4 * 135, 4 * 84, 4 * 42]
