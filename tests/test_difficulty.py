"""Tuning difficulty (Section 4, Eq. 1): fitness flow graph, PageRank and the
p-proportion of centrality. The oracle is pinned by hand-derived closed forms;
the analysis module (sparse power iteration) is checked against it."""
import os

import numpy as np
import pytest

from oracle import space as ospace
from oracle import tuning as ot
from paper_2407_11488_amd import analysis as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
AXES6 = [list(v) for _, v in ospace.AXES]


def test_pagerank_two_nodes_closed_form():
    # 0 -> 1, node 1 has no out-edge. With d = 0.85 the PageRank equations
    #   r0 = 0.075 + 0.85*r1/2,  r1 = 0.075 + 0.85*(r0 + r1/2)
    # solve by hand to r1 = 0.13875/0.21375 = 37/57, r0 = 20/57.
    r = ot.pagerank_dense(2, [(0, 1)])
    assert r == pytest.approx([20 / 57, 37 / 57], abs=1e-15)
    assert A.pagerank([[1], []]) == pytest.approx([20 / 57, 37 / 57], abs=1e-12)


@pytest.mark.parametrize("n", [1, 3, 7])
def test_pagerank_symmetric_graphs_are_uniform(n):
    cycle = [(i, (i + 1) % n) for i in range(n)] if n > 1 else []
    assert ot.pagerank_dense(n, cycle) == pytest.approx(np.full(n, 1 / n), abs=1e-15)
    assert ot.pagerank_dense(n, []) == pytest.approx(np.full(n, 1 / n), abs=1e-15)
    assert A.pagerank([[(i + 1) % n] if n > 1 else [] for i in range(n)]) == pytest.approx(np.full(n, 1 / n))


def test_ffg_single_valley():
    axes = [["a", "b", "c"]]
    times = {("a",): 3.0, ("b",): 2.0, ("c",): 1.0}
    nodes, edges = ot.ffg_edges(times, axes)
    assert sorted(edges) == [(0, 1), (1, 2)]
    for p in (0.0, 0.05, 1.0):
        assert ot.proportion_of_centrality(times, axes, p) == 1.0


def test_ffg_two_symmetric_valleys():
    # b sits between two minima a (time 1) and c (time 2): the walk reaches
    # each with the same probability, so C_0 = 1/2; once p admits c, C_p = 1.
    axes = [["a", "b", "c"]]
    times = {("a",): 1.0, ("b",): 5.0, ("c",): 2.0}
    assert ot.proportion_of_centrality(times, axes, 0.0) == pytest.approx(0.5, abs=1e-15)
    assert ot.proportion_of_centrality(times, axes, 0.99) == pytest.approx(0.5, abs=1e-15)
    assert ot.proportion_of_centrality(times, axes, 1.0) == 1.0


def _synthetic_times(seed):
    rng = np.random.default_rng(seed)
    return {c: float(rng.lognormal(0, 0.5)) for c in ospace.restricted()}


@pytest.mark.parametrize("seed", [1, 2])
def test_analysis_matches_oracle_on_the_real_lattice(seed):
    times = _synthetic_times(seed)
    ps = (0.0, 0.02, 0.1, 0.5)
    got = A.proportion_of_centrality(times, ps)
    for p in ps:
        assert got[p] == pytest.approx(ot.proportion_of_centrality(times, AXES6, p), abs=1e-9)
    vals = [got[p] for p in ps]
    assert all(0 <= v <= 1 for v in vals) and vals == sorted(vals)


def test_committed_sweep_difficulty():
    db = os.path.join(ROOT, "paper_2407_11488_amd", "tuned", "results_gfx950_4096x4096_17x17.jsonl")
    times = A.base_space_times(db, (4096, 4096, 17, 17))
    assert len(times) > 1100
    ps = (0.0, 0.05, 0.15)
    got = A.proportion_of_centrality(times, ps)
    for p in ps:
        assert got[p] == pytest.approx(ot.proportion_of_centrality(times, AXES6, p), abs=1e-9)


def test_hotspot_sweep_loader_and_axes(tmp_path):
    """hotspot_sweep_times keeps the last verified record of each
    configuration of one grid and step count; every committed hotspot point
    lies on the hotspot axes, so the fitness flow graph covers it."""
    import json as _json
    import os as _os
    db = tmp_path / "h.jsonl"
    rows = [
        {"shape": [64, 64], "steps": 60, "config": [32, 8, 1, 1, 1, 1, 1], "status": "ok", "ms": 2.0},
        {"shape": [64, 64], "steps": 60, "config": [32, 8, 1, 1, 1, 1, 1], "status": "ok", "ms": 1.5},
        {"shape": [64, 64], "steps": 60, "config": [64, 8, 1, 1, 1, 1, 1], "status": "verify", "ms": 0.0},
        {"shape": [64, 64], "steps": 30, "config": [16, 8, 1, 1, 1, 1, 1], "status": "ok", "ms": 1.0},
        {"shape": [32, 32], "steps": 60, "config": [16, 8, 1, 1, 1, 1, 1], "status": "ok", "ms": 1.0},
    ]
    db.write_text("".join(_json.dumps(r) + "\n" for r in rows) + "{broken\n")
    assert A.hotspot_sweep_times(str(db), (64, 64), 60) == {(32, 8, 1, 1, 1, 1, 1): 1.5}
    here = _os.path.join(_os.path.dirname(_os.path.dirname(_os.path.abspath(__file__))), "paper_2407_11488_amd",
                         "tuned", "hotspot_results_gfx950_4096x4096_s60.jsonl")
    times = A.hotspot_sweep_times(here, (4096, 4096), 60)
    assert len(times) == 2040
    for c in times:
        assert all(v in axis for v, axis in zip(c, A.HOTSPOT_AXES)), c
    nodes, out = A.fitness_flow_graph(times, A.HOTSPOT_AXES)
    assert any(out) and not out[nodes.index(min(times, key=times.get))]   # the optimum is a sink
