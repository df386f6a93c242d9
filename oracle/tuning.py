"""Oracle for the tuner's statistics — TEST INFRASTRUCTURE ONLY.

Plain Python/numpy definitions, each citing where the paper defines it, used
by the tests to check the statistics the C++ tuner and serving loop report.

* Tuning impact (Section 4, "Tuning impact"; Table 3 caption): performance of
  the global optimum divided by the median performance over the search space.
* Application efficiency e_i(x) (Section 4, Eq. 3): P_i(x) / max_x P_i(x).
* Performance portability PP(x, H) (Section 4, Eq. 2): the harmonic mean of
  e_i(x) over the set H (|H| / sum 1/e_i); 0 when any e_i is 0.
* Medians follow the numpy convention (mean of the two middle values for an
  even count); the paper does not fix one.
* Winner selection (the paper is silent): the lowest time wins; times within
  ``rel_tie`` of the lowest count as ties, and a tie goes to the
  lexicographically smallest configuration tuple.
* Latency percentiles (the paper has none; the serving loop reports them):
  nearest rank, the ceil(p/100 * n)-th smallest value.
"""
from __future__ import annotations

import math

import numpy as np


def median(values) -> float:
    v = np.sort(np.asarray(values, dtype=np.float64))
    n = v.size
    if n == 0:
        raise ValueError("median of an empty set")
    if n % 2:
        return float(v[n // 2])
    return float(0.5 * (v[n // 2 - 1] + v[n // 2]))


def tuning_impact(perf) -> float:
    """max(perf) / median(perf), perf as throughput (higher is better)."""
    return float(np.max(perf)) / median(perf)


def gflops(out_h: int, out_w: int, fh: int, fw: int, seconds: float) -> float:
    """Convolution throughput: 2*H*W*fh*fw floating-point operations per run."""
    return 2.0 * out_h * out_w * fh * fw / seconds / 1e9


def pick_winner(times: dict, rel_tie: float = 0.005):
    """``times`` maps configuration tuples to seconds; returns the winner."""
    best = min(times.values())
    tied = [c for c, t in times.items() if t <= best * (1.0 + rel_tie)]
    return min(tied)


def top_k(times: dict, k: int = 5):
    """The ``k`` fastest configurations, fastest first (ties by tuple order)."""
    return sorted(times, key=lambda c: (times[c], c))[:k]


def efficiency(perf_x: float, perf_all) -> float:
    """Eq. 3: P_i(x) / max over the space of P_i."""
    return float(perf_x) / float(np.max(perf_all))


def performance_portability(effs) -> float:
    """Eq. 2: |H| / sum_i 1/e_i (0 if any e_i is 0)."""
    effs = [float(e) for e in effs]
    if not effs:
        raise ValueError("empty device/shape set")
    if any(e <= 0.0 for e in effs):
        return 0.0
    return len(effs) / sum(1.0 / e for e in effs)


def ffg_edges(times: dict, axes):
    """Fitness flow graph (Section 4, "Tuning difficulty"): nodes are the
    timed configurations; x -> y for every neighbour y of x with strictly
    lower time. Neighbours differ in one parameter by one step of that
    parameter's ordered value list (the paper does not define the
    neighbourhood; this is the reading taken). Returns (nodes, edges) with
    edges as (i, j) index pairs into the sorted node list."""
    nodes = sorted(times)
    index = {c: i for i, c in enumerate(nodes)}
    edges = []
    for c in nodes:
        for k, values in enumerate(axes):
            pos = values.index(c[k])
            for q in (pos - 1, pos + 1):
                if 0 <= q < len(values):
                    n = c[:k] + (values[q],) + c[k + 1:]
                    if n in index and times[n] < times[c]:
                        edges.append((index[c], index[n]))
    return nodes, edges


def pagerank_dense(n: int, edges, damping: float = 0.85) -> np.ndarray:
    """PageRank (Brin and Page 1998) by a direct linear solve: with M the
    column-stochastic transition matrix (each node's out-edges weighted
    equally; a node without out-edges links to every node), r solves
    (I - d M) r = (1 - d)/n * 1. The damping 0.85 is the usual value (the
    paper does not state one)."""
    M = np.zeros((n, n))
    out = [[] for _ in range(n)]
    for i, j in edges:
        out[i].append(j)
    for i in range(n):
        if out[i]:
            for j in out[i]:
                M[j, i] += 1.0 / len(out[i])
        else:
            M[:, i] = 1.0 / n
    r = np.linalg.solve(np.eye(n) - damping * M, np.full(n, (1.0 - damping) / n))
    return r / r.sum()


def proportion_of_centrality(times: dict, axes, p: float, damping: float = 0.85) -> float:
    """Eq. 1: the PageRank mass of the local minima whose time is at most
    (1 + p) * best, over the mass of all local minima (nodes of the FFG with
    no better neighbour). The paper writes "less than", but plots p = 0 as
    the global optimum itself, so the bound is read as inclusive."""
    nodes, edges = ffg_edges(times, axes)
    r = pagerank_dense(len(nodes), edges, damping)
    has_out = {i for i, _ in edges}
    minima = [i for i in range(len(nodes)) if i not in has_out]
    best = min(times.values())
    good = [i for i in minima if times[nodes[i]] <= (1.0 + p) * best]
    return float(sum(r[i] for i in good) / sum(r[i] for i in minima))


def local_search(times: dict, legal: list, axes, max_evals: int, seed: int):
    """Random-restart hill climbing as the tuner's local-search strategy
    defines it, written plainly. times[c] is the time of configuration c, or
    None for a point that fails. legal lists the points in enumeration order.
    A walk evaluates every unevaluated neighbour (one parameter one step, in
    axis order, the lower value first) and moves to the fastest while that
    improves; restart k starts at the idx-th unevaluated point, idx =
    splitmix64(seed, k) mod count (the counter form of SplitMix64). Returns
    (best configuration, configurations in evaluation order)."""
    from datagen import splitmix64
    index = set(legal)
    state, order = {}, []

    def evaluate(cfgs):
        for c in cfgs:
            if len(order) >= max_evals:
                return
            state[c] = times[c]
            order.append(c)

    def neighbours(c):
        out = []
        for k, vals in enumerate(axes):
            pos = list(vals).index(c[k])
            for q in (pos - 1, pos + 1):
                if 0 <= q < len(vals):
                    n = c[:k] + (vals[q],) + c[k + 1:]
                    if n in index:
                        out.append(n)
        return out

    restart = 0
    while len(order) < max_evals:
        fresh = [c for c in legal if c not in state]
        if not fresh:
            break
        z = int(splitmix64(seed, np.array([restart], dtype=np.uint64))[0])
        restart += 1
        cur = fresh[z % len(fresh)]
        evaluate([cur])
        if state.get(cur) is None:
            continue
        while len(order) < max_evals:
            nb = neighbours(cur)
            evaluate([n for n in nb if n not in state])
            ok = [n for n in nb if state.get(n) is not None]
            if not ok:
                break
            nxt = min(ok, key=lambda c: (state[c], c))
            if not state[nxt] < state[cur]:
                break
            cur = nxt
    ok = [c for c in state if state[c] is not None]
    return min(ok, key=lambda c: (state[c], c)), order


def percentile_nearest_rank(values, p: float) -> float:
    v = np.sort(np.asarray(values, dtype=np.float64))
    if v.size == 0:
        raise ValueError("percentile of an empty set")
    rank = max(1, math.ceil(p / 100.0 * v.size))
    return float(v[rank - 1])
