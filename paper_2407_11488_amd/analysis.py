"""Search-space statistics over the tuner's results database (JSON lines, one
per timed configuration), following the paper's Section 4 metrics:

* tuning impact: best over median throughput (Table 3's statistic);
* the distribution of throughput relative to the optimum (the violin plots of
  Figs. 3, 5, 7, 9, summarised here as percentiles);
* application efficiency e_i(x) = P_i(x) / max_x P_i(x) (Eq. 3), with the
  "devices" i replaced by problem shapes on one GPU;
* performance portability PP(x, H) = |H| / sum_i 1/e_i(x) (Eq. 2), and the
  configuration that maximises it over a set of shapes.
"""
from __future__ import annotations

import json
import math
import os


def results_name(arch: str, shape) -> str:
    H, W, fh, fw = shape
    return f"results_{arch}_{H}x{W}_{fh}x{fw}.jsonl"


def flops(shape) -> float:
    H, W, fh, fw = shape
    return 2.0 * H * W * fh * fw


def algorithmic_bytes(shape) -> int:
    """Bytes a convolution must move at least once: input, output, filter."""
    H, W, fh, fw = shape
    return 4 * ((H + fh - 1) * (W + fw - 1) + H * W + fh * fw)


def load(db: str, shape, src: str | None = None) -> dict:
    """config tuple -> record for `shape` (the last line of a config wins)."""
    out = {}
    if not os.path.exists(db):
        return out
    with open(db) as fh:
        for line in fh:
            try:
                r = json.loads(line)
            except json.JSONDecodeError:
                continue
            if tuple(r.get("shape", ())) != tuple(shape) or (src and r.get("src") != src):
                continue
            out[tuple(int(v) for v in r["config"])] = r
    return out


def throughputs(db: str, shape, src: str | None = None) -> dict:
    """config -> GFLOP/s for the configurations that compiled, ran and verified."""
    return {c: flops(shape) / (r["ms"] * 1e-3) / 1e9 for c, r in load(db, shape, src).items()
            if r.get("status") == "ok" and r.get("ms", 0) > 0}


def _median(v):
    v = sorted(v)
    n = len(v)
    return v[n // 2] if n % 2 else 0.5 * (v[n // 2 - 1] + v[n // 2])


def impact(db: str, shape, src: str | None = None) -> float:
    p = list(throughputs(db, shape, src).values())
    return max(p) / _median(p)


def percentiles(db: str, shape, qs=(0, 10, 25, 50, 75, 90, 100), src: str | None = None) -> dict:
    """Throughput relative to the optimum at the given percentiles (nearest rank)."""
    p = sorted(throughputs(db, shape, src).values())
    best = p[-1]
    out = {}
    for q in qs:
        k = max(1, math.ceil(q / 100 * len(p))) - 1 if q > 0 else 0
        out[f"p{q}"] = round(p[k] / best, 4)
    return out


def winner_of(db: str, shape, winners_path: str | None = None):
    """The cached winner of `shape` (last entry), else the fastest in the DB."""
    if winners_path and os.path.exists(winners_path):
        win = None
        with open(winners_path) as fh:
            for line in fh:
                try:
                    r = json.loads(line)
                except json.JSONDecodeError:
                    continue
                if tuple(r.get("shape", ())) == tuple(shape):
                    win = tuple(int(v) for v in r["config"])
        if win is not None:
            return win
    p = throughputs(db, shape)
    return max(p, key=p.get) if p else None


def efficiency_of(db: str, shape, cfg) -> dict:
    """Eq. 3 for one configuration on one shape."""
    p = throughputs(db, shape)
    if not p:
        return {}
    best = max(p.values())
    got = p.get(tuple(cfg))
    return {"ref_config_gflops": None if got is None else round(got, 1), "own_best_gflops": round(best, 1),
            "efficiency": None if got is None else round(got / best, 4)}


def performance_portability(effs) -> float:
    """Eq. 2: harmonic mean of the efficiencies (0 if any is 0 or missing)."""
    effs = list(effs)
    if not effs or any(e is None or e <= 0 for e in effs):
        return 0.0
    return len(effs) / sum(1.0 / e for e in effs)


def portability_table(dbs: dict) -> dict:
    """dbs: shape -> db path. Returns, for every configuration timed on every
    shape, its efficiencies per shape and its PP over the set."""
    per = {s: throughputs(db, s) for s, db in dbs.items()}
    common = set.intersection(*(set(p) for p in per.values())) if per else set()
    best = {s: max(p.values()) for s, p in per.items()}
    table = {}
    for c in common:
        e = {s: per[s][c] / best[s] for s in per}
        table[c] = {"efficiency": e, "pp": performance_portability(e.values())}
    return table


def most_portable(dbs: dict):
    """The configuration with the highest PP over the shapes (ties: smallest tuple)."""
    t = portability_table(dbs)
    if not t:
        return None, {}
    c = max(sorted(t), key=lambda k: t[k]["pp"])
    return c, t[c]


# ---------------------------------------------------------------- tuning difficulty

SPACE_AXES = ((16, 32, 64, 128), (1, 2, 4, 8, 16), (1, 2, 4, 8), (1, 2, 4, 8), (0, 1), (0, 1))
# The hotspot space (block_x, block_y, tile_x, tile_y, temporal, unroll_t, sh_power).
HOTSPOT_AXES = ((16, 32, 64, 128, 256), (1, 2, 4, 8, 16), (1, 2, 4), (1, 2, 4), (1, 2, 3, 4, 6, 8), (0, 1), (0, 1))


def fitness_flow_graph(times: dict, axes=SPACE_AXES):
    """The fitness flow graph of Section 4: timed configurations as nodes and
    an edge from each node to every neighbour with a strictly lower time.
    Neighbours differ in one parameter by one step of its ordered value list.
    Returns (nodes, out_lists)."""
    nodes = sorted(times)
    index = {c: i for i, c in enumerate(nodes)}
    out = [[] for _ in nodes]
    for i, c in enumerate(nodes):
        t = times[c]
        for k, values in enumerate(axes):
            pos = values.index(c[k])
            for q in (pos - 1, pos + 1):
                if 0 <= q < len(values):
                    j = index.get(c[:k] + (values[q],) + c[k + 1:])
                    if j is not None and times[nodes[j]] < t:
                        out[i].append(j)
    return nodes, out


def pagerank(out, damping: float = 0.85, tol: float = 1e-14, max_iter: int = 10000):
    """PageRank by power iteration: a node spreads its rank equally over its
    out-edges; nodes without out-edges spread theirs over every node."""
    import numpy as np
    n = len(out)
    src = np.array([i for i, o in enumerate(out) for _ in o], dtype=np.int64)
    dst = np.array([j for o in out for j in o], dtype=np.int64)
    deg = np.array([len(o) for o in out], dtype=np.float64)
    dangling = deg == 0
    w = np.zeros(len(src)) if len(src) == 0 else 1.0 / deg[src]
    r = np.full(n, 1.0 / n)
    for _ in range(max_iter):
        nxt = np.zeros(n)
        np.add.at(nxt, dst, r[src] * w)
        nxt = damping * (nxt + r[dangling].sum() / n) + (1.0 - damping) / n
        nxt /= nxt.sum()
        if np.abs(nxt - r).sum() < tol:
            return nxt
        r = nxt
    return r


def proportion_of_centrality(times: dict, ps=(0.0, 0.01, 0.02, 0.05, 0.10, 0.15), axes=SPACE_AXES,
                             damping: float = 0.85) -> dict:
    """Eq. 1 for each p: PageRank mass of the local minima within (1 + p) of
    the best time, over the mass of all local minima."""
    nodes, out = fitness_flow_graph(times, axes)
    r = pagerank(out, damping)
    minima = [i for i, o in enumerate(out) if not o]
    best = min(times.values())
    total = sum(r[i] for i in minima)
    return {p: float(sum(r[i] for i in minima if times[nodes[i]] <= (1.0 + p) * best) / total) for p in ps}


def base_space_times(db: str, shape, unroll: int = 1) -> dict:
    """Times (ms) of the timed points of the base sweep (one unroll value),
    keyed by the 6-parameter tuple."""
    return {c[:6]: r["ms"] for c, r in load(db, shape).items()
            if r.get("status") == "ok" and r.get("ms", 0) > 0 and c[6] == unroll}


# ---------------------------------------------------------------- local-search effort

def local_search_effort(times: dict, shape, ps=(0.0, 0.01, 0.05), seeds=range(50), max_evals: int = 400,
                        unroll: int = 1) -> dict:
    """How many evaluations the tuner's local-search strategy needs to come
    within p of the optimum of a timed space (the use of Section 4's
    difficulty measure: a walk that reaches a good minimum early makes the
    space cheap to tune). `times` maps the 6-parameter base tuple to ms (the
    base sweep); the search runs through conv2d_tune_synthetic with those
    times as its cost (points without a time fail to compile), once per seed,
    and the evaluation order it records is replayed against the times. For
    each p: the median and 90th percentile of the evaluation count at which
    the best time so far first falls within (1 + p) of the sweep's optimum,
    and the fraction of seeds that got there within max_evals."""
    import tempfile

    from . import _binding as B
    s = B.shape(*shape)
    best = min(times.values())
    counts = {p: [] for p in ps}
    with tempfile.TemporaryDirectory() as tmp:
        for seed in seeds:
            path = os.path.join(tmp, f"r{seed}.jsonl")
            o = B.conv2d_tune_defaults()
            o.strategy, o.max_evals, o.seed, o.unroll = 1, max_evals, int(seed), unroll
            o.retime_reps = 0
            o.results_path = path.encode()
            B.conv2d_tune_synthetic(s, lambda c: times.get(tuple(c[:6]), B.CONV2D_ECOMPILE), o)
            order = []
            with open(path) as fh:
                for line in fh:
                    c = tuple(json.loads(line)["config"][:6])
                    if c not in order:
                        order.append(c)
            run = math.inf
            first = {}
            for k, c in enumerate(order, 1):
                run = min(run, times.get(c, math.inf))
                for p in ps:
                    if p not in first and run <= (1.0 + p) * best:
                        first[p] = k
            for p in ps:
                counts[p].append(first.get(p))

    def q(v, f):
        # nearest-rank quantile over every seed; a seed that never got there
        # counts as beyond the budget (None when the quantile falls there)
        v = sorted(math.inf if k is None else k for k in v)
        x = v[min(len(v) - 1, int(f * len(v)))]
        return None if x == math.inf else x

    out = {"space": len(times), "seeds": len(list(seeds)), "max_evals": max_evals}
    for p in ps:
        got = [k for k in counts[p] if k is not None]
        out[f"p{round(100 * p)}"] = {"reached": round(len(got) / len(counts[p]), 3),
                                     "median_evals": q(counts[p], 0.5), "p90_evals": q(counts[p], 0.9),
                                     "per_seed": counts[p]}
    return out


def _current_source_hash() -> str:
    from . import _binding as B
    return B.conv2d_kernel_hash()


def hotspot_sweep_times(db: str, grid, steps: int = 60, src: str | None = None) -> dict:
    """Times (ms) of the verified points of a hotspot sweep (the last record
    of each configuration), keyed by the 7-parameter tuple."""
    out = {}
    if not os.path.exists(db):
        return out
    with open(db) as fh:
        for line in fh:
            try:
                r = json.loads(line)
            except json.JSONDecodeError:
                continue
            if tuple(r.get("shape", ())) != tuple(grid) or r.get("steps") != steps or (src and r.get("src") != src):
                continue
            c = tuple(int(v) for v in r["config"])
            if r.get("status") == "ok" and r.get("ms", 0) > 0:
                out[c] = r["ms"]
            else:
                out.pop(c, None)
    return out


def main(argv=None) -> int:
    """`python -m paper_2407_11488_amd.analysis effort [--seeds 50] [--max-evals 400]`:
    the local-search effort over every committed 4096 x 4096 sweep;
    `... analysis hotspot-difficulty`: Eq. 1's centrality over the committed
    hotspot sweeps."""
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=("effort", "hotspot-difficulty"))
    ap.add_argument("--seeds", type=int, default=50)
    ap.add_argument("--max-evals", type=int, default=400)
    ap.add_argument("--filters", type=int, nargs="*", default=[3, 5, 7, 9, 15, 17, 31])
    a = ap.parse_args(argv)
    if a.what == "hotspot-difficulty":
        from . import _binding as B
        hsrc = B.hotspot_kernel_hash()
        here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned")
        for n in (2048, 4096, 8192):
            db = os.path.join(here, f"hotspot_results_gfx950_{n}x{n}_s60.jsonl")
            times = hotspot_sweep_times(db, (n, n), 60, hsrc)
            if not times:
                continue
            pc = proportion_of_centrality(times, axes=HOTSPOT_AXES)
            print(json.dumps({"grid": [n, n], "points": len(times),
                              "C": {f"{round(100 * p)}%": round(v, 3) for p, v in pc.items()}}), flush=True)
        return 0
    src = _current_source_hash()
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned")
    for f in a.filters:
        shape = (4096, 4096, f, f)
        db = os.path.join(here, results_name("gfx950", shape))
        times = {c[:6]: r["ms"] for c, r in load(db, shape, src).items()
                 if r.get("status") == "ok" and r.get("ms", 0) > 0 and c[6] == 1}
        if not times:
            continue
        r = local_search_effort(times, shape, seeds=range(a.seeds), max_evals=a.max_evals)
        for k in list(r):
            if isinstance(r[k], dict):
                r[k].pop("per_seed", None)
        print(json.dumps({"filter": f, **r}), flush=True)
    return 0


if __name__ == "__main__":
    import sys
    sys.exit(main())
