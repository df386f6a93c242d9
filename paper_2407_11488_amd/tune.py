"""Command-line driver of the tuner (conv2d_tune in the C library).

One shape:
    python -m paper_2407_11488_amd.tune --shape 4096 4096 17 17 [--results PATH]
        [--winners PATH] [--reps 20] [--retime-reps 200] [--no-flush] [--unroll 1]
        [--no-refine-unroll] [--max-configs N] [--json OUT]

Filter-size sweep (each shape tuned, then compared with a reference shape's
winner applied unchanged):
    python -m paper_2407_11488_amd.tune --size 4096 --filters 3 7 15 31 --ref-filter 17 \
        --results-dir DIR

The batched path's configurations on the 64-problem uneven workload (each
filter size's fastest 4096x4096 sweep points, timed as that size's batched
kernel over the batch's problems; stored as the (0, 0, fh, fw) winners):
    python -m paper_2407_11488_amd.tune --batch [--candidates 12]
The served path's configurations per filter size and size bucket (sizes up
to 384, 768, 1536, 3072 and above), tuned on a sample of shapes drawn like the
served workload's, stored as the (0, bucket, fh, fw) winners:
    python -m paper_2407_11488_amd.tune --buckets [--sample 160]
The batched path's configurations chosen in context (each group's
candidates timed as the whole 64-problem batch, the other groups held,
coordinate descent; appended as the (0, 0, fh, fw) winners):
    python -m paper_2407_11488_amd.tune --batch-context [--candidates 24] [--rounds 2]
The server's stream count and batch-size cap (streams 1-8 x caps 1-256, each
serving one Poisson trace at a fraction of serial capacity; lowest p99 wins),
stored in tuned/serve_params.json:
    python -m paper_2407_11488_amd.tune --serving [--rate 0.8 --duration 3]

Hotspot stencil (the second tunable kernel), one grid and step count:
    python -m paper_2407_11488_amd.tune --hotspot 4096 4096 --steps 60 [--results PATH]

Prints JSON reports: the winner and its throughput, the top five, the median,
the tuning impact (best over median throughput, the paper's Section 4
metric), tuned/default, and compile/launch/verify failure counts. Winners are
appended to the winners cache, which later plans of the same shape pick up.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

from . import _binding as B
from . import analysis

DEFAULT_WINNERS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned", "winners.jsonl")
PEAK_FP32_TFLOPS = 157.3


def report(shape, r) -> dict:
    H, W, fh, fw = shape
    flops = 2.0 * H * W * fh * fw
    top = [{"config": list(r.top[k].tuple()), "ms": round(r.top_ms[k], 5),
            "gflops": round(flops / (r.top_ms[k] * 1e-3) / 1e9, 1)} for k in range(5) if r.top_ms[k] > 0]
    return {
        "shape": [H, W, fh, fw],
        "winner": list(r.best.tuple()),
        "best_ms": round(r.best_ms, 5),
        "best_gflops": round(r.best_gflops, 1),
        "best_gbs": round(analysis.algorithmic_bytes(shape) / (r.best_ms * 1e-3) / 1e9, 1),
        "pct_fp32_peak": round(r.best_gflops / 1e3 / PEAK_FP32_TFLOPS * 100, 2),
        "median_gflops": round(r.median_gflops, 1),
        "impact": round(r.impact, 3),
        "default_ms": round(r.default_ms, 5),
        "default_gflops": round(r.default_gflops, 1),
        # both in the sustained re-timing's mode; the sweep-mode ratio beside it
        "tuned_vs_default": round(r.default_ms / r.best_ms, 3) if r.default_ms > 0 else None,
        "best_sweep_ms": round(r.best_sweep_ms, 5), "default_sweep_ms": round(r.default_sweep_ms, 5),
        "tuned_vs_default_sweep": (round(r.default_sweep_ms / r.best_sweep_ms, 3)
                                   if r.default_sweep_ms > 0 and r.best_sweep_ms > 0 else None),
        "default_rank": r.default_rank,
        "n_space": r.n_space, "n_illegal": r.n_illegal, "n_timed": r.n_timed,
        "n_compile_fail": r.n_compile_fail, "n_launch_fail": r.n_launch_fail,
        "n_verify_fail": r.n_verify_fail, "n_resumed": r.n_resumed,
        "compile_s": round(r.compile_s, 1), "measure_s": round(r.measure_s, 1),
        "top5": top,
    }


def tune_one(shape, a, results_path):
    o = B.conv2d_tune_defaults()
    o.winners_path = a.winners.encode() if a.winners else None
    o.results_path = results_path.encode() if results_path else None
    o.reps, o.retime_reps, o.warmup = a.reps, a.retime_reps, a.warmup
    o.flush_mall = 0 if a.no_flush else 1
    o.unroll, o.max_configs, o.threads, o.verbose = a.unroll, a.max_configs, a.threads, 1
    o.refine_unroll = 0 if a.no_refine_unroll else 1
    if a.strategy == "local":
        o.strategy, o.max_evals, o.seed = 1, a.max_evals, a.seed
    r = B.conv2d_tune(B.shape(*shape), o)
    rep = report(shape, r)
    rep["strategy"] = a.strategy
    rep["evaluations"] = r.evaluations
    return rep


HOTSPOT_WINNERS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned", "hotspot_winners.jsonl")


def tune_hotspot(rows, cols, steps, a, results_path):
    o = B.hotspot_tune_defaults()
    o.winners_path = HOTSPOT_WINNERS.encode() if a.winners == DEFAULT_WINNERS else a.winners.encode()
    o.results_path = results_path.encode() if results_path else None
    o.reps, o.retime_reps, o.warmup = a.reps, a.retime_reps, a.warmup
    o.flush_mall = 0 if a.no_flush else 1
    o.max_configs, o.threads, o.verbose = a.max_configs, a.threads, 1
    r = B.hotspot_tune(B.hotspot_shape(rows, cols), steps, o)
    top = [{"config": list(r.top[k].tuple()), "ms": round(r.top_ms[k], 5)} for k in range(5) if r.top_ms[k] > 0]
    return {
        "workload": "hotspot", "grid": [rows, cols], "steps": steps,
        "winner": list(r.best.tuple()), "best_ms": round(r.best_ms, 5), "best_gflops": round(r.best_gflops, 1),
        "median_gflops": round(r.median_gflops, 1), "impact": round(r.impact, 3),
        "default_ms": round(r.default_ms, 5), "default_gflops": round(r.default_gflops, 1),
        # both in the sustained re-timing's mode; the sweep-mode ratio beside it
        "tuned_vs_default": round(r.default_ms / r.best_ms, 3) if r.default_ms > 0 else None,
        "best_sweep_ms": round(r.best_sweep_ms, 5), "default_sweep_ms": round(r.default_sweep_ms, 5),
        "tuned_vs_default_sweep": (round(r.default_sweep_ms / r.best_sweep_ms, 3)
                                   if r.default_sweep_ms > 0 and r.best_sweep_ms > 0 else None),
        "default_rank": r.default_rank, "n_space": r.n_space, "n_illegal": r.n_illegal, "n_timed": r.n_timed,
        "n_compile_fail": r.n_compile_fail, "n_launch_fail": r.n_launch_fail, "n_verify_fail": r.n_verify_fail,
        "n_resumed": r.n_resumed, "compile_s": round(r.compile_s, 1), "measure_s": round(r.measure_s, 1),
        "top5": top,
    }


def emit(rep, path):
    line = json.dumps(rep)
    print(line, flush=True)
    if path:
        with open(path, "a") as fh:
            fh.write(line + "\n")


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--shape", type=int, nargs=4, metavar=("OUT_H", "OUT_W", "FH", "FW"))
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--filters", type=int, nargs="*")
    ap.add_argument("--ref-filter", type=int, default=17)
    ap.add_argument("--results-dir", default=None)
    ap.add_argument("--winners", default=DEFAULT_WINNERS)
    ap.add_argument("--results", default=None)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--retime-reps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-flush", action="store_true")
    ap.add_argument("--unroll", type=int, default=1)
    ap.add_argument("--no-refine-unroll", action="store_true")
    ap.add_argument("--max-configs", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--strategy", choices=("brute", "local"), default="brute",
                    help="brute: the whole space; local: random-restart hill climbing")
    ap.add_argument("--max-evals", type=int, default=100)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--json", default=None)
    ap.add_argument("--hotspot", type=int, nargs=2, metavar=("ROWS", "COLS"))
    ap.add_argument("--batch", action="store_true")
    ap.add_argument("--batch-context", action="store_true",
                    help="the batched groups' configurations by the whole batch's time (coordinate descent)")
    ap.add_argument("--rounds", type=int, default=2, help="--batch-context: passes over the groups")
    ap.add_argument("--candidates", type=int, default=None,
                    help="sweep points tried per group (default 12; --batch-context: 24)")
    ap.add_argument("--buckets", action="store_true",
                    help="batched kernels per filter size and size bucket, on a sample of served shapes")
    ap.add_argument("--sample", type=int, default=160)
    ap.add_argument("--serving", action="store_true",
                    help="the server's stream count and batch-size cap, by p99 on a trace of its own")
    ap.add_argument("--rate", type=float, default=0.8, help="--serving: load as a fraction of serial capacity")
    ap.add_argument("--duration", type=float, default=3.0, help="--serving: trace seconds per point")
    ap.add_argument("--steps", type=int, default=60)
    a = ap.parse_args(argv)

    if a.serving:
        from . import workloads
        emit(workloads.tune_serving(a.rate, a.duration), a.json)
        return 0
    if a.batch_context:
        from . import workloads
        emit(workloads.batch_context_tune(candidates=a.candidates or 24, rounds=a.rounds, winners=a.winners,
                                          results_dir=a.results_dir), a.json)
        return 0
    if a.batch or a.buckets:
        import datagen
        o = B.conv2d_batch_tune_defaults()
        o.winners_path = a.winners.encode()
        o.results_dir = (a.results_dir or os.path.dirname(DEFAULT_WINNERS)).encode()
        o.candidates, o.verbose = a.candidates or 12, 1
        if a.buckets:
            # one configuration per filter size and size bucket, tuned on a
            # sample of the served distribution
            o.buckets = 1
            shapes = datagen.serving_sample(a.sample)
            what = f"{a.sample} request shapes like the served workload's (sides log-uniform [128, 4096])"
        else:
            shapes = datagen.batch_shapes(64)
            what = "batched, 64 problems (sides log-uniform [256, 2048], filters {3,5,9,17})"
        r = B.conv2d_batch_tune(shapes, o)
        emit({"workload": what, "groups": r.groups()}, a.json)
        return 0
    if a.hotspot:
        rows, cols = a.hotspot
        results = a.results or os.path.join(os.path.dirname(DEFAULT_WINNERS),
                                            f"hotspot_results_gfx950_{rows}x{cols}_s{a.steps}.jsonl")
        emit(tune_hotspot(rows, cols, a.steps, a, results), a.json)
        return 0

    if a.shape:
        emit(tune_one(tuple(a.shape), a, a.results), a.json)
        return 0
    if not a.filters:
        ap.error("give --shape, or --filters for a filter-size sweep")
    rdir = a.results_dir or os.path.dirname(DEFAULT_WINNERS)
    os.makedirs(rdir, exist_ok=True)
    n = a.size
    ref_shape = (n, n, a.ref_filter, a.ref_filter)
    ref_db = os.path.join(rdir, analysis.results_name("gfx950", ref_shape))
    for f in a.filters:
        shape = (n, n, f, f)
        db = os.path.join(rdir, analysis.results_name("gfx950", shape))
        rep = tune_one(shape, a, db)
        ref_cfg = analysis.winner_of(ref_db, ref_shape, winners_path=a.winners)
        if ref_cfg is not None:
            rep["ref_shape"] = list(ref_shape)
            rep["ref_winner"] = list(ref_cfg)
            eff = analysis.efficiency_of(db, shape, ref_cfg)
            if eff.get("efficiency") is None and B.conv2d_config_check(B.shape(*shape), ref_cfg) == 0:
                # The reference winner is not a point of this sweep (another
                # unroll value): time it the same way.
                ms, _ = B.conv2d_benchmark(B.shape(*shape), ref_cfg, a.warmup, a.reps, 0 if a.no_flush else 1)
                got = analysis.flops(shape) / (ms * 1e-3) / 1e9
                eff = {"ref_config_gflops": round(got, 1), "own_best_gflops": eff.get("own_best_gflops"),
                       "efficiency": round(got / max(got, eff.get("own_best_gflops") or got), 4)}
            rep.update(eff)
        emit(rep, a.json)
    return 0


if __name__ == "__main__":
    sys.exit(main())
