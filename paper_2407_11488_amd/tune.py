"""Command-line driver of the tuner (conv2d_tune in the C library).

    python -m paper_2407_11488_amd.tune --shape 4096 4096 17 17 [--results PATH]
        [--winners PATH] [--reps 20] [--retime-reps 50] [--no-flush] [--unroll 1]
        [--max-configs N] [--json OUT]

Prints one JSON report: the winner and its throughput, the top five, the
median configuration, the tuning impact (best over median throughput, the
paper's Section 4 metric), tuned/default, and compile/launch/verify failure
counts. The winner is appended to the winners cache, which later plans of the
same shape pick up.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

from . import _binding as B

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
        "pct_fp32_peak": round(r.best_gflops / 1e3 / PEAK_FP32_TFLOPS * 100, 2),
        "median_gflops": round(r.median_gflops, 1),
        "impact": round(r.impact, 3),
        "default_ms": round(r.default_ms, 5),
        "default_gflops": round(r.default_gflops, 1),
        "tuned_vs_default": round(r.default_ms / r.best_ms, 3) if r.default_ms > 0 else None,
        "default_rank": r.default_rank,
        "n_space": r.n_space, "n_illegal": r.n_illegal, "n_timed": r.n_timed,
        "n_compile_fail": r.n_compile_fail, "n_launch_fail": r.n_launch_fail,
        "n_verify_fail": r.n_verify_fail, "n_resumed": r.n_resumed,
        "compile_s": round(r.compile_s, 1), "measure_s": round(r.measure_s, 1),
        "top5": top,
    }


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--shape", type=int, nargs=4, metavar=("OUT_H", "OUT_W", "FH", "FW"), required=True)
    ap.add_argument("--winners", default=DEFAULT_WINNERS)
    ap.add_argument("--results", default=None)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--retime-reps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-flush", action="store_true")
    ap.add_argument("--unroll", type=int, default=1)
    ap.add_argument("--max-configs", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    o = B.conv2d_tune_defaults()
    o.winners_path = a.winners.encode() if a.winners else None
    o.results_path = a.results.encode() if a.results else None
    o.reps, o.retime_reps, o.warmup = a.reps, a.retime_reps, a.warmup
    o.flush_mall = 0 if a.no_flush else 1
    o.unroll, o.max_configs, o.threads, o.verbose = a.unroll, a.max_configs, a.threads, 1
    r = B.conv2d_tune(B.shape(*a.shape), o)
    rep = report(a.shape, r)
    line = json.dumps(rep)
    print(line, flush=True)
    if a.json:
        with open(a.json, "a") as fh:
            fh.write(line + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
