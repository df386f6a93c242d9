"""Measurement drivers for the batched and served workloads.

    python -m paper_2407_11488_amd.workloads batch [--reps 20]
    python -m paper_2407_11488_amd.workloads serve [--duration 60] [--rates 0.5 0.8 1.0 1.2]

batch: the 64-problem uneven workload (square outputs log-uniform in
[256, 2048], filters from {3, 5, 9, 17}) as one graph launch of the batched
path, against 64 separate conv2d_run launches of the plain path, each with
the tuned configuration of its filter size.

serve: Poisson arrivals of requests with sides log-uniform in [128, 4096] and
filters from {3, 5, 9, 17}, images generated on the device, admission by an
HBM budget. The serial plain capacity is probed first (a trace whose requests
all arrive at once); the trace then runs at fractions of that rate through the
continuous-batching server and through the serial plain baseline.

hotspot: the 4096 x 4096 chip workload of the hotspot stencil, 60 steps per
run, in the plan's configuration (tuned winner when cached) against the
default configuration.

    python -m paper_2407_11488_amd.workloads hotspot [--reps 20] [--steps 60]

Each prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import datagen

from . import _binding as B
from . import analysis

WINNERS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned", "winners.jsonl")


def _torch():
    import torch
    return torch


def tuned_config_for_filter(fh, fw):
    c = analysis.winner_of("", (4096, 4096, fh, fw), winners_path=WINNERS)
    return c if c is not None else B.conv2d_default_config().tuple()


def batch_benchmark(reps: int = 20, warmup: int = 3, n: int = 64) -> dict:
    torch = _torch()
    from .api import Batch, Plan
    shapes = datagen.batch_shapes(n)
    st = torch.cuda.current_stream()
    ins, fs, outs = [], [], []
    for p, (H, W, fh, fw) in enumerate(shapes):
        inp = torch.empty((H + fh - 1, W + fw - 1), dtype=torch.float32, device="cuda")
        f = torch.empty((fh, fw), dtype=torch.float32, device="cuda")
        B.conv2d_fill_uniform(inp.data_ptr(), inp.numel(), datagen.SEED_BATCH_INPUT_BASE + p, 0, st.cuda_stream)
        B.conv2d_fill_uniform(f.data_ptr(), f.numel(), datagen.SEED_BATCH_FILTER_BASE + p, 0, st.cuda_stream)
        ins.append(inp)
        fs.append(f)
        outs.append(torch.empty((H, W), dtype=torch.float32, device="cuda"))
    flops = sum(analysis.flops(s) for s in shapes)
    batch = Batch(shapes)
    plans = [Plan(*s, config=tuned_config_for_filter(s[2], s[3])) for s in shapes]
    torch.cuda.synchronize()

    def timed(fn, k):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(st)
        for _ in range(k):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k, 1e3 * (time.perf_counter() - t0) / k

    def run_batch():
        batch(ins, fs, outs)

    def run_plain():
        for p in range(len(shapes)):
            plans[p](ins[p], fs[p], out=outs[p])

    b_ms, b_wall = timed(run_batch, reps)
    p_ms, p_wall = timed(run_plain, reps)
    res = {
        "workload": f"{n} convolutions, sides log-uniform [256, 2048], filters {{3,5,9,17}}",
        "gflop": round(flops / 1e9, 3),
        "batch_ms": round(b_ms, 4), "batch_gflops": round(flops / (b_ms * 1e-3) / 1e9, 1),
        "plain_ms": round(p_ms, 4), "plain_gflops": round(flops / (p_ms * 1e-3) / 1e9, 1),
        "speedup": round(p_ms / b_ms, 3),
        "batch_wall_ms": round(b_wall, 4), "plain_wall_ms": round(p_wall, 4),
        "groups": batch.info["groups"], "total_tiles": batch.info["total_tiles"],
    }
    batch.close()
    for p in plans:
        p.close()
    return res


def _trace(rate, duration, seed=datagen.SEED_ARRIVALS):
    t, shapes = datagen.serving_requests(rate, duration, seed=seed)
    k = len(t)
    return B.requests_array(t, shapes, [10_000_000 + i for i in range(k)], [20_000_000 + i for i in range(k)])


def _serve(reqs, serial, budget, streams, max_batch):
    o = B.conv2d_serve_defaults()
    o.serial_plain = 1 if serial else 0
    o.hbm_budget = budget
    o.streams = streams
    o.max_batch = max_batch
    rep, _, _ = B.conv2d_serve(reqs, o)
    d = rep.as_dict()
    keep = ("n_requests", "n_batches", "wall_s", "req_per_s", "gflops", "offered_rate", "p50_ms", "p99_ms",
            "mean_ms", "max_ms", "queue_p50_ms", "queue_p99_ms", "mean_batch", "stalled_requests", "peak_bytes")
    return {k: (round(d[k], 4) if isinstance(d[k], float) else d[k]) for k in keep}


def serve_benchmark(duration: float = 60.0, rates=(0.8,), budget_gib: float = 8.0, streams: int = 4,
                    max_batch: int = 64, probe_n: int = 3000) -> dict:
    budget = int(budget_gib * (1 << 30))
    # Capacity probes: every request arrives at t = 0.
    t, shapes = datagen.serving_requests(1e6, probe_n / 1e6 * 1.2, seed=datagen.SEED_ARRIVALS + 1)
    t = t[:probe_n] * 0.0
    probe = B.requests_array(t, shapes[:probe_n], [30_000_000 + i for i in range(len(t))],
                             [40_000_000 + i for i in range(len(t))])
    cap_serial = _serve(probe, True, budget, streams, max_batch)["req_per_s"]
    cap_batched = _serve(probe, False, budget, streams, max_batch)["req_per_s"]
    out = {"workload": "Poisson arrivals, sides log-uniform [128, 4096], filters {3,5,9,17}, images generated "
                       "on the device", "duration_s": duration, "hbm_budget_gib": budget_gib, "streams": streams,
           "max_batch": max_batch, "serial_capacity_req_s": round(cap_serial, 1),
           "batched_capacity_req_s": round(cap_batched, 1), "runs": []}
    for frac in rates:
        rate = frac * cap_serial
        reqs = _trace(rate, duration)
        run = {"rate_fraction_of_serial_capacity": frac, "rate_req_s": round(rate, 1), "n": len(reqs)}
        for mode, serial in (("batched", False), ("serial", True)):
            run[mode] = _serve(reqs, serial, budget, streams, max_batch)
            print(f"[serve] rate {frac} x serial capacity, {mode}: p50 {run[mode]['p50_ms']} ms, "
                  f"p99 {run[mode]['p99_ms']} ms", file=sys.stderr, flush=True)
        out["runs"].append(run)
    return out


HOTSPOT_FLOP_PER_CELL_STEP = 14
HOTSPOT_BYTES_PER_CELL_LAUNCH = 12   # read temperature and power, write temperature


def hotspot_benchmark(reps: int = 20, warmup: int = 3, steps: int = 60, rows: int = 4096, cols: int = 4096) -> dict:
    """Times whole runs of `steps` steps (HIP events on the current stream)."""
    torch = _torch()
    from .api import Hotspot
    temp, power, k = datagen.hotspot_problem(rows, cols)
    td = torch.from_numpy(temp).cuda()
    pd = torch.from_numpy(power).cuda()
    out = torch.empty_like(td)
    st = torch.cuda.current_stream()
    res = {"workload": f"hotspot chip {rows}x{cols}, {steps} steps", "steps": steps}
    for name, cfg in (("plan", None), ("default", B.hotspot_default_config().tuple())):
        plan = Hotspot(rows, cols, cfg)
        for _ in range(warmup):
            plan(td, pd, steps, k, out=out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            plan(td, pd, steps, k, out=out)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        launches = -(-steps // plan.config[4])
        res[name] = {
            "config": list(plan.config), "source": plan.source, "ms": round(ms, 4),
            "gflops": round(HOTSPOT_FLOP_PER_CELL_STEP * rows * cols * steps / (ms * 1e-3) / 1e9, 1),
            "launches": launches, "ms_per_launch": round(ms / launches, 4),
            "gbs_per_launch": round(HOTSPOT_BYTES_PER_CELL_LAUNCH * rows * cols / (ms / launches * 1e-3) / 1e9, 1),
        }
        plan.close()
    res["tuned_vs_default"] = round(res["default"]["ms"] / res["plan"]["ms"], 3)
    return res


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    b = sub.add_parser("batch")
    b.add_argument("--reps", type=int, default=20)
    s = sub.add_parser("serve")
    s.add_argument("--duration", type=float, default=60.0)
    s.add_argument("--rates", type=float, nargs="*", default=[0.8])
    s.add_argument("--budget-gib", type=float, default=8.0)
    s.add_argument("--streams", type=int, default=4)
    s.add_argument("--max-batch", type=int, default=64)
    h = sub.add_parser("hotspot")
    h.add_argument("--reps", type=int, default=20)
    h.add_argument("--steps", type=int, default=60)
    a = ap.parse_args(argv)
    if a.cmd == "batch":
        print(json.dumps(batch_benchmark(a.reps)), flush=True)
    elif a.cmd == "hotspot":
        print(json.dumps(hotspot_benchmark(a.reps, steps=a.steps)), flush=True)
    else:
        print(json.dumps(serve_benchmark(a.duration, tuple(a.rates), a.budget_gib, a.streams, a.max_batch)),
              flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
