"""GPU runs of the two tuners through the C ABI on small problems: every
configuration compiled, verified and timed, the winner cached, a plan made
afterwards picking it up and matching the FP64 oracle, and a second run
resuming from the results file."""
import json

import numpy as np
import pytest

import datagen
import oracle
from tests.gpu_util import TOL, say, torch_cuda
from tests.test_gpu_hotspot import bound as hotspot_bound

pytestmark = pytest.mark.gpu
C = pytest.importorskip("paper_2407_11488_amd")

CONV_SHAPE = (512, 512, 5, 5)
N_CONFIGS = 24


def _conv_opts(tmp_path):
    o = C.conv2d_tune_defaults()
    o.winners_path = str(tmp_path / "winners.jsonl").encode()
    o.results_path = str(tmp_path / "results.jsonl").encode()
    o.max_configs, o.reps, o.warmup, o.retime_reps = N_CONFIGS, 5, 1, 10
    return o


def test_conv_tuner_sweep_cache_and_resume(tmp_path, monkeypatch):
    torch = torch_cuda()
    s = C.shape(*CONV_SHAPE)
    o = _conv_opts(tmp_path)
    r = C.conv2d_tune(s, o)
    best = r.best.tuple()
    say(f"conv tune {CONV_SHAPE}: best {best} {r.best_ms:.4f} ms, median {r.median_ms:.4f}, "
        f"default {r.default_ms:.4f}, timed {r.n_timed}")
    assert r.n_compile_fail == r.n_launch_fail == r.n_verify_fail == 0
    assert r.n_timed >= N_CONFIGS and r.n_resumed == 0
    space = C.conv2d_space(s)[:N_CONFIGS]
    assert best in space or best == C.conv2d_default_config().tuple()
    assert r.best_ms > 0 and r.median_ms > 0
    assert (r.default_rank > 0) == (r.default_ms > 0)   # the default is timed only when in the swept part
    assert r.impact >= 1.0                      # fastest over median throughput, both from the sweep
    assert r.median_gflops == pytest.approx(2 * 512 * 512 * 25 / (r.median_ms * 1e-3) / 1e9, rel=1e-6)
    assert r.best_gflops == pytest.approx(2 * 512 * 512 * 25 / (r.best_ms * 1e-3) / 1e9, rel=1e-6)
    top_ms = [r.top_ms[k] for k in range(5)]
    assert top_ms == sorted(top_ms)
    assert r.top[0].tuple() == best or top_ms[0] <= r.best_ms
    # the results file holds one line per timed point, the cache the winner
    lines = [json.loads(x) for x in (tmp_path / "results.jsonl").read_text().splitlines() if x.strip()]
    assert len(lines) >= r.n_timed and all(x["status"] == "ok" for x in lines)
    got = C.conv2d_cache_lookup(str(tmp_path / "winners.jsonl"), None, s)
    assert got is not None and got[0].tuple() == best
    # a plan made afterwards takes the winner and matches the oracle
    monkeypatch.setenv("CONV2D_WINNERS", str(tmp_path / "winners.jsonl"))
    plan = C.Plan(*CONV_SHAPE)
    assert tuple(plan.config) == best and plan.source == "tuned"
    inp, f = datagen.conv_problem(*CONV_SHAPE)
    out = plan(torch.from_numpy(inp).cuda(), torch.from_numpy(f).cuda())
    torch.cuda.synchronize()
    ref, sabs = oracle.conv2d_f64(inp, f)
    assert oracle.normalized_error(out.cpu().numpy(), ref, sabs) <= TOL
    plan.close()
    # a second run resumes every point from the results file
    r2 = C.conv2d_tune(s, _conv_opts(tmp_path))
    say(f"resumed {r2.n_resumed} of {r2.n_timed}")
    assert r2.n_resumed >= N_CONFIGS and r2.n_verify_fail == 0


def test_hotspot_tuner_sweep_and_cache(tmp_path, monkeypatch):
    torch = torch_cuda()
    rows, cols, steps = 256, 320, 6
    s = C.hotspot_shape(rows, cols)
    o = C.hotspot_tune_defaults()
    o.winners_path = str(tmp_path / "hs_winners.jsonl").encode()
    o.results_path = str(tmp_path / "hs_results.jsonl").encode()
    o.max_configs, o.reps, o.warmup, o.retime_reps = 20, 5, 1, 10
    r = C.hotspot_tune(s, steps, o)
    best = r.best.tuple()
    say(f"hotspot tune {rows}x{cols}/{steps}: best {best} {r.best_ms:.4f} ms, timed {r.n_timed}")
    assert r.n_compile_fail == r.n_launch_fail == r.n_verify_fail == 0
    assert r.n_timed >= 20 and r.best_ms > 0
    assert r.best_gflops == pytest.approx(14 * rows * cols * steps / (r.best_ms * 1e-3) / 1e9, rel=1e-6)
    monkeypatch.setenv("HOTSPOT_WINNERS", str(tmp_path / "hs_winners.jsonl"))
    hs = C.Hotspot(rows, cols)
    assert tuple(hs.config) == best and hs.source == "tuned"
    temp, power, k = datagen.hotspot_problem(rows, cols)
    out = hs(torch.from_numpy(temp).cuda(), torch.from_numpy(power).cuda(), steps, k)
    torch.cuda.synchronize()
    ref = oracle.hotspot_f64(temp, power, steps, *k)
    got = out.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - ref)) <= hotspot_bound(temp, power, steps, k)
    hs.close()


def test_conv_tuner_local_search_on_gpu(tmp_path):
    """The local-search strategy with real timings: exactly max_evals points
    evaluated, all verified, the winner among them and cached."""
    s = C.shape(*CONV_SHAPE)
    o = _conv_opts(tmp_path)
    o.max_configs = 0
    o.strategy, o.max_evals, o.seed = 1, 30, 5
    r = C.conv2d_tune(s, o)
    say(f"local search {CONV_SHAPE}: best {r.best.tuple()} {r.best_ms:.4f} ms, evaluations {r.evaluations}")
    assert r.evaluations == 30 and r.n_verify_fail == 0 and r.n_launch_fail == 0
    lines = [json.loads(x) for x in (tmp_path / "results.jsonl").read_text().splitlines() if x.strip()]
    evaluated = {tuple(x["config"]) for x in lines}
    assert len(evaluated) == 30 and r.best.tuple() in evaluated
    got = C.conv2d_cache_lookup(str(tmp_path / "winners.jsonl"), None, s)
    assert got is not None and got[0].tuple() == r.best.tuple()


def test_benchmark_one_configuration():
    """conv2d_benchmark times one configuration the tuner's way: a verified
    launch, then timed launches; the median is at least the minimum, both
    positive; a configuration illegal for the shape is rejected."""
    s = C.shape(*CONV_SHAPE)
    cfg = (64, 2, 4, 4, 1, 0, 1)
    med, mn = C.conv2d_benchmark(s, cfg, 1, 7, 1)
    say(f"benchmark {cfg}: median {med:.4f} ms, min {mn:.4f} ms")
    assert 0 < mn <= med
    with pytest.raises(C.Conv2dError):
        C.conv2d_benchmark(C.shape(64, 64, 63, 63), (128, 8, 8, 8, 1, 0, 1), 1, 3, 0)   # LDS too large
