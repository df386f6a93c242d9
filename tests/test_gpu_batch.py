"""GPU parity of the batched path (conv2d_batch_plan / conv2d_batch_run),
through the C ABI: the 64-problem uneven workload against the FP64 oracle and
bitwise against the plain path, graph replays, pointer changes, and errors."""
import os

import numpy as np
import pytest

import datagen
import oracle
from tests.gpu_util import TOL, say, torch_cuda

pytestmark = pytest.mark.gpu

C = pytest.importorskip("paper_2407_11488_amd")


def _device_problem(torch, shape, p):
    H, W, fh, fw = shape
    n_in = (H + fh - 1) * (W + fw - 1)
    inp = torch.empty((H + fh - 1, W + fw - 1), dtype=torch.float32, device="cuda")
    f = torch.empty((fh, fw), dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    C.conv2d_fill_uniform(inp.data_ptr(), n_in, datagen.SEED_BATCH_INPUT_BASE + p, 0, st)
    C.conv2d_fill_uniform(f.data_ptr(), fh * fw, datagen.SEED_BATCH_FILTER_BASE + p, 0, st)
    return inp, f


@pytest.fixture(scope="module")
def workload():
    torch = torch_cuda()
    shapes = datagen.batch_shapes()
    ins, fs = zip(*[_device_problem(torch, s, p) for p, s in enumerate(shapes)])
    torch.cuda.synchronize()
    return shapes, list(ins), list(fs)


def test_batch_uneven_workload_matches_oracle_and_plain(workload):
    """64 problems, square outputs log-uniform in [256, 2048], filters from
    {3, 5, 9, 17}: every output within tolerance of the FP64 oracle and bitwise
    equal to a plain conv2d_run of the same problem."""
    torch = torch_cuda()
    shapes, ins, fs = workload
    batch = C.Batch(shapes)
    say(f"batch groups {batch.info}")
    outs = [torch.full((H, W), float("nan"), device="cuda") for (H, W, _, _) in shapes]
    batch(ins, fs, outs)
    torch.cuda.synchronize()
    for p, (H, W, fh, fw) in enumerate(shapes):
        got = outs[p].cpu().numpy()
        assert np.all(np.isfinite(got)), p
        inp, f = datagen.conv_problem(H, W, fh, fw, seed_in=datagen.SEED_BATCH_INPUT_BASE + p,
                                      seed_f=datagen.SEED_BATCH_FILTER_BASE + p)
        assert np.array_equal(ins[p].cpu().numpy().view(np.uint32), inp.view(np.uint32))
        ref, s = oracle.conv2d_f64(inp, f)
        err = oracle.normalized_error(got, ref, s)
        assert err <= TOL, (p, err)
        plain = C.conv2d(ins[p], fs[p])
        torch.cuda.synchronize()
        assert np.array_equal(plain.cpu().numpy().view(np.uint32), got.view(np.uint32)), p
    batch.close()


def test_graph_replays_and_pointer_changes(workload):
    """The graph replayed several times, with eager work and synchronisation in
    between, and with new output buffers (descriptor re-upload): every replay
    equals the first result; the direct-launch path agrees."""
    torch = torch_cuda()
    shapes, ins, fs = workload
    sel = list(range(0, 64, 4))
    sub = [shapes[k] for k in sel]
    batch = C.Batch(sub)
    outs = [torch.full((H, W), float("nan"), device="cuda") for (H, W, _, _) in sub]
    batch([ins[k] for k in sel], [fs[k] for k in sel], outs)
    torch.cuda.synchronize()
    first = [o.cpu().numpy().copy() for o in outs]
    for rep in range(4):
        say(f"replay {rep}")
        for o in outs:
            o.fill_(float("nan"))                        # eager work between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        if rep == 2:
            outs = [torch.full((H, W), float("nan"), device="cuda") for (H, W, _, _) in sub]
        batch([ins[k] for k in sel], [fs[k] for k in sel], outs)
        torch.cuda.synchronize()
        for a, o in zip(first, outs):
            assert np.array_equal(a.view(np.uint32), o.cpu().numpy().view(np.uint32))
        del junk
    batch.close()
    direct = C.Batch(sub, flags=C.CONV2D_BATCH_NO_GRAPH)
    outs2 = direct([ins[k] for k in sel], [fs[k] for k in sel])
    torch.cuda.synchronize()
    for a, o in zip(first, outs2):
        assert np.array_equal(a.view(np.uint32), o.cpu().numpy().view(np.uint32))
    direct.close()
    # the bound form: tensors checked once, then repeated runs on them
    again = C.Batch(sub)
    outs3 = [torch.full((H, W), float("nan"), device="cuda") for (H, W, _, _) in sub]
    with pytest.raises(ValueError):
        again.bind([ins[k] for k in sel], [fs[k] for k in sel], outs3[1:] + outs3[:1])
    run = again.bind([ins[k] for k in sel], [fs[k] for k in sel], outs3)
    for _ in range(3):
        for o in outs3:
            o.fill_(float("nan"))
        run()
        torch.cuda.synchronize()
        for a, o in zip(first, outs3):
            assert np.array_equal(a.view(np.uint32), o.cpu().numpy().view(np.uint32))
    again.close()
    assert not again.handle
    with pytest.raises(RuntimeError, match="non-NULL"):   # a bound run after close() is refused
        run()


def test_batch_edge_cases():
    """One problem; tiny problems smaller than a tile; a rectangular filter."""
    torch = torch_cuda()
    shapes = [(1, 1, 3, 3), (2, 300, 5, 5), (77, 1, 17, 17), (33, 65, 3, 7), (40, 40, 3, 3)]
    ins, fs = zip(*[_device_problem(torch, s, 50 + p) for p, s in enumerate(shapes)])
    for sub in (shapes[:1], shapes):
        b = C.Batch(sub)
        outs = b(list(ins[:len(sub)]), list(fs[:len(sub)]))
        torch.cuda.synchronize()
        for p, (H, W, fh, fw) in enumerate(sub):
            inp, f = datagen.conv_problem(H, W, fh, fw, seed_in=datagen.SEED_BATCH_INPUT_BASE + 50 + p,
                                          seed_f=datagen.SEED_BATCH_FILTER_BASE + 50 + p)
            ref, s = oracle.conv2d_f64(inp, f)
            assert oracle.normalized_error(outs[p].cpu().numpy(), ref, s) <= TOL
        b.close()


def test_batch_many_filter_sizes():
    """Eleven filter sizes (eleven kernels as graph branches),
    uneven images, integer data: bitwise equal to the oracle on every replay."""
    torch = torch_cuda()
    filters = [(1, 1), (3, 3), (5, 5), (7, 7), (9, 9), (11, 11), (2, 6), (6, 2), (17, 17), (31, 31), (4, 4)]
    shapes = [(40 + 13 * k, 70 - 5 * k, fh, fw) for k, (fh, fw) in enumerate(filters)]
    shapes += [(9, 300, fh, fw) for fh, fw in filters[::3]]
    probs = [datagen.conv_problem(H, W, fh, fw, kind="int", seed_in=700 + p, seed_f=800 + p)
             for p, (H, W, fh, fw) in enumerate(shapes)]
    ins = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a, _ in probs]
    fs = [torch.from_numpy(np.ascontiguousarray(f)).cuda() for _, f in probs]
    b = C.Batch(shapes)
    say(f"many filters: {b.info['n_groups']} groups")
    assert b.info["n_groups"] == len(filters)
    for rep in range(3):
        outs = b(ins, fs)
        torch.cuda.synchronize()
        for p, (inp, f) in enumerate(probs):
            ref, _ = oracle.conv2d_f64(inp, f)
            assert np.array_equal(outs[p].cpu().numpy().astype(np.float64), ref), (rep, p)
    b.close()


def test_batch_integer_data_bitwise():
    """Integer data (inputs and filters in [-4, 4]) keeps every partial sum an
    exact integer, so each output of an uneven batch over all four filter
    sizes equals the FP64 oracle bit for bit."""
    torch = torch_cuda()
    shapes = [(300, 257, 17, 17), (77, 401, 9, 9), (256, 256, 5, 5), (129, 65, 3, 3), (1, 1, 17, 17),
              (520, 33, 9, 9), (33, 520, 3, 3), (1000, 3, 5, 5)]
    probs = [datagen.conv_problem(*s, kind="int", seed_in=300 + k, seed_f=400 + k) for k, s in enumerate(shapes)]
    b = C.Batch(shapes)
    ins = [torch.from_numpy(i).cuda() for i, _ in probs]
    fs = [torch.from_numpy(f).cuda() for _, f in probs]
    outs = [torch.full((H, W), float("nan"), device="cuda") for (H, W, _, _) in shapes]
    b(ins, fs, outs)
    torch.cuda.synchronize()
    for k, (inp, f) in enumerate(probs):
        ref, _ = oracle.conv2d_f64(inp, f)
        assert np.array_equal(outs[k].cpu().numpy().astype(np.float64), ref), shapes[k]
    b.close()


def test_batch_thousands_of_tiny_problems():
    """2,000 problems of 1-40 pixels a side with 1x1, 2x3 and 5x5 filters
    (descriptor and owner tables far larger than a workgroup's tile list,
    many problems per tile-owner run, images smaller than one tile), integer
    data: every output equals the oracle bit for bit."""
    torch = torch_cuda()
    rng = np.random.default_rng(17)
    filters = [(1, 1), (2, 3), (5, 5)]
    shapes = []
    for k in range(2000):
        fh, fw = filters[k % 3]
        shapes.append((int(rng.integers(1, 41)), int(rng.integers(1, 41)), fh, fw))
    probs = [datagen.conv_problem(*s, kind="int", seed_in=5000 + k, seed_f=9000 + k) for k, s in enumerate(shapes)]
    b = C.Batch(shapes)
    say(f"tiny batch: {b.info['n_groups']} groups, {b.info['total_tiles']} tiles")
    ins = [torch.from_numpy(i).cuda() for i, _ in probs]
    fs = [torch.from_numpy(f).cuda() for _, f in probs]
    outs = [torch.full((H, W), float("nan"), device="cuda") for (H, W, _, _) in shapes]
    b(ins, fs, outs)
    torch.cuda.synchronize()
    bad = []
    for k, (inp, f) in enumerate(probs):
        ref, _ = oracle.conv2d_f64(inp, f)
        if not np.array_equal(outs[k].cpu().numpy().astype(np.float64), ref):
            bad.append(k)
    assert not bad, bad[:10]
    b.close()


def test_batch_errors():
    torch = torch_cuda()
    with pytest.raises(C.Conv2dError):
        C.conv2d_batch_plan([])
    with pytest.raises(C.Conv2dError):
        C.conv2d_batch_plan([(10, 10, 3, 3), (0, 10, 3, 3)])
    b = C.conv2d_batch_plan([(10, 10, 3, 3)])
    try:
        inp = torch.zeros((12, 12), device="cuda")
        f = torch.zeros((3, 3), device="cuda")
        with pytest.raises(C.Conv2dError):
            C.conv2d_batch_run(b, [inp.data_ptr()], [f.data_ptr()], [0])
        with pytest.raises(C.Conv2dError):
            C.conv2d_batch_run(b, [inp.data_ptr()], [f.data_ptr()], [inp.data_ptr()])
    finally:
        C.conv2d_batch_destroy(b)


def _tune_env(tmp_path):
    import shutil
    wp = tmp_path / "winners.jsonl"
    here = os.path.join(os.path.dirname(C.LIB_PATH), "tuned")
    shutil.copy(os.path.join(here, "winners.jsonl"), wp)
    for f in (3, 9):
        src = os.path.join(here, f"results_gfx950_4096x4096_{f}x{f}.jsonl")
        if os.path.exists(src):
            shutil.copy(src, tmp_path / os.path.basename(src))
    return wp


def _check_batch_matches_oracle(torch, b, shapes, base):
    ins, fs = zip(*[_device_problem(torch, s, base + p) for p, s in enumerate(shapes)])
    outs = b(list(ins), list(fs))
    torch.cuda.synchronize()
    for p, (H, W, fh, fw) in enumerate(shapes):
        inp, f = datagen.conv_problem(H, W, fh, fw, seed_in=datagen.SEED_BATCH_INPUT_BASE + base + p,
                                      seed_f=datagen.SEED_BATCH_FILTER_BASE + base + p)
        ref, s = oracle.conv2d_f64(inp, f)
        assert oracle.normalized_error(outs[p].cpu().numpy(), ref, s) <= TOL, p


def test_batch_tune_stores_and_is_used(tmp_path, monkeypatch):
    """conv2d_batch_tune on a small two-filter batch: every filter size gets a
    verified winner no slower than the current choice, stored as the
    (0, 0, fh, fw) entry; a batch planned afterwards uses it, and its outputs
    still match the oracle."""
    torch = torch_cuda()
    wp = _tune_env(tmp_path)
    shapes = [(300, 300, 9, 9), (200, 260, 9, 9), (150, 150, 3, 3), (520, 400, 3, 3)]
    o = C.conv2d_batch_tune_defaults()
    o.winners_path = str(wp).encode()
    o.results_dir = str(tmp_path).encode()
    o.candidates, o.reps = 4, 5
    r = C.conv2d_batch_tune(shapes, o)
    groups = r.groups()
    say(f"batch tune: {groups}")
    assert r.n_groups == 2
    for g in groups:
        assert g["tried"] >= 1 and g["after_ms"] > 0 and g["bucket"] == 0
        assert g["after_ms"] <= g["before_ms"] * (1 + o.tie_rel) + 1e-9
        got = C.conv2d_cache_lookup(str(wp), None, C.shape(0, 0, *g["filter"]))[0].tuple()
        assert got == tuple(g["after"])
    monkeypatch.setenv("CONV2D_WINNERS", str(wp))
    b = C.Batch(shapes)
    used = {tuple(x["filter"]): tuple(x["config"]) for x in b.info["groups"]}
    for g in groups:
        assert used[tuple(g["filter"])][:6] == tuple(g["after"])[:6]   # the build may roll the row loop
    _check_batch_matches_oracle(torch, b, shapes, 90)
    b.close()


def test_batch_tune_by_size_bucket(tmp_path, monkeypatch):
    """With buckets on, one entry (0, b, fh, fw) per filter size and size
    bucket; a CONV2D_BATCH_BY_SIZE batch planned afterwards gives each problem
    its bucket's configuration (one kernel per distinct filter and
    configuration) and still matches the oracle, a problem of a bucket with no
    entry falling back to the filter's other entries; a plain batch keeps one
    kernel per filter size, its whole-batch entry."""
    torch = torch_cuda()
    wp = _tune_env(tmp_path)
    tuned = [(200, 200, 9, 9), (300, 260, 9, 9), (1100, 900, 9, 9), (150, 150, 3, 3), (700, 600, 3, 3)]
    o = C.conv2d_batch_tune_defaults()
    o.winners_path = str(wp).encode()
    o.results_dir = str(tmp_path).encode()
    o.candidates, o.reps, o.buckets = 3, 5, 1
    r = C.conv2d_batch_tune(tuned, o)
    groups = r.groups()
    say(f"bucket tune: {groups}")
    assert sorted((g["filter"][0], g["bucket"], g["problems"]) for g in groups) == \
        [(3, 1, 1), (3, 2, 1), (9, 1, 2), (9, 3, 1)]
    for g in groups:
        got = C.conv2d_cache_lookup(str(wp), None, C.shape(0, g["bucket"], *g["filter"]))[0].tuple()
        assert got == tuple(g["after"])
    monkeypatch.setenv("CONV2D_WINNERS", str(wp))
    shapes = tuned + [(2000, 1800, 9, 9)]          # bucket 4 of 9x9 has no entry of its own
    b = C.Batch(shapes, flags=C.CONV2D_BATCH_BY_SIZE)
    info = b.info["groups"]
    want = {(g["filter"][0], tuple(g["after"])[:6]) for g in groups}
    have = {(x["filter"][0], tuple(x["config"])[:6]) for x in info}
    assert want <= have                                               # every bucket's winner is used
    assert len(info) == len({(x["filter"][0], tuple(x["config"])) for x in info})   # one kernel per config
    _check_batch_matches_oracle(torch, b, shapes, 120)
    b.close()
    # without the flag, a filter's whole-batch entry wins: one kernel per filter
    whole = C.Batch(shapes)
    assert sorted(x["filter"][0] for x in whole.info["groups"]) == [3, 9]
    for x in whole.info["groups"]:
        got = C.conv2d_cache_lookup(str(wp), None, C.shape(0, 0, *x["filter"]))
        if got is not None:
            assert tuple(x["config"])[:6] == got[0].tuple()[:6]
    whole.close()


def test_batch_context_tune_stores_and_is_used(tmp_path, monkeypatch):
    """The in-context tuning of the batched path (workloads.batch_context_tune)
    on the first 12 problems of the batched workload, two candidates per
    group, one pass: every trial's outputs equal the first trial's bit for
    bit (checked inside), the result covers every filter group, the chosen
    configurations are appended as the (0, 0, fh, fw) winners, and a batch
    planned afterwards uses them and matches the oracle."""
    import shutil

    from paper_2407_11488_amd import workloads
    torch = torch_cuda()
    wp = tmp_path / "winners.jsonl"
    shutil.copy(os.path.join(os.path.dirname(C.LIB_PATH), "tuned", "winners.jsonl"), wp)
    monkeypatch.delenv("CONV2D_WINNERS", raising=False)
    r = workloads.batch_context_tune(n=12, candidates=2, rounds=1, reps=5, winners=str(wp), log=say)
    say(f"batch context tune: {r}")
    shapes = datagen.batch_shapes(12)
    filters = sorted({s[2] for s in shapes})
    assert sorted(int(f) for f in r["assignment"]) == filters
    assert r["trials"] >= 1 and r["final_ms"] > 0 and r["best_ms"] <= r["start_ms"]
    assert os.environ.get("CONV2D_WINNERS") is None          # restored
    for f, cfg in r["assignment"].items():
        got = C.conv2d_cache_lookup(str(wp), None, C.shape(0, 0, int(f), int(f)))[0].tuple()
        assert got == tuple(cfg)
    monkeypatch.setenv("CONV2D_WINNERS", str(wp))
    b = C.Batch(shapes)
    used = {x["filter"][0]: tuple(x["config"]) for x in b.info["groups"]}
    for f, cfg in r["assignment"].items():
        assert used[int(f)][:6] == tuple(cfg)[:6]   # the build may roll the row loop
    _check_batch_matches_oracle(torch, b, shapes, 130)
    b.close()
