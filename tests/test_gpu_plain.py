"""GPU parity of the plain path (conv2d_plan / conv2d_run) against the FP64
oracle, through the C ABI."""
import numpy as np
import pytest

import datagen
import oracle
from tests.gpu_util import TOL, VEC, nan_like, precompile, run_config, say, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

C = pytest.importorskip("paper_2407_11488_amd")


def _check_uniform(out_dev, inp, filt, tol=TOL):
    ref, s = oracle.conv2d_f64(inp, filt)
    got = out_dev.cpu().numpy()
    assert np.all(np.isfinite(got)), "unwritten (NaN) outputs"
    err = oracle.normalized_error(got, ref, s)
    assert err <= tol, f"normalised error {err:.3e} > {tol}"
    return got


def test_device_generator_matches_host():
    torch = torch_cuda()
    n = 1 << 20
    d = torch.empty(n, dtype=torch.float32, device="cuda")
    say("fill_uniform seed 7 start 123")
    C.conv2d_fill_uniform(d.data_ptr(), n, 7, 123, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy().view(np.uint32), datagen.uniform_pm1(7, n, start=123).view(np.uint32))


def test_reference_kernel_matches_oracle():
    for (H, W, fh, fw) in [(1, 1, 1, 1), (37, 53, 17, 17), (64, 3, 5, 9), (5, 200, 31, 3)]:
        inp, f = datagen.conv_problem(H, W, fh, fw, seed_in=3, seed_f=4)
        say(f"reference {H}x{W} f{fh}x{fw}")
        out = C.reference(to_dev(inp), to_dev(f))
        torch_cuda().cuda.synchronize()
        _check_uniform(out, inp, f)
        ia, fa = datagen.conv_problem(H, W, fh, fw, kind="int")
        out = C.reference(to_dev(ia), to_dev(fa))
        ref, _ = oracle.conv2d_f64(ia, fa)
        assert np.array_equal(out.cpu().numpy().astype(np.float64), ref)


def test_plain_workload_default_config():
    """Output 1024x1024, filter 17x17, input 1040x1040 with a zero halo, the
    default configuration, no tuning."""
    inp, f = datagen.conv_problem(1024, 1024, 17, 17, zero_halo=True)
    say("plain 1024x1024 f17 default config")
    out = run_config(C, to_dev(inp), to_dev(f), C.conv2d_default_config())
    _check_uniform(out, inp, f)


def test_whole_space_integer_data_bitwise():
    """Every one of the 1216 configurations on a ragged shape that spans several
    tiles: integer data makes every partial sum exact, so each configuration
    must equal the oracle bit for bit."""
    H, W, fh, fw = 70, 45, 5, 3
    s = C.shape(H, W, fh, fw)
    every = C.conv2d_space(s, 1, -1)
    assert len(every) == 1216
    cfgs = [c for c in every if C.conv2d_config_check(s, c) == 0]
    illegal = [c for c in every if c not in cfgs]
    assert all(C.conv2d_lds_bytes(fh, fw, c) > 163840 for c in illegal)
    for c in illegal:
        with pytest.raises(C.Conv2dError):
            C.conv2d_plan(s, c)
    precompile(C, s, cfgs, VEC, VEC)
    inp, f = datagen.conv_problem(H, W, fh, fw, kind="int", seed_in=8, seed_f=9)
    ref, _ = oracle.conv2d_f64(inp, f)
    di, df = to_dev(inp), to_dev(f)
    bad = []
    for k, c in enumerate(cfgs):
        if k % 200 == 0:
            say(f"whole space: config {k}/{len(cfgs)} {c}")
        got = run_config(C, di, df, c).cpu().numpy().astype(np.float64)
        if not np.array_equal(got, ref):
            bad.append(c)
    assert not bad, f"{len(bad)} configurations differ, first {bad[:5]}"


STRATIFIED = [
    (16, 16, 1, 1, 1, 1), (16, 1, 1, 1, 0, 0), (32, 2, 2, 4, 0, 1), (64, 1, 2, 4, 0, 0), (64, 1, 8, 8, 0, 0),
    (64, 1, 8, 8, 1, 0), (64, 4, 4, 8, 1, 1), (128, 1, 8, 4, 0, 1), (128, 8, 1, 2, 1, 0), (16, 16, 8, 8, 0, 0),
    (32, 16, 4, 1, 1, 1), (128, 4, 2, 8, 0, 0), (64, 2, 1, 8, 1, 0), (16, 4, 8, 2, 1, 1), (128, 1, 4, 1, 1, 1),
    (32, 8, 8, 1, 0, 1),
]


@pytest.mark.parametrize("fh,fw", [(17, 17), (3, 3), (7, 7), (15, 15), (31, 31), (1, 1), (5, 9), (9, 5),
                                   (1, 7), (7, 1)])
def test_stratified_configs_uniform(fh, fw):
    """Uniform data on a ragged shape: each configuration within tolerance of the
    oracle, no unwritten outputs, and all configurations bitwise identical
    (fixed accumulation order)."""
    H, W = 203, 317
    s = C.shape(H, W, fh, fw)
    cfgs = [c + (1,) for c in STRATIFIED if C.conv2d_config_check(s, c + (1,)) == 0]
    precompile(C, s, cfgs, VEC, VEC)
    inp, f = datagen.conv_problem(H, W, fh, fw, seed_in=10 + fh, seed_f=20 + fw)
    di, df = to_dev(inp), to_dev(f)
    first = None
    for c in cfgs:
        say(f"uniform {H}x{W} f{fh}x{fw} cfg {c}")
        got = _check_uniform(run_config(C, di, df, c), inp, f)
        if first is None:
            first = got
        else:
            assert np.array_equal(got.view(np.uint32), first.view(np.uint32)), c


@pytest.mark.parametrize("cfg", [(64, 1, 8, 8, 0, 0, 1), (16, 16, 1, 1, 1, 1, 1), (64, 2, 4, 4, 1, 0, 2),
                                 (64, 1, 2, 4, 0, 1, 0), (32, 4, 8, 2, 0, 0, 4)])
def test_unroll_and_alignment_variants(cfg):
    """Unroll factors, and input/output pointers one float past a 16-byte
    boundary (views offset by one float), which the plan's one module (4-wide
    loads and stores at any dword offset) takes as they are."""
    torch = torch_cuda()
    H, W, fh, fw = 129, 260, 17, 17
    inp, f = datagen.conv_problem(H, W, fh, fw, seed_in=31, seed_f=32)
    say(f"unroll/alignment cfg {cfg}")
    out = run_config(C, to_dev(inp), to_dev(f), cfg)
    _check_uniform(out, inp, f)
    big_in = torch.zeros(inp.size + 1, dtype=torch.float32, device="cuda")
    big_in[1:] = to_dev(inp).reshape(-1)
    big_out = torch.full((H * W + 1,), float("nan"), dtype=torch.float32, device="cuda")
    s = C.shape(H, W, fh, fw)
    plan = C.conv2d_plan(s, cfg)
    try:
        C.conv2d_run(plan, big_in.data_ptr() + 4, to_dev(f).data_ptr(), big_out.data_ptr() + 4,
                     torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
    finally:
        C.conv2d_destroy(plan)
    got = big_out[1:].reshape(H, W)
    assert np.array_equal(got.cpu().numpy().view(np.uint32), out.cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("fh,fw", [(63, 63), (1, 63), (63, 1)])
def test_largest_filters_integer_bitwise(fh, fw):
    """The largest filters the library accepts (63 taps a side), constant and
    global filter placement, with and without LDS: integer data keeps every
    partial sum an integer below 2^24 (63*63*16 < 2^16), so each output equals
    the oracle bit for bit."""
    H, W = 70, 90
    s = C.shape(H, W, fh, fw)
    cfgs = [c for c in [(64, 1, 1, 1, 0, 0, 1), (16, 16, 2, 2, 1, 0, 1), (32, 4, 4, 2, 0, 1, 1),
                        (128, 2, 2, 4, 1, 1, 1)] if C.conv2d_config_check(s, c) == 0]
    assert len(cfgs) >= 3
    precompile(C, s, cfgs, VEC, VEC)
    inp, f = datagen.conv_problem(H, W, fh, fw, kind="int", seed_in=41, seed_f=42)
    ref, _ = oracle.conv2d_f64(inp, f)
    di, df = to_dev(inp), to_dev(f)
    for c in cfgs:
        say(f"largest filter {fh}x{fw} cfg {c}")
        got = run_config(C, di, df, c).cpu().numpy().astype(np.float64)
        assert np.array_equal(got, ref), c
    with pytest.raises(C.Conv2dError):
        C.conv2d_plan(C.shape(H, W, fh + (fh == 63), fw + (fw == 63)), None)


@pytest.mark.parametrize("fsize", [17, 3, 5, 7, 9, 15, 31])
def test_full_size_whole_image(fsize):
    """4096x4096 outputs with each filter of the filter-size sweep, in the
    configuration the plan picks (the tuned winner when the winners cache
    holds one, the configuration the benchmark times): every one of the 16.8 M
    outputs within tolerance of the full FP64 oracle, and bit for bit equal to
    the reference kernel (same accumulation order) on the same buffers."""
    torch = torch_cuda()
    H = W = 4096
    fh = fw = fsize
    n_in = (H + fh - 1) * (W + fw - 1)
    inp = datagen.uniform_pm1(1, n_in).reshape(H + fh - 1, W + fw - 1)
    f = datagen.uniform_pm1(2, fh * fw).reshape(fh, fw)
    plan = C.Plan(H, W, fh, fw)
    say(f"full size 4096 f{fsize} with {plan.source} config {plan.config}")
    di, df = to_dev(inp), to_dev(f)
    out = plan(di, df, out=nan_like(H, W))
    ref_dev = C.reference(di, df, out=nan_like(H, W))
    torch.cuda.synchronize()
    plan.close()
    mism = int((out.view(torch.int32) != ref_dev.view(torch.int32)).sum().item())
    assert mism == 0, f"{mism} outputs differ from the reference kernel"
    got = out.cpu().numpy()
    del out, ref_dev, di
    ref, s = oracle.conv2d_f64(inp, f)
    err = oracle.normalized_error(got, ref, s)
    say(f"full size 4096 f{fsize}: normalised error {err:.3e}")
    assert err <= TOL, err


def test_full_size_integer_data_bitwise():
    """4096x4096 / 17x17 with integer data in [-4, 4] in the plan's (tuned)
    configuration: every partial sum is an integer below 2^24, so the whole
    output equals the FP64 oracle bit for bit."""
    torch = torch_cuda()
    H = W = 4096
    inp, f = datagen.conv_problem(H, W, 17, 17, kind="int", seed_in=81, seed_f=82)
    plan = C.Plan(H, W, 17, 17)
    say(f"full size 4096 f17 integer data with {plan.source} config {plan.config}")
    out = plan(to_dev(inp), to_dev(f), out=nan_like(H, W))
    torch.cuda.synchronize()
    plan.close()
    got = out.cpu().numpy().astype(np.float64)
    ref, _ = oracle.conv2d_f64(inp, f, with_abs=False)
    assert np.array_equal(got, ref), int(np.count_nonzero(got != ref))


@pytest.mark.parametrize("H,W,fsize", [(4093, 4095, 17), (4095, 4093, 3), (4094, 4093, 9), (2049, 4094, 5)])
def test_full_size_odd_widths_integer_bitwise(H, W, fsize):
    """Outputs whose rows are 1, 2 or 3 floats past a multiple of 4, so that
    the plan's four-dword stores start at every dword position of a 16-byte
    line, in the configuration the plan picks (the filter's 4096x4096
    winner): with integer data in [-4, 4] every partial sum is an integer
    below 2^24 and the whole output equals the FP64 oracle bit for bit."""
    torch = torch_cuda()
    inp, f = datagen.conv_problem(H, W, fsize, fsize, kind="int", seed_in=91, seed_f=92)
    plan = C.Plan(H, W, fsize, fsize)
    say(f"odd width {H}x{W} f{fsize} with {plan.source} config {plan.config}")
    out = plan(to_dev(inp), to_dev(f), out=nan_like(H, W))
    torch.cuda.synchronize()
    plan.close()
    got = out.cpu().numpy().astype(np.float64)
    del out
    ref, _ = oracle.conv2d_f64(inp, f, with_abs=False)
    assert np.array_equal(got, ref), int(np.count_nonzero(got != ref))


def test_input_above_2gib_runs_in_bands():
    """An input above 2 GiB (output 24000 x 24000, 3 x 3 filter: 2.3 GB) runs
    as several launches over horizontal bands (32-bit buffer offsets): sampled
    outputs on both sides of every band boundary, at the corners and inside
    match the oracle, each computed from the generator's values of its own
    window; every sampled output finite."""
    torch = torch_cuda()
    H = W = 24000
    fh = fw = 3
    P = W + fw - 1
    n_in = (H + fh - 1) * P
    assert 4 * n_in > 2**31
    st = torch.cuda.current_stream().cuda_stream
    d_in = torch.empty(n_in, dtype=torch.float32, device="cuda")
    d_f = torch.empty(fh * fw, dtype=torch.float32, device="cuda")
    C.conv2d_fill_uniform(d_in.data_ptr(), n_in, 61, 0, st)
    C.conv2d_fill_uniform(d_f.data_ptr(), fh * fw, 62, 0, st)
    plan = C.Plan(H, W, fh, fw)
    say(f"banded 24000x24000 f3 with {plan.source} config {plan.config}")
    out = torch.full((H, W), float("nan"), dtype=torch.float32, device="cuda")
    C.conv2d_run(plan.handle, d_in.data_ptr(), d_f.data_ptr(), out.data_ptr(), st)
    torch.cuda.synchronize()
    rows = (2**31 - 1) // (4 * P) - (fh - 1)          # output rows per band
    assert rows < H
    bounds = list(range(rows, H, rows))
    rng = np.random.default_rng(7)
    ys = [0, 0, H - 1, H - 1] + [b + d for b in bounds for d in (-2, -1, 0, 1)] + list(rng.integers(0, H, 40))
    xs = [0, W - 1, 0, W - 1] + [int(v) for v in rng.integers(0, W, 4 * len(bounds))] + list(rng.integers(0, W, 40))
    f = datagen.uniform_pm1(62, fh * fw).reshape(fh, fw)
    for y, x in zip(ys, xs):
        win = np.stack([datagen.uniform_pm1(61, fw, start=(y + i) * P + x) for i in range(fh)])
        ref, sabs = oracle.conv2d_f64(win, f)
        v = out[y, x].item()
        assert np.isfinite(v), (y, x)
        assert oracle.normalized_error(np.array([[v]], np.float32), ref, sabs) <= TOL, (y, x)
    plan.close()
    del out, d_in


def test_untuned_shape_takes_the_filters_winner(tmp_path, monkeypatch):
    """A shape with no winners entry of its own takes the same filter's
    4096 x 4096 winner (source "tuned-other-shape"); a filter with no entry
    at all takes the default; either way the result matches the oracle."""
    torch = torch_cuda()
    wp = tmp_path / "winners.jsonl"
    cfg = (64, 2, 4, 4, 1, 0, 1)
    C.conv2d_cache_store(str(wp), "gfx950", C.shape(4096, 4096, 9, 9), cfg, 1.0)
    monkeypatch.setenv("CONV2D_WINNERS", str(wp))
    for (H, W, fh, fw), want in (((300, 260, 9, 9), ("tuned-other-shape", cfg)),
                                 ((300, 260, 7, 7), ("default", C.conv2d_default_config().tuple()))):
        plan = C.Plan(H, W, fh, fw)
        say(f"untuned {H}x{W} f{fh}: {plan.source} {plan.config}")
        assert (plan.source, tuple(plan.config)) == want
        inp, f = datagen.conv_problem(H, W, fh, fw, seed_in=71, seed_f=72)
        out = plan(to_dev(inp), to_dev(f))
        torch.cuda.synchronize()
        _check_uniform(out, inp, f)
        plan.close()


def test_errors_are_reported_not_faulted():
    torch = torch_cuda()
    s = C.shape(64, 64, 5, 5)
    plan = C.conv2d_plan(s, (64, 1, 4, 4, 0, 0, 1))
    try:
        inp = torch.zeros((68, 68), dtype=torch.float32, device="cuda")
        f = torch.zeros((5, 5), dtype=torch.float32, device="cuda")
        out = torch.empty((64, 64), dtype=torch.float32, device="cuda")
        st = torch.cuda.current_stream().cuda_stream
        with pytest.raises(C.Conv2dError) as e:
            C.conv2d_run(plan, inp.data_ptr(), f.data_ptr(), 0, st)
        assert e.value.status == C.CONV2D_EINVAL
        with pytest.raises(C.Conv2dError):
            C.conv2d_run(plan, inp.data_ptr() + 2, f.data_ptr(), out.data_ptr(), st)  # not 4-byte aligned
        host = np.zeros(64 * 64, np.float32)
        with pytest.raises(C.Conv2dError):
            C.conv2d_run(plan, inp.data_ptr(), f.data_ptr(), host.ctypes.data, st)
        with pytest.raises(C.Conv2dError):
            C.conv2d_run(plan, inp.data_ptr(), f.data_ptr(), inp.data_ptr(), st)  # aliasing
        torch.cuda.synchronize()
    finally:
        C.conv2d_destroy(plan)
    with pytest.raises(C.Conv2dError):
        C.conv2d_plan(C.shape(0, 5, 3, 3), None)
    with pytest.raises(C.Conv2dError):
        C.conv2d_plan(C.shape(8, 8, 64, 3), None)
