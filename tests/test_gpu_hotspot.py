"""GPU parity of the hotspot stencil (hotspot_plan / hotspot_run /
hotspot_reference) through the C ABI: the one-step reference against the FP64
oracle, a stratified sample of the tuning space bitwise against the reference,
the 4096 x 4096 chip workload against the oracle, edge cases and errors."""
import concurrent.futures as cf

import numpy as np
import pytest

import datagen
import oracle
from tests.gpu_util import hip_free, hip_malloc, say, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

C = pytest.importorskip("paper_2407_11488_amd")

STRESS = (0.2, 0.5, 0.75, 0.05, 0.25)   # every term of the step matters at this scale


def bound(temp, power, steps, k):
    """FP32 error bound of `steps` explicit steps (each step's rounding is at
    most a few units in the last place of the largest term it touches, and a
    stable step does not amplify earlier errors): 8 n u (max|T| + |t_amb| +
    n cc max|P|)."""
    cc, _, _, _, t_amb = k
    m = float(np.max(np.abs(temp))) + abs(t_amb) + steps * cc * float(np.max(np.abs(power)))
    return 8.0 * max(steps, 1) * 2.0 ** -24 * m


def stored_winners():
    """The configurations of the hotspot winners cache shipped with the
    library (one per tuned grid)."""
    import json
    import os
    path = os.path.join(os.path.dirname(C.LIB_PATH), "tuned", "hotspot_winners.jsonl")
    with open(path) as fh:
        cfgs = {tuple(json.loads(line)["config"]) for line in fh if line.strip()}
    assert cfgs
    return sorted(cfgs)


def _run_plan(cfg, temp_d, power_d, steps, k, rows, cols):
    torch = torch_cuda()
    plan = C.Hotspot(rows, cols, cfg)
    try:
        out = torch.full((rows, cols), float("nan"), device="cuda")
        plan(temp_d, power_d, steps, k, out=out)
        torch.cuda.synchronize()
        return out.cpu().numpy()
    finally:
        plan.close()


@pytest.mark.parametrize("rows,cols,steps", [(1, 1, 3), (1, 17, 4), (33, 1, 5), (64, 64, 1), (100, 77, 13),
                                             (5, 300, 0)])
def test_reference_matches_oracle(rows, cols, steps):
    torch = torch_cuda()
    temp = datagen.uniform_pm1(61, rows * cols).reshape(rows, cols)
    power = datagen.uniform_pm1(62, rows * cols).reshape(rows, cols)
    out = C.reference_hotspot(to_dev(temp), to_dev(power), steps, STRESS)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = oracle.hotspot_f64(temp, power, steps, *STRESS)
    assert np.max(np.abs(got - ref)) <= bound(temp, power, steps, STRESS)


def test_stratified_configs_bitwise():
    """About 130 points of the space (every 16th in enumeration order, plus the
    default, the stored winners of every tuned grid and the extremes of each
    axis) on a ragged 181 x 97 grid, 13 steps (partial last launches for most
    temporal factors): every point equals the reference bit for bit. The
    stress coefficients make every term of the step larger than the error
    bound, so a point that dropped one would fail."""
    torch = torch_cuda()
    rows, cols, steps = 181, 97, 13
    space = C.hotspot_space(C.hotspot_shape(rows, cols))
    pick = space[::16] + [C.hotspot_default_config().tuple()] + stored_winners()
    for ax in range(7):
        vals = sorted({c[ax] for c in space})
        for v in (vals[0], vals[-1]):
            pick.append(next(c for c in space if c[ax] == v))
    pick = sorted(set(pick))
    with cf.ThreadPoolExecutor(16) as ex:
        list(ex.map(C.hotspot_compile, pick))
    temp = datagen.uniform_pm1(63, rows * cols).reshape(rows, cols)
    power = datagen.uniform_pm1(64, rows * cols).reshape(rows, cols)
    td, pd = to_dev(temp), to_dev(power)
    ref = C.reference_hotspot(td, pd, steps, STRESS)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    assert np.max(np.abs(ref - oracle.hotspot_f64(temp, power, steps, *STRESS))) <= bound(temp, power, steps, STRESS)
    say(f"hotspot: {len(pick)} configurations")
    for cfg in pick:
        got = _run_plan(cfg, td, pd, steps, STRESS, rows, cols)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), cfg


def test_chip_workload_full_size():
    """4096 x 4096 chip workload, 60 steps, in the configuration the plan picks
    (the tuned winner when cached, the one the benchmark times): bit for bit
    equal to the one-step reference kernel, and every cell within the bound
    of the FP64 oracle."""
    torch = torch_cuda()
    rows = cols = 4096
    steps = 60
    temp, power, k = datagen.hotspot_problem(rows, cols)
    plan = C.Hotspot(rows, cols)
    say(f"hotspot 4096 with {plan.source} config {plan.config}")
    td, pd = to_dev(temp), to_dev(power)
    out = plan(td, pd, steps, k)
    ref_dev = C.reference_hotspot(td, pd, steps, k)
    torch.cuda.synchronize()
    plan.close()
    mism = int((out.view(torch.int32) != ref_dev.view(torch.int32)).sum().item())
    assert mism == 0, f"{mism} cells differ from the reference kernel"
    got = out.cpu().numpy()
    ref = oracle.hotspot_f64(temp, power, steps, *k)
    err = float(np.max(np.abs(got - ref)))
    say(f"hotspot 4096 max error {err:.3e} K (bound {bound(temp, power, steps, k):.3e})")
    assert err <= bound(temp, power, steps, k)


def test_full_size_every_term_visible():
    """4096 x 4096, 60 steps, in the plan's (tuned) configuration, with the
    stress coefficients on uniform [-1, 1) temperatures and powers: dropping
    the power term or the vertical sink from the oracle moves its result by
    far more than the FP32 bound, so a kernel that lost either term fails;
    the plan's result is within the bound of the oracle."""
    torch = torch_cuda()
    rows = cols = 4096
    steps = 60
    temp = datagen.uniform_pm1(91, rows * cols).reshape(rows, cols)
    power = datagen.uniform_pm1(92, rows * cols).reshape(rows, cols)
    plan = C.Hotspot(rows, cols)
    say(f"hotspot 4096 stress coefficients with {plan.source} config {plan.config}")
    out = plan(to_dev(temp), to_dev(power), steps, STRESS)
    torch.cuda.synchronize()
    plan.close()
    got = out.cpu().numpy()
    b = bound(temp, power, steps, STRESS)
    ref = oracle.hotspot_f64(temp, power, steps, *STRESS)
    no_power = oracle.hotspot_f64(temp, power * 0, steps, *STRESS)
    cc, gx, gy, _, t_amb = STRESS
    no_sink = oracle.hotspot_f64(temp, power, steps, cc, gx, gy, 0.0, t_amb)
    assert np.max(np.abs(ref - no_power)) > 100 * b
    assert np.max(np.abs(ref - no_sink)) > 100 * b
    err = float(np.max(np.abs(got - ref)))
    say(f"hotspot 4096 stress max error {err:.3e} (bound {b:.3e})")
    assert err <= b


def test_edge_cases():
    """Zero steps copy the grid; a grid smaller than one output tile; the same
    plan reused on new data; a temporal factor above the step count."""
    torch = torch_cuda()
    for rows, cols, steps, cfg in [(7, 5, 0, None), (3, 2, 9, (16, 4, 4, 4, 6, 0, 1)), (2, 1, 2, (64, 2, 1, 4, 3, 1, 0))]:
        temp = datagen.uniform_pm1(65, rows * cols).reshape(rows, cols)
        power = datagen.uniform_pm1(66, rows * cols).reshape(rows, cols)
        got = _run_plan(cfg, to_dev(temp), to_dev(power), steps, STRESS, rows, cols)
        ref = oracle.hotspot_f64(temp, power, steps, *STRESS)
        assert np.max(np.abs(got - ref)) <= bound(temp, power, steps, STRESS), (rows, cols, steps, cfg)
    plan = C.Hotspot(40, 40, (32, 8, 2, 1, 2, 1, 1))
    for seed in (67, 68):
        temp = datagen.uniform_pm1(seed, 1600).reshape(40, 40)
        got = plan(to_dev(temp), to_dev(temp * 0), 5, STRESS)
        torch.cuda.synchronize()
        ref = oracle.hotspot_f64(temp, temp * 0, 5, *STRESS)
        assert np.max(np.abs(got.cpu().numpy() - ref)) <= bound(temp, temp * 0, 5, STRESS)
    plan.close()


def test_ungridded_plan_takes_another_grids_winner(tmp_path, monkeypatch):
    """A grid with no winners entry of its own takes the 4096 x 4096 winner
    (source "tuned-other-grid"); with no entry at all it takes the default;
    either way the result stays within the FP32 bound of the oracle."""
    import json
    torch = torch_cuda()
    cfg = (64, 4, 2, 4, 4, 1, 1)
    full = tmp_path / "hs_winners.jsonl"
    full.write_text(json.dumps({"arch": "gfx950", "src": "0000000000000000", "shape": [4096, 4096],
                                "config": list(cfg), "ms": 1.0}) + "\n")
    empty = tmp_path / "none.jsonl"
    empty.write_text("")
    rows, cols = 300, 200
    temp, power, k = datagen.hotspot_problem(rows, cols)
    ref = oracle.hotspot_f64(temp, power, 9, *k)
    for path, want in ((full, ("tuned-other-grid", cfg)), (empty, ("default", C.hotspot_default_config().tuple()))):
        monkeypatch.setenv("HOTSPOT_WINNERS", str(path))
        hs = C.Hotspot(rows, cols)
        say(f"hotspot {rows}x{cols} with {path.name}: {hs.source} {hs.config}")
        assert (hs.source, tuple(hs.config)) == want
        out = hs(torch.from_numpy(temp).cuda(), torch.from_numpy(power).cuda(), 9, k)
        torch.cuda.synchronize()
        assert np.max(np.abs(out.cpu().numpy().astype(np.float64) - ref)) <= bound(temp, power, 9, k)
        hs.close()


def test_errors_are_reported_not_faulted():
    torch = torch_cuda()
    s = C.hotspot_shape(64, 64)
    h = C.hotspot_plan(s, (32, 8, 1, 1, 2, 1, 1))
    k = C.hotspot_coeffs(*STRESS)
    st = torch.cuda.current_stream().cuda_stream
    try:
        a = torch.zeros((64, 64), device="cuda")
        b = torch.zeros((64, 64), device="cuda")
        o = torch.zeros((64, 64), device="cuda")
        small = hip_malloc(400)                   # a real 400-byte allocation
        with pytest.raises(C.Conv2dError):        # two launches, no work buffer
            C.hotspot_run(h, a.data_ptr(), b.data_ptr(), o.data_ptr(), 0, 3, k, st)
        with pytest.raises(C.Conv2dError):        # output overlaps the input
            C.hotspot_run(h, a.data_ptr(), b.data_ptr(), a.data_ptr(), 0, 1, k, st)
        with pytest.raises(C.Conv2dError):        # buffer too small for the grid
            C.hotspot_run(h, small, b.data_ptr(), o.data_ptr(), 0, 1, k, st)
        with pytest.raises(C.Conv2dError):
            C.hotspot_run(h, a.data_ptr(), b.data_ptr(), o.data_ptr(), 0, -1, k, st)
        with pytest.raises(C.Conv2dError):        # work buffer is the output
            C.hotspot_run(h, a.data_ptr(), b.data_ptr(), o.data_ptr(), o.data_ptr(), 3, k, st)
        C.hotspot_run(h, a.data_ptr(), b.data_ptr(), o.data_ptr(), 0, 2, k, st)   # one launch: no work buffer
        torch.cuda.synchronize()
        hip_free(small)
    finally:
        C.hotspot_destroy(h)
    with pytest.raises(C.Conv2dError):
        C.hotspot_plan(s, (16, 1, 1, 1, 1, 1, 1))    # 16 threads: below the minimum
    with pytest.raises(C.Conv2dError):
        C.hotspot_plan(C.hotspot_shape(0, 5))


def test_reference_helpers_check_shapes_on_the_host():
    """The reference helpers reject a power grid or output of another shape
    before any launch (each wrong buffer here is larger than the right one)."""
    torch = torch_cuda()
    say("reference helpers: shape checks")
    temp = torch.zeros((64, 48), device="cuda")
    with pytest.raises(ValueError, match="power"):
        C.reference_hotspot(temp, torch.zeros((65, 48), device="cuda"), 2, STRESS)
    with pytest.raises(ValueError, match="out"):
        C.reference_hotspot(temp, torch.zeros((64, 48), device="cuda"), 2, STRESS,
                            out=torch.zeros((64, 49), device="cuda"))
    with pytest.raises(ValueError, match="2-D"):
        C.reference_hotspot(torch.zeros((4, 64, 48), device="cuda"), temp, 2, STRESS)
    inp = torch.zeros((40, 40), device="cuda")
    f = torch.zeros((5, 5), device="cuda")
    with pytest.raises(ValueError, match="out"):
        C.reference(inp, f, out=torch.zeros((37, 36), device="cuda"))
    with pytest.raises(ValueError, match="float32"):
        C.reference(inp, f.double())
    torch.cuda.synchronize()


def test_grid_too_wide_for_region_offsets():
    """A grid so wide (9 x (2^27 + 1000) cells, 4.8 GB per array) that the
    rows of a region span 2^31 bytes or more: every region, interior ones
    included, takes the clamped 64-bit path. Three steps in two
    configurations (one step and two steps per launch); windows at the left
    edge, in the middle and at the right edge are compared with the FP64
    oracle run on each window widened by steps + 1 columns, so that the
    window's own borders, where the oracle would apply the grid-edge rule,
    do not reach the compared cells."""
    torch = torch_cuda()
    rows, cols, steps = 9, (1 << 27) + 1000, 3
    n = rows * cols
    st = torch.cuda.current_stream().cuda_stream
    temp = torch.empty((rows, cols), dtype=torch.float32, device="cuda")
    power = torch.empty((rows, cols), dtype=torch.float32, device="cuda")
    C.conv2d_fill_uniform(temp.data_ptr(), n, 71, 0, st)
    C.conv2d_fill_uniform(power.data_ptr(), n, 72, 0, st)
    m, w = steps + 1, 300
    for cfg in [(16, 4, 1, 1, 1, 1, 1), (16, 4, 1, 2, 2, 0, 1)]:
        plan = C.Hotspot(rows, cols, cfg)
        say(f"hotspot {rows}x{cols} config {cfg}")
        out = plan(temp, power, steps, STRESS)
        torch.cuda.synchronize()
        for c0 in (0, cols // 2 - w // 2, cols - w):
            lo, hi = max(0, c0 - m), min(cols, c0 + w + m)
            t = temp[:, lo:hi].cpu().numpy()
            p = power[:, lo:hi].cpu().numpy()
            ref = oracle.hotspot_f64(t, p, steps, *STRESS)[:, c0 - lo:c0 - lo + w]
            got = out[:, c0:c0 + w].cpu().numpy()
            assert np.all(np.isfinite(got)), (cfg, c0)
            err = float(np.max(np.abs(got - ref)))
            assert err <= bound(t, p, steps, STRESS), (cfg, c0, err)
        del out
        plan.close()
        del plan                                    # and its 4.8 GB work grid
    del temp, power
    import gc
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()                        # the next tests measure free device memory
