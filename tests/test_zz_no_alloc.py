"""GPU test of hotspot_run_noalloc, the hotspot entry point that allocates
nothing (its work grid is a fixed array of the library's device code),
through the C ABI: two calls in a row, the second on a smaller grid, each
bit for bit equal to hotspot_run with a caller-given work buffer; a grid
above the fixed array's size is refused when it needs the work grid."""
import numpy as np
import pytest

import datagen
from tests.gpu_util import say, torch_cuda

pytestmark = pytest.mark.gpu

C = pytest.importorskip("paper_2407_11488_amd")
B = pytest.importorskip("paper_2407_11488_amd._binding")

STRESS = (0.2, 0.5, 0.75, 0.05, 0.25)


def _one(rows, cols, steps, cfg, seed):
    torch = torch_cuda()
    st = torch.cuda.current_stream().cuda_stream
    temp = torch.from_numpy(datagen.uniform_pm1(seed, rows * cols).reshape(rows, cols)).cuda()
    power = torch.from_numpy(datagen.uniform_pm1(seed + 1, rows * cols).reshape(rows, cols)).cuda()
    want = torch.full((rows, cols), float("nan"), device="cuda")
    work = torch.empty((rows, cols), device="cuda")
    got = torch.full((rows, cols), float("nan"), device="cuda")
    k = B.hotspot_coeffs(*STRESS)
    plan = B.hotspot_plan(B.hotspot_shape(rows, cols), cfg)
    try:
        say(f"noalloc: {rows}x{cols} steps {steps} config {cfg}")
        B.hotspot_run(plan, temp.data_ptr(), power.data_ptr(), want.data_ptr(), work.data_ptr(), steps, k, st)
        B.hotspot_run_noalloc(plan, temp.data_ptr(), power.data_ptr(), got.data_ptr(), steps, k, st)
        torch.cuda.synchronize()
    finally:
        B.hotspot_destroy(plan)
    g, w = got.cpu().numpy(), want.cpu().numpy()
    assert np.all(np.isfinite(g))
    assert np.array_equal(g.view(np.uint32), w.view(np.uint32))


def test_noalloc_matches_hotspot_run_twice_second_smaller():
    # 4096 x 4096 fills the fixed work grid exactly; 60 steps at temporal 6
    # are ten launches that alternate between the output and the work grid.
    _one(4096, 4096, 60, (64, 16, 2, 4, 6, 1, 1), 131)
    # a smaller, ragged grid right after: its launches reuse the same work
    # grid, whose old contents must not leak into the result
    _one(1000, 777, 13, (32, 8, 2, 2, 3, 0, 1), 141)
    _one(1, 1, 5, (64, 4, 1, 1, 1, 1, 1), 151)


def test_noalloc_refuses_a_grid_above_the_fixed_work_grid():
    torch = torch_cuda()
    rows, cols = 4097, 4096
    assert rows * cols > B.HOTSPOT_NOALLOC_CELLS
    t = torch.zeros((rows, cols), device="cuda")
    p = torch.zeros((rows, cols), device="cuda")
    o = torch.zeros((rows, cols), device="cuda")
    plan = B.hotspot_plan(B.hotspot_shape(rows, cols), (32, 8, 1, 1, 2, 1, 1))
    st = torch.cuda.current_stream().cuda_stream
    try:
        with pytest.raises(C.Conv2dError) as e:         # 3 launches: needs the work grid
            B.hotspot_run_noalloc(plan, t.data_ptr(), p.data_ptr(), o.data_ptr(), 5, B.hotspot_coeffs(*STRESS), st)
        assert e.value.status == C.CONV2D_EINVAL
        # one launch needs no work grid: accepted
        B.hotspot_run_noalloc(plan, t.data_ptr(), p.data_ptr(), o.data_ptr(), 2, B.hotspot_coeffs(*STRESS), st)
        torch.cuda.synchronize()
    finally:
        B.hotspot_destroy(plan)
