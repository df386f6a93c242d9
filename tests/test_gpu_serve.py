"""GPU tests of the serving loop (conv2d_serve) through the C ABI: each result
the same alone and in the mix, HBM-budget admission, the serial baseline, and
argument errors."""
import ctypes

import numpy as np
import pytest

import datagen
import oracle
from tests.gpu_util import TOL, say, torch_cuda

pytestmark = pytest.mark.gpu

C = pytest.importorskip("paper_2407_11488_amd")


def small_trace(n=48, rate=20000.0, seed=11, lo=32, hi=384, burst=0):
    """n requests, Poisson arrivals; the first `burst` arrive together at t = 0
    (they are admitted together and so share a batch)."""
    t = datagen.poisson_arrivals(rate, n / rate * 3, seed=seed)[:n]
    t[:burst] = 0.0
    sides = datagen.log_uniform_sides(seed + 1, len(t), lo, hi)
    fs = datagen.filter_choices(seed + 1, len(t))
    shapes = [(int(s), int(s) + (k % 3), int(f), int(f)) for k, (s, f) in enumerate(zip(sides, fs))]
    seeds_in = [5000 + k for k in range(len(t))]
    seeds_f = [6000 + k for k in range(len(t))]
    return C.requests_array(t, shapes, seeds_in, seeds_f), shapes


def _hip_runtime():
    """The HIP runtime this process already uses (the one torch loaded)."""
    with open("/proc/self/maps") as fh:
        paths = sorted({ln.split()[-1] for ln in fh if "libamdhip64" in ln})
    assert len(paths) == 1, paths
    hip = ctypes.CDLL(paths[0])
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return hip


def _copy_out(ptr, H, W):
    torch = torch_cuda()
    out = torch.empty((H, W), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    hip = _hip_runtime()
    assert hip.hipMemcpy(out.data_ptr(), ptr, H * W * 4, 3) == 0  # device to device
    return out


def _plain(shape, seed_in, seed_f):
    """The same request alone: device-generated data, one plain conv2d_run."""
    torch = torch_cuda()
    H, W, fh, fw = shape
    inp = torch.empty((H + fh - 1, W + fw - 1), dtype=torch.float32, device="cuda")
    f = torch.empty((fh, fw), dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    C.conv2d_fill_uniform(inp.data_ptr(), inp.numel(), seed_in, 0, st)
    C.conv2d_fill_uniform(f.data_ptr(), f.numel(), seed_f, 0, st)
    out = C.conv2d(inp, f)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("serial", [0, 1])
def test_results_same_alone_and_in_the_mix(serial):
    reqs, shapes = small_trace(burst=12)
    o = C.conv2d_serve_defaults()
    o.serial_plain = serial
    o.streams = 3
    o.max_batch = 16
    say(f"serve {len(reqs)} requests serial={serial}")
    rep, lat, outs = C.conv2d_serve(reqs, o, keep_outputs=True)
    try:
        assert rep.n_requests == len(reqs) and np.all(lat > 0)
        if not serial:
            assert rep.n_batches < len(reqs), "no request was batched with another"
        for k, (H, W, fh, fw) in enumerate(shapes):
            got = _copy_out(outs[k], H, W).cpu().numpy()
            alone = _plain(shapes[k], int(reqs["seed_in"][k]), int(reqs["seed_f"][k])).cpu().numpy()
            assert np.array_equal(got.view(np.uint32), alone.view(np.uint32)), k
            if k % 8 == 0:
                inp, f = datagen.conv_problem(H, W, fh, fw, seed_in=int(reqs["seed_in"][k]),
                                              seed_f=int(reqs["seed_f"][k]))
                ref, s = oracle.conv2d_f64(inp, f)
                assert oracle.normalized_error(got, ref, s) <= TOL
    finally:
        C.conv2d_serve_free(outs)


def test_mixed_size_buckets_same_alone_and_in_the_mix():
    """Requests spanning every size bucket (sides 200 to 3,500, all four
    filter sizes), most arriving together: the server gives each its bucket's
    configuration and launches one kernel per filter size and configuration
    of a batch; every output equals the plain path's on the same data, bit
    for bit (the plain path is pinned against the oracle elsewhere)."""
    sides = [200, 450, 900, 1700, 3500, 300, 700, 1200, 2500, 3100, 380, 1000]
    fs = [3, 5, 9, 17, 3, 17, 9, 5, 3, 9, 17, 5]
    shapes = [(s, s + (k % 3), f, f) for k, (s, f) in enumerate(zip(sides, fs))]
    assert {C.conv2d_size_bucket(h, w) for (h, w, _, _) in shapes} == {1, 2, 3, 4, 5}
    t = np.zeros(len(shapes))
    t[8:] = [1e-4, 2e-4, 3e-4, 4e-4]
    reqs = C.requests_array(t, shapes, [7000 + k for k in range(len(shapes))],
                            [8000 + k for k in range(len(shapes))])
    o = C.conv2d_serve_defaults()
    o.streams, o.max_batch = 2, 8
    rep, lat, outs = C.conv2d_serve(reqs, o, keep_outputs=True)
    try:
        say(f"mixed buckets: {rep.as_dict()}")
        assert rep.n_requests == len(shapes) and rep.n_batches < len(shapes)
        for k, (H, W, fh, fw) in enumerate(shapes):
            got = _copy_out(outs[k], H, W).cpu().numpy()
            alone = _plain(shapes[k], 7000 + k, 8000 + k).cpu().numpy()
            assert np.array_equal(got.view(np.uint32), alone.view(np.uint32)), k
    finally:
        C.conv2d_serve_free(outs)


def test_budget_admission_bounds_memory():
    reqs, shapes = small_trace(n=40, rate=1e6, seed=21, lo=200, hi=400)
    need = [4 * ((H + fh - 1) * (W + fw - 1) + fh * fw + H * W) + 3 * 256 for (H, W, fh, fw) in shapes]
    o = C.conv2d_serve_defaults()
    o.hbm_budget = int(max(need) * 1.5)
    o.streams = 2
    rep, lat, _ = C.conv2d_serve(reqs, o)
    say(f"tight budget: {rep.as_dict()}")
    assert rep.n_requests == len(reqs)
    assert rep.peak_bytes <= o.hbm_budget
    assert rep.stalled_requests > 0


def test_serve_argument_errors():
    reqs, _ = small_trace(n=4)
    o = C.conv2d_serve_defaults()
    o.hbm_budget = 1 << 20
    big = C.requests_array([0.0], [(1024, 1024, 17, 17)], [1], [2])
    with pytest.raises(C.Conv2dError):
        C.conv2d_serve(big, o)                       # alone above the budget
    bad = reqs.copy()
    bad["arrival_s"] = bad["arrival_s"][::-1]
    if len(bad) > 1 and bad["arrival_s"][0] != bad["arrival_s"][-1]:
        with pytest.raises(C.Conv2dError):
            C.conv2d_serve(bad)                      # arrivals out of order
    o = C.conv2d_serve_defaults()
    o.streams = 0
    with pytest.raises(C.Conv2dError):
        C.conv2d_serve(reqs, o)


def test_kept_output_allocation_failure_is_reported():
    """With keep_outputs, a request whose own output allocation fails (the
    device is full: a blocker tensor leaves less free memory than the output
    needs) makes conv2d_serve return CONV2D_ENOMEM instead of waiting for
    memory that retiring requests cannot free; the outputs it had allocated
    are released (the free memory afterwards is what it was before)."""
    import gc
    torch = torch_cuda()
    gc.collect()                     # tensors of earlier tests still waiting for collection
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0, _ = torch.cuda.mem_get_info()
    H = W = 16384                                   # 1 GiB output, 1.07 GB input
    first = (256, 256, 3, 3)
    reqs = C.requests_array([0.0, 0.0], [first, (H, W, 3, 3)], [1, 2], [3, 4])
    o = C.conv2d_serve_defaults()
    o.hbm_budget = 4 * (H + 2) * (W + 2) + (64 << 20)
    o.streams = 1
    leave = o.hbm_budget + (512 << 20)               # the arena fits, a 1 GiB output does not
    blocker = torch.empty(max(free0 - leave, 0) // 4, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    say(f"kept-output allocation failure: blocker {blocker.numel() * 4 / 2**30:.1f} GiB")
    try:
        with pytest.raises(C.Conv2dError) as e:
            C.conv2d_serve(reqs, o, keep_outputs=True)
        assert e.value.status == C.CONV2D_ENOMEM
        assert "output allocation" in str(e.value)
    finally:
        del blocker
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 >= free0 - (64 << 20), (free0, free1)
