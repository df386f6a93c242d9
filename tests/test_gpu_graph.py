"""The plain path under stream capture and under concurrent use.

conv2d_run recorded into a graph (torch.cuda.graph) and replayed several
times, with eager work and synchronisation between the replays: every replay
equals the eager result bit for bit, for a constant-memory filter (a
device-to-device copy node before the kernel) and a global-pointer filter.
One plan shared by several host threads, each on its own stream: every
output equals a single-threaded run."""
import numpy as np
import pytest

import datagen
from tests.gpu_util import say, to_dev, torch_cuda

pytestmark = pytest.mark.gpu
C = pytest.importorskip("paper_2407_11488_amd")


@pytest.mark.parametrize("cfg", [(16, 16, 1, 1, 1, 1, 1), (64, 2, 4, 4, 1, 0, 1)])
def test_plain_run_captured_and_replayed(cfg):
    torch = torch_cuda()
    H, W, fh, fw = 300, 260, 9, 9
    inp, f = datagen.conv_problem(H, W, fh, fw, seed_in=51, seed_f=52)
    di, df = to_dev(inp), to_dev(f)
    plan = C.Plan(H, W, fh, fw, config=cfg)
    eager = plan(di, df)
    torch.cuda.synchronize()
    want = eager.cpu().numpy().copy()
    out = torch.full((H, W), float("nan"), device="cuda")
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        C.conv2d_run(plan.handle, di.data_ptr(), df.data_ptr(), out.data_ptr(),
                     torch.cuda.current_stream().cuda_stream)
    for rep in range(4):
        say(f"graph replay {rep} cfg {cfg}")
        out.fill_(float("nan"))                       # eager work between replays
        junk = torch.randn(1 << 18, device="cuda").sum()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint32), want.view(np.uint32)), rep
        del junk
    # a new filter written into the same buffer is picked up by the next replay
    f2 = datagen.uniform_pm1(77, fh * fw).reshape(fh, fw)
    df.copy_(torch.from_numpy(f2).cuda())
    g.replay()
    want2 = plan(di, df)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint32), want2.cpu().numpy().view(np.uint32))
    del g
    plan.close()


def test_plan_shared_by_threads_on_their_own_streams():
    """One plan (filter through its pointer) used by four host threads at
    once, each on its own stream with its own buffers, twenty runs each, the
    first call of each thread with pointers one float past a 16-byte
    boundary: every output equals a single-threaded run bit for bit."""
    import threading
    torch = torch_cuda()
    H, W, fh, fw = 200, 132, 7, 7   # input rows of 138 floats: 4-wide loads cross 16-byte boundaries
    plan = C.Plan(H, W, fh, fw, config=(32, 4, 4, 2, 0, 0, 1))
    data = [datagen.conv_problem(H, W, fh, fw, seed_in=80 + k, seed_f=90 + k) for k in range(4)]
    want = []
    for inp, f in data:
        o = plan(to_dev(inp), to_dev(f))
        torch.cuda.synchronize()
        want.append(o.cpu().numpy().copy())
    errors = []

    def worker(k):
        try:
            s = torch.cuda.Stream()
            inp, f = data[k]
            di, df = to_dev(inp), to_dev(f)
            big_in = torch.zeros(di.numel() + 1, device="cuda")
            big_in[1:] = di.reshape(-1)
            big_out = torch.full((H * W + 1,), float("nan"), device="cuda")
            torch.cuda.synchronize()
            # first call one float past a 16-byte boundary, then aligned calls
            C.conv2d_run(plan.handle, big_in.data_ptr() + 4, df.data_ptr(), big_out.data_ptr() + 4, s.cuda_stream)
            s.synchronize()
            if not np.array_equal(big_out[1:].cpu().numpy().view(np.uint32), want[k].reshape(-1).view(np.uint32)):
                errors.append((k, "offset by one float"))
            out = torch.full((H, W), float("nan"), device="cuda")
            torch.cuda.synchronize()                   # the fill runs on the default stream
            for _ in range(20):
                C.conv2d_run(plan.handle, di.data_ptr(), df.data_ptr(), out.data_ptr(), s.cuda_stream)
            s.synchronize()
            if not np.array_equal(out.cpu().numpy().view(np.uint32), want[k].view(np.uint32)):
                errors.append((k, "aligned"))
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append((k, repr(e)))

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors
    plan.close()


def test_conv2d_helper_constant_filter_on_two_streams():
    """conv2d() with a configuration whose filter goes to constant memory,
    called on two streams with different filters and no synchronisation
    between the calls: each stream gets a plan (and a constant array) of its
    own, so each output equals a single-stream run bit for bit."""
    torch = torch_cuda()
    H, W, fh, fw = 256, 320, 9, 9
    cfg = (16, 16, 1, 1, 1, 1, 1)                 # the default: LDS, filter in constant memory
    data = [datagen.conv_problem(H, W, fh, fw, seed_in=110 + k, seed_f=120 + k) for k in range(2)]
    dev = [(to_dev(inp), to_dev(f)) for inp, f in data]
    want = []
    for di, df in dev:
        want.append(C.conv2d(di, df, config=cfg).cpu().numpy().copy())
        torch.cuda.synchronize()
    assert not np.array_equal(want[0], want[1])
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [torch.full((H, W), float("nan"), device="cuda") for _ in range(2)]
    torch.cuda.synchronize()
    say("conv2d() constant-filter plan on two streams")
    for _ in range(20):
        for k in range(2):
            C.conv2d(dev[k][0], dev[k][1], config=cfg, out=outs[k], stream=streams[k])
    torch.cuda.synchronize()
    for k in range(2):
        assert np.array_equal(outs[k].cpu().numpy().view(np.uint32), want[k].view(np.uint32)), k


def test_close_waits_for_queued_work_and_keeps_a_captured_plan():
    """A plan dropped right after an asynchronous call (a temporary object)
    frees its code only after the device has finished the queued work: the
    output still equals a kept plan's, bit for bit. close() inside a capture
    keeps the handle, the graph replays, and a later close() frees it."""
    import gc
    torch = torch_cuda()
    H, W, fh, fw = 700, 640, 17, 17
    inp, f = datagen.conv_problem(H, W, fh, fw, seed_in=61, seed_f=62)
    di, df = to_dev(inp), to_dev(f)
    keep = C.Plan(H, W, fh, fw)
    want = keep(di, df)
    torch.cuda.synchronize()
    want = want.cpu().numpy().copy()
    say("temporary plans closed with queued work")
    outs = []
    for _ in range(4):
        junk = torch.randn(1 << 22, device="cuda")              # queued work ahead of the launch
        outs.append(C.Plan(H, W, fh, fw, config=(64, 2, 4, 4, 1, 0, 1))(di, df))
        gc.collect()
        del junk
    torch.cuda.synchronize()
    for o in outs:
        assert np.array_equal(o.cpu().numpy().view(np.uint32), want.view(np.uint32))

    say("close inside a capture")
    plan = C.Plan(H, W, fh, fw, config=(16, 16, 1, 1, 1, 1, 1))
    out = torch.full((H, W), float("nan"), device="cuda")
    plan(di, df, out=out)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan(di, df, out=out)
        plan.close()
        assert plan.handle                                     # kept while capturing
    for rep in range(3):
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint32), want.view(np.uint32)), rep
    del g
    plan.close()
    assert not plan.handle
    keep.close()
