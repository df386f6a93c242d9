"""The plain path under stream capture: conv2d_run recorded into a graph
(torch.cuda.graph) and replayed several times, with eager work and
synchronisation between the replays; every replay must equal the eager
result bit for bit, for a constant-memory filter (a device-to-device copy
node before the kernel) and a global-pointer filter."""
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
