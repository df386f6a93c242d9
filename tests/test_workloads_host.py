"""Host-side helpers of the workloads module: the hotspot roofline and the
candidate lists of the in-context batch tuning, on the stored sweeps."""
import json
import os

import pytest

C = pytest.importorskip("paper_2407_11488_amd")
from paper_2407_11488_amd import workloads  # noqa: E402


def test_hotspot_roofline():
    """60 steps in 8 launches: 7.5 x 14 / 12 = 8.75 FLOP/B, roof min(78.6,
    8.75 x 8 TB/s = 70) TFLOP/s; one step per launch: 1.1667 FLOP/B, HBM
    roof 9.33; 60 steps in one launch: ALU roof 78.6."""
    r = workloads.hotspot_roofline(35000.0, 60, 8)
    assert r["flop_per_byte"] == 8.75 and r["roof_tflops"] == 70.0 and r["frac"] == 0.5
    r = workloads.hotspot_roofline(4000.0, 60, 60)
    assert r["flop_per_byte"] == pytest.approx(14 / 12, abs=1e-3) and r["roof_tflops"] == pytest.approx(9.33, abs=0.01)
    assert workloads.hotspot_roofline(1000.0, 60, 1)["roof_tflops"] == 78.6


@pytest.mark.parametrize("f", [3, 5, 9, 17])
def test_batch_context_candidates_from_the_stored_sweep(f):
    """The k fastest verified points of the filter's stored 4096 x 4096
    sweep for the current kernel, filter through its pointer, distinct,
    in time order (checked against the results file read here directly)."""
    k = 6
    got = workloads.batch_context_candidates(f, f, k)
    path = os.path.join(os.path.dirname(C.LIB_PATH), "tuned", f"results_gfx950_4096x4096_{f}x{f}.jsonl")
    src = C.conv2d_kernel_hash()
    best = {}
    with open(path) as fh:
        for line in fh:
            try:
                r = json.loads(line)
            except json.JSONDecodeError:
                continue
            if r.get("src") == src and r.get("status") == "ok" and tuple(r["shape"]) == (4096, 4096, f, f):
                best[tuple(r["config"])] = r["ms"]          # the last record of a configuration wins
    want = []
    for c, _ in sorted(best.items(), key=lambda kv: (kv[1], kv[0])):
        c = c[:5] + (0,) + c[6:]
        if c not in want:
            want.append(c)
    assert got == want[:k]
    assert len(got) == k and all(c[5] == 0 for c in got)
