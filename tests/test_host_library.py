"""Host-side behaviour of the C library (no GPU): exported symbols, the search
space and its restrictions, code-object properties of compiled
configurations, the tile mapping, and the tuner's selection and statistics
against the plain-Python oracle (with a synthetic cost in place of the GPU)."""
import json
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2407_11488_amd as C
from oracle import space as ospace
from oracle import tuning as otune

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "conv2d.h")
OBJDUMP = "/opt/rocm/llvm/bin/llvm-objdump"
READELF = "/opt/rocm/llvm/bin/llvm-readelf"


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(conv2d_[a-z0-9_]+)\s*\(", text)
    return sorted(set(n for n in names if not n.endswith("_fn")))


def test_library_exports_every_declared_function():
    names = header_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(C.lib, n)]
    assert not missing, missing


def test_space_matches_oracle_enumeration():
    s = C.shape(4096, 4096, 17, 17)
    got = C.conv2d_space(s, 1, -1)
    assert got == [c + (1,) for c in ospace.restricted()]
    legal = C.conv2d_space(s, 1, 0)
    assert len(legal) == 1202                       # 14 points need more than 160 KiB of LDS
    assert all(C.conv2d_lds_bytes(17, 17, c) <= 163840 for c in legal)
    assert len(C.conv2d_space(C.shape(4096, 4096, 31, 31), 1, 0)) == 1192


def test_config_check_errors():
    s = C.shape(64, 64, 3, 3)
    assert C.conv2d_config_check(s, (64, 1, 8, 8, 0, 0, 1)) == 0
    for bad in [(48, 1, 1, 1, 0, 0, 1), (64, 3, 1, 1, 0, 0, 1), (128, 16, 1, 1, 0, 0, 1), (64, 1, 3, 1, 0, 0, 1),
                (64, 1, 1, 1, 2, 0, 1), (64, 1, 1, 1, 0, 0, 3)]:
        assert C.conv2d_config_check(s, bad) == C.CONV2D_EINVAL, bad
        assert C.conv2d_last_error()
    assert C.conv2d_config_check(C.shape(0, 4, 3, 3), (64, 1, 1, 1, 0, 0, 1)) == C.CONV2D_EINVAL
    assert C.conv2d_config_check(C.shape(4, 4, 64, 3), (64, 1, 1, 1, 0, 0, 1)) == C.CONV2D_EINVAL


def _notes(path):
    out = subprocess.run([READELF, "--notes", path], capture_output=True, text=True).stdout
    get = lambda k: int(re.search(rf"\.{k}:\s+(\d+)", out).group(1))  # noqa: E731
    return {k: get(k) for k in ("group_segment_fixed_size", "private_segment_fixed_size", "vgpr_count",
                                "vgpr_spill_count")}


@pytest.mark.parametrize("cfg,vin", [((16, 16, 1, 1, 1, 1, 1), 4), ((64, 1, 8, 8, 1, 0, 1), 1),
                                     ((32, 4, 4, 2, 1, 1, 1), 2), ((128, 2, 2, 8, 1, 0, 1), 4)])
def test_lds_bytes_bound_the_compiled_kernel(cfg, vin):
    s = C.shape(512, 512, 17, 17)
    notes = _notes(C.conv2d_compile(s, cfg, vin, 4))
    assert 0 < notes["group_segment_fixed_size"] <= C.conv2d_lds_bytes(17, 17, cfg)


@pytest.mark.parametrize("cfg", [(16, 16, 4, 2, 1, 0, 1), (64, 1, 8, 8, 0, 0, 1), (128, 8, 8, 2, 0, 1, 1),
                                 (64, 1, 2, 4, 0, 1, 1)])
def test_compiled_code_is_plain_fp32_fma_without_spills(cfg):
    """No packed FP32 instruction anywhere; the row loop's body holds exactly
    tile_y*tile_x*17 single FMAs (rolled loop, unroll 1); no scratch."""
    s = C.shape(4096, 4096, 17, 17)
    path = C.conv2d_compile(s, cfg, 4, 4)
    isa = subprocess.run([OBJDUMP, "-d", path], capture_output=True, text=True).stdout
    assert "v_pk_" not in isa
    assert isa.count("v_fmac_f32") + isa.count("v_fma_f32") == cfg[2] * cfg[3] * 17
    n = _notes(path)
    assert n["private_segment_fixed_size"] == 0 and n["vgpr_spill_count"] == 0


def test_batched_kernel_is_built_four_wide(tmp_path):
    """The batched kernel is built with four-dword loads and stores (rows of
    every alignment in one launch), as the compile log of a fresh process
    records it."""
    log = tmp_path / "compiles.log"
    code = ("import paper_2407_11488_amd as C; "
            "C.conv2d_compile_batch(C.shape(4096, 4096, 5, 5), (64, 4, 4, 4, 0, 0, 1))")
    env = dict(os.environ, CONV2D_COMPILE_LOG=str(log))
    subprocess.run(["python3", "-c", code], check=True, env=env, cwd=os.path.dirname(os.path.dirname(__file__)),
                   timeout=300)
    lines = [ln for ln in log.read_text().splitlines() if ln.startswith("conv2d_direct.hip")]
    assert len(lines) == 1, lines
    assert "-DCONV_VIN=4 -DCONV_VOUT=4 -DCONV_BATCH=1" in lines[0], lines[0]


def test_batched_kernels_of_the_cached_choices_compile_without_spills():
    """The batched kernel of every configuration the batched path and the
    server take from the committed winners cache (whole-batch and size-bucket
    entries; filter through its pointer, rolled row loop as the library
    builds it when needed): no packed FP32, no scratch, no VGPR spills."""
    import json as _json
    wp = os.path.join(ROOT, "paper_2407_11488_amd", "tuned", "winners.jsonl")
    seen = set()
    for line in open(wp):
        r = _json.loads(line)
        sh, c = r["shape"], tuple(r["config"])
        if sh[0] != 0 or r.get("arch") != "gfx950":
            continue
        for unroll in sorted({c[6], 1}):
            cfg = c[:5] + (0, unroll)
            key = (sh[2], sh[3], cfg)
            if key in seen:
                continue
            seen.add(key)
            path = C.conv2d_compile_batch(C.shape(4096, 4096, sh[2], sh[3]), cfg)
            isa = subprocess.run([OBJDUMP, "-d", path], capture_output=True, text=True).stdout
            assert "v_pk_" not in isa, key
            n = _notes(path)
            if unroll == 1:
                assert n["private_segment_fixed_size"] == 0 and n["vgpr_spill_count"] == 0, key
    assert len(seen) >= 8


def xcd_remap(i, n):
    q, rem = n >> 3, n & 7
    x, k = i & 7, i >> 3
    return x * q + min(x, rem) + k


def test_xcd_remap_is_a_bijection():
    for n in list(range(1, 70)) + [4095, 4096, 8191, 65536 + 3]:
        t = [xcd_remap(i, n) for i in range(n)]
        assert sorted(t) == list(range(n)), n


@pytest.mark.parametrize("shape", [(70, 45, 5, 3), (1, 1, 1, 1), (4096, 4096, 17, 17), (203, 317, 31, 31)])
def test_tiles_cover_every_output_once(shape):
    """Model of the kernel's index mapping (workgroup -> tile via the XCD
    remap, thread -> tile_y x tile_x outputs): every output of the image is
    owned by exactly one thread, for a sample of configurations."""
    H, W, fh, fw = shape
    s = C.shape(*shape)
    rng = np.random.default_rng(1)
    cfgs = C.conv2d_space(s, 1, 0)
    for idx in rng.choice(len(cfgs), size=12, replace=False):
        c = cfgs[idx]
        bx, by, tx, ty = c[:4]
        tiles_x, tiles_y, nt = C.conv2d_geometry(s, c)
        assert nt == bx * by and tiles_x == -(-W // (bx * tx)) and tiles_y == -(-H // (by * ty))
        if H * W > 1 << 20:
            continue
        count = np.zeros((H + by * ty, W + bx * tx), np.int32)
        n_tiles = tiles_x * tiles_y
        for wg in range(n_tiles):
            t = xcd_remap(wg, n_tiles)
            ty_, tx_ = divmod(t, tiles_x)
            y0 = ty_ * by * ty
            x0 = tx_ * bx * tx
            count[y0:y0 + by * ty, x0:x0 + bx * tx] += 1
        assert np.all(count[:H, :W] == 1), c


# ---------------------------------------------------------------- tuner with a synthetic cost

def _cost_table(seed=3):
    rng = np.random.default_rng(seed)
    cfgs = C.conv2d_space(C.shape(4096, 4096, 17, 17), 1, 0)
    return {c: float(rng.uniform(0.1, 5.0)) for c in cfgs}


def test_synthetic_tuner_matches_statistics_oracle(tmp_path):
    table = _cost_table()
    # two near-ties with the fastest: the smaller tuple within 0.5 % must win
    fastest = min(table, key=table.get)
    others = sorted(c for c in table if c < fastest)
    if others:
        table[others[0]] = table[fastest] * 1.004
    winners = tmp_path / "w.jsonl"
    results = tmp_path / "r.jsonl"
    o = C.conv2d_tune_defaults()
    o.winners_path, o.results_path = str(winners).encode(), str(results).encode()
    s = C.shape(4096, 4096, 17, 17)
    r = C.conv2d_tune_synthetic(s, lambda c: table[c], o)
    assert r.best.tuple() == otune.pick_winner(table)
    assert [r.top[k].tuple() for k in range(5)] == otune.top_k(table, 5)
    perf = [2 * 4096 * 4096 * 289 / (t * 1e-3) / 1e9 for t in table.values()]
    assert r.impact == pytest.approx(otune.tuning_impact(perf), rel=1e-12)
    assert r.median_gflops == pytest.approx(otune.median(perf), rel=1e-12)
    assert r.n_space == 1216 and r.n_illegal == 14 and r.n_timed == 1202
    d = (16, 16, 1, 1, 1, 1, 1)
    assert r.default_ms == table[d]                  # the synthetic cost has one timing mode
    assert r.default_sweep_ms == table[d] and r.best_sweep_ms == table[r.best.tuple()]
    assert r.default_rank == 1 + sum(1 for t in table.values() if t < table[d])
    # the winners cache and the results DB
    assert C.conv2d_cache_lookup(str(winners), "synthetic", s)[0].tuple() == r.best.tuple()
    lines = [json.loads(x) for x in open(results)]
    assert len(lines) == 1202 and all(x["status"] == "ok" for x in lines)
    # resume: nothing is measured again, the same winner comes out
    calls = []
    r2 = C.conv2d_tune_synthetic(s, lambda c: calls.append(c) or table[c], o)
    assert r2.n_resumed == 1202 and r2.best.tuple() == r.best.tuple()
    # only the re-timing of the ten fastest and of the default (prepare + measure each)
    assert len(calls) <= 22


def test_synthetic_tuner_records_failures(tmp_path):
    table = _cost_table(5)
    fail = {}
    for k, c in enumerate(sorted(table)):
        if k % 97 == 0:
            fail[c] = C.CONV2D_ECOMPILE
        elif k % 89 == 0:
            fail[c] = C.CONV2D_ELAUNCH
        elif k % 83 == 0:
            fail[c] = C.CONV2D_EVERIFY
    cost = lambda c: float(fail.get(c, table[c]))  # noqa: E731
    r = C.conv2d_tune_synthetic(C.shape(4096, 4096, 17, 17), cost, None)
    assert r.n_compile_fail == sum(1 for v in fail.values() if v == C.CONV2D_ECOMPILE)
    assert r.n_launch_fail == sum(1 for v in fail.values() if v == C.CONV2D_ELAUNCH)
    assert r.n_verify_fail == sum(1 for v in fail.values() if v == C.CONV2D_EVERIFY)
    ok = {c: t for c, t in table.items() if c not in fail}
    assert r.best.tuple() == otune.pick_winner(ok)


def test_refine_unroll_adds_variants():
    table = _cost_table(7)
    s = C.shape(4096, 4096, 17, 17)
    o = C.conv2d_tune_defaults()
    o.refine_unroll = 1
    best_plain = min(table, key=table.get)
    # unroll 2 of the fastest point is faster still
    cost = lambda c: table[c[:6] + (1,)] * (0.9 if c[6] == 2 and c[:6] == best_plain[:6] else 1.0)  # noqa: E731
    r = C.conv2d_tune_synthetic(s, cost, o)
    assert r.best.tuple() == best_plain[:6] + (2,)


def test_cache_prefers_current_kernel_source(tmp_path):
    p = tmp_path / "w.jsonl"
    s = C.shape(100, 200, 5, 5)
    old = {"arch": "gfx950", "src": "0000000000000000", "shape": [100, 200, 5, 5], "config": [64, 1, 8, 8, 0, 0, 1],
           "ms": 1.0}
    p.write_text(json.dumps(old) + "\n{not json\n")
    c, ms = C.conv2d_cache_lookup(str(p), "gfx950", s)
    assert c.tuple() == (64, 1, 8, 8, 0, 0, 1)                     # stale entry used as a fallback
    C.conv2d_cache_store(str(p), "gfx950", s, (32, 2, 4, 4, 1, 1, 2), 0.5)
    p.write_text(p.read_text() + json.dumps(old) + "\n")           # a later stale line does not win
    c, ms = C.conv2d_cache_lookup(str(p), "gfx950", s)
    assert c.tuple() == (32, 2, 4, 4, 1, 1, 2) and ms == 0.5
    assert C.conv2d_cache_lookup(str(p), "gfx942", s) is None
    assert C.conv2d_cache_lookup(str(p), "gfx950", C.shape(100, 200, 3, 3)) is None


@pytest.mark.parametrize("seed,budget", [(1, 60), (7, 200), (123, 1300)])
def test_local_search_follows_its_definition(tmp_path, seed, budget):
    """The tuner's local-search strategy (synthetic cost) evaluates exactly the
    points, in exactly the order, of the plain replay in the oracle, and
    returns the same best point; with a budget above the space it reaches
    the global optimum."""
    import json as _json
    rng = np.random.default_rng(seed)
    s = C.shape(4096, 4096, 17, 17)
    legal = C.conv2d_space(s, 1, 0)
    table = {c: float(rng.lognormal(0, 0.4)) for c in legal}
    fails = {c for k, c in enumerate(legal) if k % 53 == 0}
    cost = {c: (C.CONV2D_ECOMPILE if c in fails else t) for c, t in table.items()}
    o = C.conv2d_tune_defaults()
    o.strategy, o.max_evals, o.seed = 1, budget, seed
    res_path = tmp_path / "r.jsonl"
    o.results_path = str(res_path).encode()
    r = C.conv2d_tune_synthetic(s, lambda c: cost[c], o)
    order = [tuple(_json.loads(x)["config"]) for x in open(res_path)]
    axes = [list(v) for _, v in ospace.AXES]
    best, want = otune.local_search({c: (None if c in fails else t) for c, t in table.items()}, legal, axes,
                                    budget, seed)
    assert order == want
    assert r.best.tuple() == best and r.evaluations == len(want)
    if budget >= len(legal):
        ok = {c: t for c, t in table.items() if c not in fails}
        assert best == min(ok, key=lambda c: (ok[c], c))


# ---------------------------------------------------------------- hotspot

HS_HEADER = os.path.join(ROOT, "include", "hotspot.h")


def test_library_exports_every_hotspot_function():
    text = re.sub(r"/\*.*?\*/", "", open(HS_HEADER).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(hotspot_[a-z0-9_]+)\s*\(", text)))
    assert len(names) >= 12
    assert not [n for n in names if not hasattr(C.lib, n)]


def test_hotspot_space_matches_oracle_enumeration():
    got = C.hotspot_space(C.hotspot_shape(4096, 4096))
    assert got == ospace.hotspot_restricted()
    assert len(got) == 2040
    assert all(C.hotspot_lds_bytes(c) <= 163840 for c in got)


def test_hotspot_config_check_errors():
    s = C.hotspot_shape(64, 64)
    assert C.hotspot_config_check(s, (32, 8, 1, 1, 1, 1, 1)) == 0
    for bad in [(16, 2, 1, 1, 1, 1, 1),      # 32 threads
                (48, 2, 1, 1, 1, 1, 1),      # block_x off its axis
                (256, 8, 1, 1, 1, 1, 1),     # 2048 threads
                (64, 1, 1, 1, 1, 1, 1),      # one region row: not larger than 2 * temporal
                (32, 4, 1, 2, 4, 1, 1),      # 8 rows, temporal 4
                (32, 8, 3, 1, 1, 1, 1),      # tile_x off its axis
                (32, 8, 1, 1, 5, 1, 1),      # temporal off its axis
                (32, 8, 1, 1, 1, 2, 1),
                (32, 8, 1, 1, 1, 1, 2)]:
        assert C.hotspot_config_check(s, bad) == C.CONV2D_EINVAL, bad
        assert C.conv2d_last_error()
    # a 16 x 1024 region in two ringed buffers needs 147,888 bytes of LDS:
    # legal at 160 KiB, rejected under a 64 KiB limit
    assert C.hotspot_lds_bytes((256, 4, 4, 4, 1, 1, 1)) == 147888
    assert C.hotspot_config_check(s, (256, 4, 4, 4, 1, 1, 1)) == 0
    assert C.hotspot_config_check(s, (256, 4, 4, 4, 1, 1, 1), 65536) == C.CONV2D_EINVAL
    assert C.hotspot_config_check(C.hotspot_shape(0, 4), (32, 8, 1, 1, 1, 1, 1)) == C.CONV2D_EINVAL


@pytest.mark.parametrize("cfg", [(32, 8, 1, 1, 1, 1, 1), (64, 4, 2, 4, 4, 0, 1), (16, 16, 4, 4, 6, 0, 0),
                                 (128, 2, 4, 2, 1, 1, 0), (128, 8, 1, 4, 8, 0, 1)])
def test_hotspot_code_is_plain_fp32_without_spills(cfg):
    """No packed FP32 instruction; three FMAs per cell and step in each of
    the two step loops (grid edge, interior), fully unrolled or one step
    rolled, plus the source term's FMAs: at most one per cell in each of the
    two paths, per step when power is read per step (the compiler may merge
    the paths' copies or hoist a step's out of the loop); LDS within the
    stated bound; no scratch."""
    path = C.hotspot_compile(cfg)
    isa = subprocess.run([OBJDUMP, "-d", path], capture_output=True, text=True).stdout
    assert "v_pk_" not in isa
    bx, by, tx, ty, tt, unroll_t, sh_power = cfg
    steps_in_code = 1 if unroll_t else tt
    n_source = isa.count("v_fmac_f32") + isa.count("v_fma_f32") - 2 * 3 * tx * ty * steps_in_code
    assert 0 < n_source <= 2 * tx * ty * (1 if sh_power else steps_in_code)
    n = _notes(path)
    assert n["private_segment_fixed_size"] == 0 and n["vgpr_spill_count"] == 0
    assert 0 < n["group_segment_fixed_size"] <= C.hotspot_lds_bytes(cfg)


def test_serving_tuner_pick():
    """The server-parameter tuner's choice: lowest p99, p99s within 2 % tie,
    ties to the lowest p50, then fewer streams, then the smaller cap."""
    from paper_2407_11488_amd.workloads import pick_serving
    t = [{"streams": 4, "max_batch": 64, "p50_ms": 0.05, "p99_ms": 0.300},
         {"streams": 2, "max_batch": 16, "p50_ms": 0.04, "p99_ms": 0.305},
         {"streams": 8, "max_batch": 16, "p50_ms": 0.04, "p99_ms": 0.303},
         {"streams": 1, "max_batch": 1, "p50_ms": 0.02, "p99_ms": 0.400}]
    assert pick_serving(t) == t[1]                      # tie on p99 and p50: fewer streams
    assert pick_serving(t, tie_rel=0.0) == t[0]         # no ties: strictly lowest p99
    assert pick_serving(t[3:]) == t[3]


def test_size_buckets_follow_the_larger_side():
    """Bucket edges at larger sides 384, 768, 1536, 3072 (inclusive), and the
    same rule for the batched path's tuning and its plans."""
    cases = {(1, 1): 1, (384, 10): 1, (385, 385): 2, (10, 768): 2, (769, 1): 3, (1536, 1536): 3,
             (1537, 200): 4, (3072, 3072): 4, (3073, 5): 5, (100000, 1): 5, (0, 0): 1}
    for (h, w), b in cases.items():
        assert C.conv2d_size_bucket(h, w) == b, (h, w)
    assert C.conv2d_size_bucket(200, 3000) == C.conv2d_size_bucket(3000, 200) == 4


def test_bench_traffic_record_matches_only_its_kernel():
    """bench.py reports the committed rocprofv3 traffic only for the kernel
    source and configuration it was measured on (else null): the record
    matches the committed 4096x4096 / 17x17 winner of the current source."""
    import sys as _sys
    _sys.path.insert(0, ROOT)
    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "conv2d_direct_4096x4096_f17_traffic.json")))

    class Plan:
        config = tuple(rec["config"])
    assert rec["kernel_hash"] == C.conv2d_kernel_hash()
    got, src = bench.measured_traffic(C, Plan())
    assert got == rec["traffic_bytes_per_launch"] and src.endswith("_traffic.json")
    assert 1.0 <= got / rec["algorithmic_bytes_per_launch"] < 1.1

    class Other:
        config = (16, 16, 1, 1, 1, 1, 1)
    assert bench.measured_traffic(C, Other()) == (None, None)
    win = C.conv2d_cache_lookup(os.path.join(ROOT, "paper_2407_11488_amd", "tuned", "winners.jsonl"), "gfx950",
                                C.shape(4096, 4096, 17, 17))
    assert win is not None and win[0].tuple() == tuple(rec["config"])


@pytest.mark.parametrize("arrivals", [(0.0, float("nan")), (-1.0, 0.0), (0.0, float("inf")), (0.5, 0.25)])
def test_serve_rejects_bad_arrival_times_before_device_work(arrivals):
    """Arrival times must be finite, >= 0 and non-decreasing; the check runs
    before the device is queried, so it holds without a GPU."""
    reqs = C.requests_array(list(arrivals), [(64, 64, 3, 3)] * len(arrivals), [1, 2], [3, 4])
    with pytest.raises(RuntimeError, match="arrival"):
        C.conv2d_serve(reqs)


def _declarations_with_comments(path):
    """(function name, the comment block above its declaration) for every
    function declared in a header. Declarations written one after another
    with no blank line (a pair such as lookup/store) share the comment above
    the first."""
    lines = open(path).read().split("\n")
    decl = re.compile(r"^[A-Za-z_][\w\s\*]*?\b((?:conv2d|hotspot)_[a-z0-9_]+)\s*\(")
    out = []
    for k, line in enumerate(lines):
        m = decl.match(line)
        if not m or line.startswith("typedef"):
            continue
        j = k - 1
        while j >= 0 and lines[j].strip() and not lines[j].rstrip().endswith("*/"):
            j -= 1                       # the previous declaration of a group, or its continuation
        comment = []
        if j >= 0 and lines[j].rstrip().endswith("*/"):
            while j >= 0:
                comment.append(lines[j])
                if lines[j].lstrip().startswith("/*"):
                    break
                j -= 1
        out.append((m.group(1), "\n".join(reversed(comment))))
    return out


@pytest.mark.parametrize("path", [HEADER, os.path.join(ROOT, "include", "hotspot.h")])
def test_every_entry_point_states_its_source(path):
    """Each declaration in the public headers is preceded by a comment with a
    'Source:' line naming the passage of the paper that defines the
    operation (a section, equation or table), or stating that none does."""
    decls = _declarations_with_comments(path)
    names = {n for n, _ in decls}
    declared = set(re.findall(r"\b((?:conv2d|hotspot)_[a-z0-9_]+)\s*\(", re.sub(r"/\*.*?\*/", "", open(path).read(),
                                                                            flags=re.S)))
    declared = {n for n in declared if not n.endswith("_fn")}
    assert declared <= names, sorted(declared - names)
    bad = []
    for name, comment in decls:
        m = re.search(r"Source:\s*(.*?)(?:\*/|$)", comment, re.S)
        if not m:
            bad.append((name, "no Source line"))
            continue
        src = " ".join(m.group(1).replace("*", " ").split())
        if not (re.search(r"\b(Section|Table|Eq)\.?\s*\d", src) or src.startswith("none in the paper")
                or src.startswith("as conv2d_tune")):
            bad.append((name, src))
    assert not bad, bad
    for must in ("conv2d_plan", "conv2d_run", "conv2d_tune", "conv2d_batch_plan", "conv2d_batch_run",
                 "hotspot_run", "hotspot_tune"):
        for name, comment in decls:
            if name == must:
                assert re.search(r"Source:.*?(Section|Table)\s*\d", comment, re.S), name
