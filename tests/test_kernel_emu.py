"""The tunable kernel source run on the CPU (tests/emu): one host thread per GPU
thread, real barriers, bounds-checked buffer loads, AddressSanitizer and
UBSan. Each configuration must equal the FP64 oracle bit for bit on integer
data (exact in any order), write every output, and make no out-of-bounds
access, on input pitches and output widths of every residue mod 4, with
the four-wide loads and stores the library builds for all of them (each
dword of a buffer load range-checked, as on the GPU). No GPU needed."""
import concurrent.futures as cf
import hashlib
import os
import subprocess
import tempfile

import numpy as np
import pytest

import datagen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.path.join(HERE, "emu")
KERNEL = os.path.join(os.path.dirname(HERE), "paper_2407_11488_amd", "csrc", "conv2d_direct.hip")
HOTSPOT = os.path.join(os.path.dirname(HERE), "paper_2407_11488_amd", "csrc", "hotspot.hip")
CXX = "/opt/rocm/llvm/bin/clang++"
BIN_DIR = os.path.join(tempfile.gettempdir(), "conv2d_emu_bins")

# (block_x, block_y) x tiles x lds x const, plus unroll variants; kept small
# enough for the CPU suite. CONV2D_EMU_FULL=1 runs the whole 1216-point space.
BLOCKS = [(16, 1), (64, 1), (32, 4), (16, 16), (128, 2)]
TILES = [(1, 1), (2, 4), (4, 1), (8, 8), (4, 2), (1, 8)]


def sample_configs():
    if os.environ.get("CONV2D_EMU_FULL") == "1":
        return [(bx, by, tx, ty, l, c, 1) for bx in (16, 32, 64, 128) for by in (1, 2, 4, 8, 16)
                for tx in (1, 2, 4, 8) for ty in (1, 2, 4, 8) for l in (0, 1) for c in (0, 1) if bx * by <= 1024]
    out = []
    for k, (bx, by) in enumerate(BLOCKS):
        for j, (tx, ty) in enumerate(TILES):
            for lds in (0, 1):
                out.append((bx, by, tx, ty, lds, (k + j + lds) % 2, 1))
    out += [(64, 1, 8, 8, 0, 0, 0), (64, 2, 4, 4, 1, 1, 2), (32, 1, 2, 8, 0, 1, 4), (16, 4, 8, 2, 1, 0, 0)]
    return out


# (H, W, fh, fw): input pitches 47, 38, 76, 8, 43 and 41 (3, 2, 0, 0, 3 and 1
# mod 4), output widths 45, 36, 72, 5, 39 and 38 (1, 0, 0, 1, 3 and 2 mod 4),
# and a shape smaller than one tile.
SHAPES = [(21, 45, 5, 3), (13, 36, 3, 3), (9, 72, 7, 5), (3, 5, 2, 4), (11, 39, 3, 5), (7, 38, 4, 4)]


def build(cfg, fh, fw, vin, vout):
    bx, by, tx, ty, lds, fc, un = cfg
    defs = dict(BX=bx, BY=by, TX=tx, TY=ty, USE_LDS=lds, FCONST=fc, UNROLL=un, FH=fh, FW=fw, VIN=vin, VOUT=vout)
    src = open(KERNEL).read() + open(os.path.join(EMU, "emu_direct.cpp")).read() + \
        open(os.path.join(EMU, "hip_emu.h")).read()
    key = hashlib.sha1((src + repr(sorted(defs.items()))).encode()).hexdigest()[:16]
    os.makedirs(BIN_DIR, exist_ok=True)
    exe = os.path.join(BIN_DIR, f"emu_{key}")
    if not os.path.exists(exe):
        cmd = [CXX, "-std=c++20", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-fno-omit-frame-pointer", *[f"-DCONV_{k}={v}" for k, v in defs.items()],
               os.path.join(EMU, "emu_direct.cpp"), "-o", exe + f".{os.getpid()}.tmp", "-lpthread"]
        subprocess.run(cmd, check=True, capture_output=True)
        os.replace(exe + f".{os.getpid()}.tmp", exe)
    return exe


def run(exe, inp, f, H, W, tmp):
    pi, pf, po = (os.path.join(tmp, n) for n in ("in.f32", "f.f32", "out.f32"))
    inp.astype(np.float32).tofile(pi)
    f.astype(np.float32).tofile(pf)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    r = subprocess.run([exe, pi, pf, po, str(H), str(W)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    return np.fromfile(po, np.float32).reshape(H, W)


@pytest.fixture(scope="module")
def binaries():
    jobs = []
    for (H, W, fh, fw) in SHAPES:
        for cfg in sample_configs():
            lds_rows = cfg[1] * cfg[3] + fh - 1
            lds_cols = cfg[0] * cfg[2] + fw - 1
            if cfg[4] and lds_rows * (lds_cols + 8) * 4 > 163840:
                continue
            jobs.append(((H, W, fh, fw), cfg))
    with cf.ThreadPoolExecutor(os.cpu_count() or 4) as ex:
        futs = {job: ex.submit(build, job[1], job[0][2], job[0][3], 4, 4) for job in jobs}
        return {job: f.result() for job, f in futs.items()}


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_emulated_kernel_exact(binaries, shape, tmp_path):
    H, W, fh, fw = shape
    inp, f = datagen.conv_problem(H, W, fh, fw, kind="int", seed_in=H, seed_f=W)
    ref, _ = oracle.conv2d_f64(inp, f)
    n = 0
    for (shp, cfg), exe in binaries.items():
        if shp != shape:
            continue
        got = run(exe, inp, f, H, W, str(tmp_path))
        assert np.all(np.isfinite(got)), f"unwritten outputs for {cfg}"
        assert np.array_equal(got.astype(np.float64), ref), f"config {cfg} differs from the oracle"
        n += 1
    assert n > 20


BATCH_CONFIGS = [(16, 1, 1, 1, 0, 0, 1), (64, 1, 4, 4, 1, 0, 0), (32, 4, 2, 8, 0, 0, 1), (16, 16, 4, 1, 1, 0, 2),
                 (128, 2, 8, 2, 1, 0, 1)]


def build_batch(cfg, fh, fw):
    bx, by, tx, ty, lds, fc, un = cfg
    defs = dict(BX=bx, BY=by, TX=tx, TY=ty, USE_LDS=lds, FCONST=0, UNROLL=un, FH=fh, FW=fw, VIN=4, VOUT=4, BATCH=1)
    src = open(KERNEL).read() + open(os.path.join(EMU, "emu_batch.cpp")).read() + \
        open(os.path.join(EMU, "hip_emu.h")).read()
    key = hashlib.sha1((src + repr(sorted(defs.items()))).encode()).hexdigest()[:16]
    os.makedirs(BIN_DIR, exist_ok=True)
    exe = os.path.join(BIN_DIR, f"emub_{key}")
    if not os.path.exists(exe):
        cmd = [CXX, "-std=c++20", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-fno-omit-frame-pointer", *[f"-DCONV_{k}={v}" for k, v in defs.items()],
               os.path.join(EMU, "emu_batch.cpp"), "-o", exe + f".{os.getpid()}.tmp", "-lpthread"]
        subprocess.run(cmd, check=True, capture_output=True)
        os.replace(exe + f".{os.getpid()}.tmp", exe)
    return exe


@pytest.mark.parametrize("fh,fw", [(3, 3), (5, 2)])
def test_emulated_batch_kernel_exact(fh, fw, tmp_path):
    """The batched kernel, built as the library builds it (4-wide loads and
    stores at any dword boundary), over uneven images on grids smaller than its tile
    count (each workgroup striding over several tiles): every output of every
    image written once and exact, for grids that are and are not multiples
    of 8, with rows of every width mod 4."""
    sizes = [(37, 45), (5, 130), (64, 64), (1, 1), (19, 7), (9, 71)]
    probs = []
    for k, (H, W) in enumerate(sizes):
        inp, f = datagen.conv_problem(H, W, fh, fw, kind="int", seed_in=100 + k, seed_f=200 + k)
        inp.astype(np.float32).tofile(tmp_path / f"in{k}.f32")
        f.astype(np.float32).tofile(tmp_path / f"f{k}.f32")
        probs.append((H, W, oracle.conv2d_f64(inp, f)[0]))
    with cf.ThreadPoolExecutor(os.cpu_count() or 4) as ex:
        exes = list(ex.map(lambda c: build_batch(c, fh, fw), BATCH_CONFIGS))
    args = [str(v) for H, W, _ in probs for v in (H, W)]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    for cfg, exe in zip(BATCH_CONFIGS, exes):
        for grid in (8, 11, 24):
            r = subprocess.run([exe, str(grid), str(tmp_path), str(len(probs)), *args], capture_output=True,
                               text=True, env=env, timeout=300)
            assert r.returncode == 0, r.stderr[-3000:]
            for k, (H, W, ref) in enumerate(probs):
                got = np.fromfile(tmp_path / f"out{k}.f32", np.float32).reshape(H, W)
                assert np.array_equal(got.astype(np.float64), ref), (cfg, grid, k)


# Hotspot configurations (block_x, block_y, tile_x, tile_y, temporal,
# unroll_t, sh_power): one cell per thread, x and y tiling, temporal factors
# from 1 to 8 with full and partial last launches, both power modes, thread
# rows of 16, 32 and 64 lanes (the lane-shift exchange) and of 128 (the
# region copy in LDS).
HOTSPOT_CONFIGS = [(16, 4, 1, 1, 1, 1, 1), (32, 2, 2, 4, 2, 0, 0), (16, 8, 4, 2, 3, 1, 1), (64, 1, 1, 4, 1, 0, 1),
                   (16, 16, 1, 1, 6, 0, 0), (32, 4, 2, 4, 3, 1, 0), (16, 8, 4, 4, 8, 0, 1), (64, 4, 2, 4, 6, 1, 1),
                   (64, 2, 2, 4, 3, 0, 1), (128, 2, 2, 4, 3, 1, 1)]


def build_hotspot(cfg):
    bx, by, tx, ty, tt, u, p = cfg
    defs = dict(BX=bx, BY=by, TX=tx, TY=ty, TT=tt, UNROLL_T=u, SH_POWER=p)
    src = open(HOTSPOT).read() + open(os.path.join(EMU, "emu_hotspot.cpp")).read() + \
        open(os.path.join(EMU, "hip_emu.h")).read()
    key = hashlib.sha1((src + repr(sorted(defs.items()))).encode()).hexdigest()[:16]
    os.makedirs(BIN_DIR, exist_ok=True)
    exe = os.path.join(BIN_DIR, f"emuh_{key}")
    if not os.path.exists(exe):
        cmd = [CXX, "-std=c++20", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-fno-omit-frame-pointer", *[f"-DHS_{k}={v}" for k, v in defs.items()],
               "-DHS_NAME=hotspot_emu", os.path.join(EMU, "emu_hotspot.cpp"), "-o", exe + f".{os.getpid()}.tmp", "-lpthread"]
        subprocess.run(cmd, check=True, capture_output=True)
        os.replace(exe + f".{os.getpid()}.tmp", exe)
    return exe


def _check_hotspot(tmp_path, cfgs, grids):
    """Every configuration in cfgs on every (rows, cols, steps) grid: the
    same bits across configurations, within the FP32 bound of the FP64
    oracle."""
    with cf.ThreadPoolExecutor(os.cpu_count() or 4) as ex:
        exes = list(ex.map(build_hotspot, cfgs))
    k = (0.2, 0.5, 0.75, 0.05, 0.25)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    for (rows, cols, steps) in grids:
        temp = datagen.uniform_pm1(61, rows * cols).reshape(rows, cols)
        power = datagen.uniform_pm1(62, rows * cols).reshape(rows, cols)
        temp.tofile(tmp_path / "temp.f32")
        power.tofile(tmp_path / "power.f32")
        ref = oracle.hotspot_f64(temp, power, steps, *k)
        bound = 8 * max(steps, 1) * 2.0 ** -24 * (1.0 + abs(k[4]) + steps * k[0] * 1.0)

        def emulate(job):
            # each configuration in a directory of its own, so that they run in parallel
            i, exe = job
            d = tmp_path / f"run{i}"
            d.mkdir(exist_ok=True)
            for name in ("temp.f32", "power.f32"):
                (d / name).write_bytes((tmp_path / name).read_bytes())
            r = subprocess.run([exe, str(rows), str(cols), str(steps), *[repr(v) for v in k], str(d)],
                               capture_output=True, text=True, env=env, timeout=300)
            assert r.returncode == 0, r.stderr[-3000:]
            return np.fromfile(d / "out.f32", np.float32).reshape(rows, cols)

        with cf.ThreadPoolExecutor(4) as ex:
            outs = list(ex.map(emulate, enumerate(exes)))
        first = None
        for cfg, got in zip(cfgs, outs):
            assert np.all(np.isfinite(got)), (cfg, rows, cols)
            assert np.max(np.abs(got - ref)) <= bound, (cfg, rows, cols, np.max(np.abs(got - ref)))
            if first is None:
                first = got
            assert np.array_equal(got.view(np.uint32), first.view(np.uint32)), (cfg, rows, cols)


def test_emulated_hotspot_kernel(tmp_path):
    """The temporally tiled hotspot kernel on uneven grids (smaller than one
    tile, several tiles with ragged edges, one row, one column)."""
    _check_hotspot(tmp_path, HOTSPOT_CONFIGS, [(37, 45, 7), (5, 130, 3), (1, 9, 4), (23, 1, 5), (70, 3, 9), (2, 2, 0)])


def test_emulated_hotspot_interior_regions(tmp_path):
    """Grids with regions away from every edge (the buffer-addressed loads and
    stores) beside edge regions, for configurations whose regions fit inside
    them several times: 64 x 16 and 64 x 8 cells, 128 x 8."""
    _check_hotspot(tmp_path, [(32, 4, 2, 4, 3, 1, 1), (16, 8, 4, 2, 2, 1, 0), (64, 2, 2, 4, 3, 0, 1)],
                   [(130, 200, 7), (61, 300, 4)])
