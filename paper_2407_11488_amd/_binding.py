"""ctypes binding of libconv2d.so: the C entry points under the same names.

Argument marshalling only; every step of the computation runs in the HIP
library. Import fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libconv2d.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2407_11488_amd/build.py` "
                      "(there is no CPU fallback)")

# PyTorch ships its own HIP runtime. Loading it first makes the library's
# libamdhip64.so.7 / libhiprtc.so.7 dependencies resolve to those already
# loaded copies, so that device memory allocated by torch and by this library
# belongs to one runtime. (Loaded the other way round, torch would map a
# second runtime beside the system one.)
try:
    import torch  # noqa: F401
except ImportError:  # standalone use: the system ROCm runtime
    torch = None

lib = ctypes.CDLL(LIB_PATH)


def _hip_runtimes():
    try:
        with open("/proc/self/maps") as fh:
            return sorted({ln.split()[-1] for ln in fh if "libamdhip64" in ln})
    except OSError:
        return []


if len(_hip_runtimes()) > 1:
    raise ImportError("two HIP runtimes are mapped in this process (" + ", ".join(_hip_runtimes()) +
                      "); import torch before loading libconv2d.so")

c_int, c_double, c_void_p, c_char_p, c_size_t, c_uint64 = (
    ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_char_p, ctypes.c_size_t, ctypes.c_uint64)

STATUS = {0: "CONV2D_OK", -1: "CONV2D_EINVAL", -2: "CONV2D_ENOMEM", -3: "CONV2D_ECOMPILE",
          -4: "CONV2D_ELAUNCH", -5: "CONV2D_ENOTUNED", -6: "CONV2D_EVERIFY", -7: "CONV2D_EHIP",
          -8: "CONV2D_EBUSY"}
CONV2D_OK, CONV2D_EINVAL, CONV2D_ENOMEM, CONV2D_ECOMPILE = 0, -1, -2, -3
CONV2D_ELAUNCH, CONV2D_ENOTUNED, CONV2D_EVERIFY, CONV2D_EHIP, CONV2D_EBUSY = -4, -5, -6, -7, -8


class Conv2dError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib.conv2d_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


class Shape(ctypes.Structure):
    _fields_ = [("out_h", c_int), ("out_w", c_int), ("filt_h", c_int), ("filt_w", c_int)]

    def tuple(self):
        return (self.out_h, self.out_w, self.filt_h, self.filt_w)


class Config(ctypes.Structure):
    _fields_ = [("block_x", c_int), ("block_y", c_int), ("tile_x", c_int), ("tile_y", c_int),
                ("use_lds", c_int), ("filter_in_const", c_int), ("unroll", c_int)]

    def tuple(self):
        return tuple(getattr(self, f) for f, _ in self._fields_)

    def __repr__(self):
        return "Config(" + ",".join(str(v) for v in self.tuple()) + ")"


class TuneOpts(ctypes.Structure):
    _fields_ = [("winners_path", c_char_p), ("results_path", c_char_p), ("warmup", c_int), ("reps", c_int),
                ("retime_reps", c_int), ("flush_mall", c_int), ("threads", c_int), ("unroll", c_int),
                ("max_configs", c_int), ("tie_rel", c_double), ("verbose", c_int),
                ("refine_unroll", c_int), ("strategy", c_int), ("max_evals", c_int), ("seed", c_uint64)]


class TuneResult(ctypes.Structure):
    _fields_ = [("best", Config), ("best_ms", c_double), ("default_ms", c_double), ("median_ms", c_double),
                ("best_gflops", c_double), ("median_gflops", c_double), ("default_gflops", c_double),
                ("impact", c_double), ("n_space", c_int), ("n_illegal", c_int), ("n_compile_fail", c_int),
                ("n_launch_fail", c_int), ("n_verify_fail", c_int), ("n_timed", c_int), ("n_resumed", c_int),
                ("default_rank", c_int), ("top", Config * 5), ("top_ms", c_double * 5),
                ("compile_s", c_double), ("measure_s", c_double), ("evaluations", c_int),
                ("best_sweep_ms", c_double), ("default_sweep_ms", c_double)]


COST_FN = ctypes.CFUNCTYPE(c_double, ctypes.POINTER(Config), c_void_p)
P = ctypes.POINTER

_SIGS = {
    "conv2d_version": (c_int, []),
    "conv2d_last_error": (c_char_p, []),
    "conv2d_kernel_hash": (c_char_p, []),
    "conv2d_default_config": (None, [P(Config)]),
    "conv2d_lds_bytes": (c_int, [c_int, c_int, P(Config)]),
    "conv2d_config_check": (c_int, [Shape, P(Config), c_int]),
    "conv2d_space": (c_int, [Shape, c_int, c_int, P(Config), c_int]),
    "conv2d_compile": (c_int, [Shape, P(Config), c_int, c_int, c_char_p, c_int]),
    "conv2d_geometry": (c_int, [Shape, P(Config), P(c_int), P(c_int), P(c_int)]),
    "conv2d_cache_lookup": (c_int, [c_char_p, c_char_p, Shape, P(Config), P(c_double)]),
    "conv2d_cache_store": (c_int, [c_char_p, c_char_p, Shape, P(Config), c_double]),
    "conv2d_plan": (c_int, [P(c_void_p), Shape, P(Config)]),
    "conv2d_plan_config": (c_int, [c_void_p, P(Config), P(c_int)]),
    "conv2d_run": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "conv2d_destroy": (None, [c_void_p]),
    "conv2d_reference": (c_int, [Shape, c_void_p, c_void_p, c_void_p, c_void_p]),
    "conv2d_fill_uniform": (c_int, [c_void_p, c_size_t, c_uint64, c_uint64, c_void_p]),
    "conv2d_tune_defaults": (None, [P(TuneOpts)]),
    "conv2d_tune": (c_int, [Shape, P(TuneOpts), P(TuneResult)]),
    "conv2d_tune_synthetic": (c_int, [Shape, COST_FN, c_void_p, P(TuneOpts), P(TuneResult)]),
    "conv2d_benchmark": (c_int, [Shape, P(Config), c_int, c_int, c_int, P(c_double), P(c_double)]),
}


def _bind():
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args


_bind()


def check(rc: int, where: str) -> int:
    if rc < 0:
        raise Conv2dError(rc, where)
    return rc


def shape(out_h, out_w, filt_h, filt_w) -> Shape:
    return Shape(int(out_h), int(out_w), int(filt_h), int(filt_w))


def config(*vals) -> Config:
    if len(vals) == 1 and isinstance(vals[0], (tuple, list, Config)):
        vals = tuple(vals[0].tuple() if isinstance(vals[0], Config) else vals[0])
    if len(vals) == 6:
        vals = (*vals, 1)
    return Config(*[int(v) for v in vals])


# ---------------------------------------------------------------- entry points (same names)

def conv2d_version() -> int:
    return lib.conv2d_version()


def conv2d_last_error() -> str:
    return lib.conv2d_last_error().decode(errors="replace")


def conv2d_kernel_hash() -> str:
    return lib.conv2d_kernel_hash().decode()


def conv2d_default_config() -> Config:
    c = Config()
    lib.conv2d_default_config(ctypes.byref(c))
    return c


def conv2d_lds_bytes(filt_h: int, filt_w: int, cfg) -> int:
    return check(lib.conv2d_lds_bytes(filt_h, filt_w, ctypes.byref(config(cfg))), "conv2d_lds_bytes")


def conv2d_config_check(s: Shape, cfg, lds_limit: int = 0) -> int:
    """Returns 0 when legal, else the negative status (no exception)."""
    return lib.conv2d_config_check(s, ctypes.byref(config(cfg)), lds_limit)


def conv2d_space(s: Shape, unroll: int = 1, lds_limit: int = 0):
    n = check(lib.conv2d_space(s, unroll, lds_limit, None, 0), "conv2d_space")
    arr = (Config * max(n, 1))()
    lib.conv2d_space(s, unroll, lds_limit, arr, n)
    return [arr[i].tuple() for i in range(n)]


def conv2d_compile(s: Shape, cfg, vec_in: int = 4, vec_out: int = 4) -> str:
    buf = ctypes.create_string_buffer(4096)
    check(lib.conv2d_compile(s, ctypes.byref(config(cfg)), vec_in, vec_out, buf, 4096), "conv2d_compile")
    return buf.value.decode()


def conv2d_geometry(s: Shape, cfg):
    tx, ty, nt = c_int(), c_int(), c_int()
    check(lib.conv2d_geometry(s, ctypes.byref(config(cfg)), ctypes.byref(tx), ctypes.byref(ty),
                              ctypes.byref(nt)), "conv2d_geometry")
    return tx.value, ty.value, nt.value


def _b(s):
    return None if s is None else (s.encode() if isinstance(s, str) else s)


def conv2d_cache_lookup(path, arch, s: Shape):
    c, ms = Config(), c_double()
    rc = lib.conv2d_cache_lookup(_b(path), _b(arch), s, ctypes.byref(c), ctypes.byref(ms))
    if rc == CONV2D_ENOTUNED:
        return None
    check(rc, "conv2d_cache_lookup")
    return c, ms.value


def conv2d_cache_store(path, arch, s: Shape, cfg, ms: float) -> None:
    check(lib.conv2d_cache_store(_b(path), _b(arch), s, ctypes.byref(config(cfg)), ms), "conv2d_cache_store")


def conv2d_plan(s: Shape, cfg=None) -> int:
    h = c_void_p()
    check(lib.conv2d_plan(ctypes.byref(h), s, None if cfg is None else ctypes.byref(config(cfg))), "conv2d_plan")
    return h.value


def conv2d_plan_config(plan: int):
    c, src = Config(), c_int()
    check(lib.conv2d_plan_config(plan, ctypes.byref(c), ctypes.byref(src)), "conv2d_plan_config")
    return c, src.value


def conv2d_run(plan: int, d_in: int, d_filter: int, d_out: int, stream: int = 0) -> None:
    check(lib.conv2d_run(plan, d_in, d_filter, d_out, stream), "conv2d_run")


def conv2d_destroy(plan: int) -> None:
    lib.conv2d_destroy(plan)


def conv2d_reference(s: Shape, d_in: int, d_filter: int, d_out: int, stream: int = 0) -> None:
    check(lib.conv2d_reference(s, d_in, d_filter, d_out, stream), "conv2d_reference")


def conv2d_fill_uniform(d_out: int, n: int, seed: int, start: int = 0, stream: int = 0) -> None:
    check(lib.conv2d_fill_uniform(d_out, n, seed, start, stream), "conv2d_fill_uniform")


def conv2d_tune_defaults() -> TuneOpts:
    o = TuneOpts()
    lib.conv2d_tune_defaults(ctypes.byref(o))
    return o


def conv2d_tune(s: Shape, opts: TuneOpts | None = None) -> TuneResult:
    r = TuneResult()
    check(lib.conv2d_tune(s, None if opts is None else ctypes.byref(opts), ctypes.byref(r)), "conv2d_tune")
    return r


def conv2d_tune_synthetic(s: Shape, cost, opts: TuneOpts | None = None) -> TuneResult:
    """``cost(config_tuple) -> ms`` (or a negative status) replaces the GPU."""
    def _cb(cp, _user):
        return float(cost(cp.contents.tuple()))
    cb = COST_FN(_cb)
    r = TuneResult()
    check(lib.conv2d_tune_synthetic(s, cb, None, None if opts is None else ctypes.byref(opts),
                                    ctypes.byref(r)), "conv2d_tune_synthetic")
    return r


def conv2d_benchmark(s: Shape, cfg, warmup: int = 2, reps: int = 20, flush_mall: int = 1):
    """(median_ms, min_ms) of one verified configuration."""
    med, mn = c_double(), c_double()
    check(lib.conv2d_benchmark(s, ctypes.byref(config(cfg)), warmup, reps, flush_mall, ctypes.byref(med),
                               ctypes.byref(mn)), "conv2d_benchmark")
    return med.value, mn.value


CONV2D_BATCH_NO_GRAPH, CONV2D_BATCH_NO_PTR_CHECK, CONV2D_BATCH_BY_SIZE = 1, 2, 4

for _name, (_res, _args) in {
    "conv2d_batch_plan": (c_int, [P(c_void_p), c_int, P(Shape), c_int]),
    "conv2d_batch_run": (c_int, [c_void_p, P(c_void_p), P(c_void_p), P(c_void_p), c_void_p]),
    "conv2d_batch_info": (c_int, [c_void_p, P(c_int), P(c_int), P(c_int), P(Config), P(c_int), c_int]),
    "conv2d_batch_destroy": (None, [c_void_p]),
    "conv2d_compile_batch": (c_int, [Shape, P(Config), c_char_p, c_int]),
    "conv2d_warm_cache": (c_int, [c_char_p, c_int, P(c_int), P(c_int)]),
}.items():
    _fn = getattr(lib, _name)
    _fn.restype, _fn.argtypes = _res, _args


def conv2d_batch_plan(shapes, flags: int = 0) -> int:
    arr = (Shape * len(shapes))(*[s if isinstance(s, Shape) else Shape(*s) for s in shapes])
    h = c_void_p()
    check(lib.conv2d_batch_plan(ctypes.byref(h), len(shapes), arr, flags), "conv2d_batch_plan")
    return h.value


def conv2d_batch_run(batch: int, d_in, d_f, d_out, stream: int = 0) -> None:
    n = len(d_in)
    a = (c_void_p * n)(*d_in)
    b = (c_void_p * n)(*d_f)
    c = (c_void_p * n)(*d_out)
    check(lib.conv2d_batch_run(batch, a, b, c, stream), "conv2d_batch_run")


def conv2d_batch_info(batch: int, cap: int = 64) -> dict:
    ng, tiles = c_int(), c_int()
    filt = (c_int * (2 * cap))()
    cfgs = (Config * cap)()
    grids = (c_int * cap)()
    check(lib.conv2d_batch_info(batch, ctypes.byref(ng), ctypes.byref(tiles), filt, cfgs, grids, cap),
          "conv2d_batch_info")
    groups = [{"filter": (filt[2 * g], filt[2 * g + 1]), "config": cfgs[g].tuple(), "grid": grids[g]}
              for g in range(min(ng.value, cap))]
    return {"n_groups": ng.value, "total_tiles": tiles.value, "groups": groups}


BATCH_TUNE_MAX = 32
SIZE_BUCKETS = 5


class BatchTuneOpts(ctypes.Structure):
    _fields_ = [("winners_path", c_char_p), ("results_dir", c_char_p), ("candidates", c_int), ("buckets", c_int),
                ("warmup", c_int), ("reps", c_int), ("tie_rel", c_double), ("verbose", c_int)]


class BatchTuneResult(ctypes.Structure):
    _fields_ = [("n_groups", c_int), ("filt", c_int * (2 * BATCH_TUNE_MAX)), ("bucket", c_int * BATCH_TUNE_MAX),
                ("n_problems", c_int * BATCH_TUNE_MAX), ("before", Config * BATCH_TUNE_MAX),
                ("after", Config * BATCH_TUNE_MAX), ("before_ms", c_double * BATCH_TUNE_MAX),
                ("after_ms", c_double * BATCH_TUNE_MAX), ("n_tried", c_int * BATCH_TUNE_MAX)]

    def groups(self):
        return [{"filter": (self.filt[2 * g], self.filt[2 * g + 1]), "bucket": self.bucket[g],
                 "problems": self.n_problems[g], "before": list(self.before[g].tuple()),
                 "before_ms": round(self.before_ms[g], 5), "after": list(self.after[g].tuple()),
                 "after_ms": round(self.after_ms[g], 5), "tried": self.n_tried[g]}
                for g in range(min(self.n_groups, BATCH_TUNE_MAX))]


lib.conv2d_batch_tune_defaults.restype = None
lib.conv2d_batch_tune_defaults.argtypes = [P(BatchTuneOpts)]
lib.conv2d_batch_tune.restype = c_int
lib.conv2d_batch_tune.argtypes = [c_int, P(Shape), P(BatchTuneOpts), P(BatchTuneResult)]


lib.conv2d_size_bucket.restype = c_int
lib.conv2d_size_bucket.argtypes = [c_int, c_int]


def conv2d_size_bucket(out_h: int, out_w: int) -> int:
    return int(lib.conv2d_size_bucket(int(out_h), int(out_w)))


def conv2d_batch_tune_defaults() -> BatchTuneOpts:
    o = BatchTuneOpts()
    lib.conv2d_batch_tune_defaults(ctypes.byref(o))
    return o


def conv2d_batch_tune(shapes, opts: BatchTuneOpts | None = None) -> BatchTuneResult:
    arr = (Shape * len(shapes))(*[shape(*s) for s in shapes])
    r = BatchTuneResult()
    check(lib.conv2d_batch_tune(len(shapes), arr, None if opts is None else ctypes.byref(opts), ctypes.byref(r)),
          "conv2d_batch_tune")
    return r


def conv2d_batch_destroy(batch: int) -> None:
    lib.conv2d_batch_destroy(batch)


def conv2d_warm_cache(manifest: str, threads: int = 0):
    """Compiles the manifest's programs missing from the code-object cache;
    returns (compiled, already cached)."""
    done, had = c_int(), c_int()
    check(lib.conv2d_warm_cache(manifest.encode(), threads, ctypes.byref(done), ctypes.byref(had)),
          "conv2d_warm_cache")
    return done.value, had.value


def conv2d_compile_batch(s: Shape, cfg) -> str:
    buf = ctypes.create_string_buffer(4096)
    check(lib.conv2d_compile_batch(s, ctypes.byref(config(cfg)), buf, 4096), "conv2d_compile_batch")
    return buf.value.decode()


class ServeOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", c_size_t), ("streams", c_int), ("max_batch", c_int), ("serial_plain", c_int),
                ("keep_outputs", c_int)]


class ServeReport(ctypes.Structure):
    _fields_ = [("n_requests", c_int), ("n_batches", c_int), ("wall_s", c_double), ("req_per_s", c_double),
                ("gflops", c_double), ("offered_rate", c_double), ("p50_ms", c_double), ("p99_ms", c_double),
                ("mean_ms", c_double), ("max_ms", c_double), ("queue_p50_ms", c_double),
                ("queue_p99_ms", c_double), ("mean_batch", c_double), ("stalled_requests", c_int),
                ("peak_bytes", c_size_t), ("late_start_ms", c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# numpy mirror of conv2d_request (40 bytes: double, 4 x int32, 2 x uint64)
REQUEST_DTYPE = [("arrival_s", "<f8"), ("out_h", "<i4"), ("out_w", "<i4"), ("filt_h", "<i4"), ("filt_w", "<i4"),
                 ("seed_in", "<u8"), ("seed_f", "<u8")]

for _name, (_res, _args) in {
    "conv2d_serve_defaults": (None, [P(ServeOpts)]),
    "conv2d_serve": (c_int, [c_void_p, c_int, P(ServeOpts), P(ServeReport), P(c_double), P(c_void_p)]),
    "conv2d_serve_free": (None, [P(c_void_p), c_int]),
}.items():
    _fn = getattr(lib, _name)
    _fn.restype, _fn.argtypes = _res, _args


def conv2d_serve_defaults() -> ServeOpts:
    o = ServeOpts()
    lib.conv2d_serve_defaults(ctypes.byref(o))
    return o


def requests_array(arrivals, shapes, seeds_in, seeds_f):
    import numpy as np
    a = np.zeros(len(arrivals), dtype=REQUEST_DTYPE)
    a["arrival_s"] = arrivals
    sh = np.asarray(shapes, dtype=np.int64).reshape(-1, 4)
    a["out_h"], a["out_w"], a["filt_h"], a["filt_w"] = sh[:, 0], sh[:, 1], sh[:, 2], sh[:, 3]
    a["seed_in"] = np.asarray(seeds_in, dtype=np.uint64)
    a["seed_f"] = np.asarray(seeds_f, dtype=np.uint64)
    assert a.dtype.itemsize == 40
    return a


def conv2d_serve(reqs, opts: ServeOpts | None = None, keep_outputs: bool = False):
    """reqs: numpy array of REQUEST_DTYPE. Returns (report, latencies_ms, outputs)
    where outputs is a list of device pointers (keep_outputs) or None."""
    import numpy as np
    reqs = np.ascontiguousarray(reqs)
    n = len(reqs)
    o = opts or conv2d_serve_defaults()
    o.keep_outputs = 1 if keep_outputs else 0
    rep = ServeReport()
    lat = np.zeros(n, np.float64)
    outs = (c_void_p * n)() if keep_outputs else None
    check(lib.conv2d_serve(reqs.ctypes.data, n, ctypes.byref(o), ctypes.byref(rep),
                           lat.ctypes.data_as(P(c_double)), outs), "conv2d_serve")
    return rep, lat, (list(outs) if keep_outputs else None)


def conv2d_serve_free(outputs) -> None:
    arr = (c_void_p * len(outputs))(*outputs)
    lib.conv2d_serve_free(arr, len(outputs))


# ---------------------------------------------------------------- hotspot stencil (hotspot.h)

class HotspotConfig(ctypes.Structure):
    _fields_ = [("block_x", c_int), ("block_y", c_int), ("tile_x", c_int), ("tile_y", c_int),
                ("temporal", c_int), ("unroll_t", c_int), ("sh_power", c_int)]

    def tuple(self):
        return tuple(getattr(self, f) for f, _ in self._fields_)

    def __repr__(self):
        return "HotspotConfig(" + ",".join(str(v) for v in self.tuple()) + ")"


class HotspotShape(ctypes.Structure):
    _fields_ = [("rows", c_int), ("cols", c_int)]


class HotspotCoeffs(ctypes.Structure):
    _fields_ = [("cc", ctypes.c_float), ("gx", ctypes.c_float), ("gy", ctypes.c_float), ("gz", ctypes.c_float),
                ("t_amb", ctypes.c_float)]


class HotspotTuneOpts(ctypes.Structure):
    _fields_ = [("winners_path", c_char_p), ("results_path", c_char_p), ("warmup", c_int), ("reps", c_int),
                ("retime_reps", c_int), ("flush_mall", c_int), ("threads", c_int), ("max_configs", c_int),
                ("tie_rel", c_double), ("verbose", c_int)]


class HotspotTuneResult(ctypes.Structure):
    _fields_ = [("best", HotspotConfig), ("best_ms", c_double), ("default_ms", c_double), ("median_ms", c_double),
                ("best_gflops", c_double), ("median_gflops", c_double), ("default_gflops", c_double),
                ("impact", c_double), ("n_space", c_int), ("n_illegal", c_int), ("n_compile_fail", c_int),
                ("n_launch_fail", c_int), ("n_verify_fail", c_int), ("n_timed", c_int), ("n_resumed", c_int),
                ("default_rank", c_int), ("top", HotspotConfig * 5), ("top_ms", c_double * 5),
                ("compile_s", c_double), ("measure_s", c_double),
                ("best_sweep_ms", c_double), ("default_sweep_ms", c_double)]


_HS_SIGS = {
    "hotspot_default_config": (None, [P(HotspotConfig)]),
    "hotspot_lds_bytes": (c_int, [P(HotspotConfig)]),
    "hotspot_config_check": (c_int, [HotspotShape, P(HotspotConfig), c_int]),
    "hotspot_space": (c_int, [HotspotShape, c_int, P(HotspotConfig), c_int]),
    "hotspot_compile": (c_int, [P(HotspotConfig), c_char_p, c_int]),
    "hotspot_plan": (c_int, [P(c_void_p), HotspotShape, P(HotspotConfig)]),
    "hotspot_plan_config": (c_int, [c_void_p, P(HotspotConfig), P(c_int)]),
    "hotspot_run": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, HotspotCoeffs, c_void_p]),
    "hotspot_run_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, HotspotCoeffs, c_void_p]),
    "hotspot_destroy": (None, [c_void_p]),
    "hotspot_reference": (c_int, [HotspotShape, c_void_p, c_void_p, c_void_p, c_void_p, c_int, HotspotCoeffs,
                                  c_void_p]),
    "hotspot_tune_defaults": (None, [P(HotspotTuneOpts)]),
    "hotspot_tune": (c_int, [HotspotShape, c_int, P(HotspotTuneOpts), P(HotspotTuneResult)]),
}
for _name, (_res, _args) in _HS_SIGS.items():
    _fn = getattr(lib, _name)
    _fn.restype, _fn.argtypes = _res, _args


def hotspot_config(*vals) -> HotspotConfig:
    if len(vals) == 1 and isinstance(vals[0], (tuple, list, HotspotConfig)):
        vals = tuple(vals[0].tuple() if isinstance(vals[0], HotspotConfig) else vals[0])
    return HotspotConfig(*[int(v) for v in vals])


def hotspot_shape(rows, cols) -> HotspotShape:
    return HotspotShape(int(rows), int(cols))


def hotspot_coeffs(cc, gx, gy, gz, t_amb) -> HotspotCoeffs:
    return HotspotCoeffs(float(cc), float(gx), float(gy), float(gz), float(t_amb))


def hotspot_default_config() -> HotspotConfig:
    c = HotspotConfig()
    lib.hotspot_default_config(ctypes.byref(c))
    return c


def hotspot_lds_bytes(cfg) -> int:
    return check(lib.hotspot_lds_bytes(ctypes.byref(hotspot_config(cfg))), "hotspot_lds_bytes")


def hotspot_config_check(s: HotspotShape, cfg, lds_limit: int = 0) -> int:
    return lib.hotspot_config_check(s, ctypes.byref(hotspot_config(cfg)), lds_limit)


def hotspot_space(s: HotspotShape, lds_limit: int = 0):
    n = check(lib.hotspot_space(s, lds_limit, None, 0), "hotspot_space")
    arr = (HotspotConfig * max(n, 1))()
    lib.hotspot_space(s, lds_limit, arr, n)
    return [arr[k].tuple() for k in range(n)]


def hotspot_compile(cfg) -> str:
    buf = ctypes.create_string_buffer(4096)
    check(lib.hotspot_compile(ctypes.byref(hotspot_config(cfg)), buf, 4096), "hotspot_compile")
    return buf.value.decode()


def hotspot_plan(s: HotspotShape, cfg=None) -> int:
    h = c_void_p()
    check(lib.hotspot_plan(ctypes.byref(h), s, None if cfg is None else ctypes.byref(hotspot_config(cfg))),
          "hotspot_plan")
    return h.value


def hotspot_plan_config(plan: int):
    c, tuned = HotspotConfig(), c_int()
    check(lib.hotspot_plan_config(plan, ctypes.byref(c), ctypes.byref(tuned)), "hotspot_plan_config")
    return c.tuple(), tuned.value


def hotspot_run(plan: int, d_temp: int, d_power: int, d_out: int, d_work, steps: int, k: HotspotCoeffs,
                stream: int = 0) -> None:
    check(lib.hotspot_run(plan, d_temp, d_power, d_out, d_work, int(steps), k, stream), "hotspot_run")


HOTSPOT_NOALLOC_CELLS = 4096 * 4096


def hotspot_run_noalloc(plan: int, d_temp: int, d_power: int, d_out: int, steps: int, k: HotspotCoeffs,
                        stream: int = 0) -> None:
    """hotspot_run with the library's fixed work grid: allocates nothing."""
    check(lib.hotspot_run_noalloc(plan, d_temp, d_power, d_out, int(steps), k, stream), "hotspot_run_noalloc")


def hotspot_destroy(plan: int) -> None:
    lib.hotspot_destroy(plan)


def hotspot_reference(s: HotspotShape, d_temp: int, d_power: int, d_out: int, d_work, steps: int,
                      k: HotspotCoeffs, stream: int = 0) -> None:
    check(lib.hotspot_reference(s, d_temp, d_power, d_out, d_work, int(steps), k, stream), "hotspot_reference")


lib.hotspot_kernel_hash.restype = c_char_p
lib.hotspot_kernel_hash.argtypes = []


def hotspot_kernel_hash() -> str:
    return lib.hotspot_kernel_hash().decode()


def hotspot_tune_defaults() -> HotspotTuneOpts:
    o = HotspotTuneOpts()
    lib.hotspot_tune_defaults(ctypes.byref(o))
    return o


def hotspot_tune(s: HotspotShape, steps: int, opts: HotspotTuneOpts | None = None) -> HotspotTuneResult:
    r = HotspotTuneResult()
    check(lib.hotspot_tune(s, int(steps), None if opts is None else ctypes.byref(opts), ctypes.byref(r)),
          "hotspot_tune")
    return r
