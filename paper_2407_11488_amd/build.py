"""Builds libconv2d.so in-tree for gfx950.

Host sources (*.cpp) are compiled with amdclang++ as plain C++ against the HIP
headers; device sources (*.hip) with hipcc for gfx950. Packed FP32
instructions are disabled in every device compilation. Run it as a script
(importing the package would load the library before it is built):

    python paper_2407_11488_amd/build.py [--warm]

With --warm it then fills the run-time code-object cache (`_cache/` beside
the library) with every program listed in `code_objects.txt` (the programs
that the GPU tests, the smoke check and the benchmark load), compiling on
the host's cores, so that those runs compile nothing on the GPU machine.
Regenerate the list by running them with CONV2D_COMPILE_LOG=<file> set.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build", "conv2d")
LIB = os.path.join(PKG, "libconv2d.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = os.environ.get("CONV2D_BUILD_ARCH", "gfx950")

HIPCC = os.path.join(ROCM, "bin", "hipcc")
CXX = os.path.join(ROCM, "llvm", "bin", "clang++")
NO_PACKED_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Kernel sources the library compiles at run time with hiprtc (embedded into
# it), not at build time.
RUNTIME_SOURCES = {"conv2d_direct.hip", "hotspot.hip"}
COMMON = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter",
          f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]


def _sources():
    cpp = sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp"))
    hip = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip") and f not in RUNTIME_SOURCES)
    return cpp, hip


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".cpp"):
        cmd = [CXX, "-x", "c++", *COMMON, "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", "-c", path, "-o", obj]
    else:
        cmd = [HIPCC, f"--offload-arch={ARCH}", *COMMON, *NO_PACKED_FP32, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def _check_direct_kernel():
    """Compiles the run-time-compiled kernel sources through the library's own
    hiprtc path (no GPU needed), each for two configurations, so that an error
    in a kernel source fails the build."""
    import ctypes

    class Shape(ctypes.Structure):
        _fields_ = [(n, ctypes.c_int) for n in ("out_h", "out_w", "filt_h", "filt_w")]

    class Config(ctypes.Structure):
        _fields_ = [(n, ctypes.c_int) for n in ("block_x", "block_y", "tile_x", "tile_y", "use_lds",
                                                 "filter_in_const", "unroll")]

    class HotspotConfig(ctypes.Structure):
        _fields_ = [(n, ctypes.c_int) for n in ("block_x", "block_y", "tile_x", "tile_y", "temporal",
                                                 "unroll_t", "sh_power")]

    try:
        import torch  # noqa: F401  (bind torch's HIP runtime, as the package does)
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB)
    lib.conv2d_last_error.restype = ctypes.c_char_p
    for cfg, vin, vout in (((16, 16, 1, 1, 1, 1, 1), 4, 4), ((64, 1, 8, 8, 0, 0, 1), 1, 2)):
        rc = lib.conv2d_compile(Shape(64, 64, 17, 17), ctypes.byref(Config(*cfg)), vin, vout, None, 0)
        if rc != 0:
            raise RuntimeError(f"kernel source check failed for {cfg}: {lib.conv2d_last_error().decode()}")
    for cfg in ((32, 8, 1, 1, 1, 1, 1), (64, 4, 2, 4, 4, 0, 0)):
        rc = lib.hotspot_compile(ctypes.byref(HotspotConfig(*cfg)), None, 0)
        if rc != 0:
            raise RuntimeError(f"hotspot source check failed for {cfg}: {lib.conv2d_last_error().decode()}")


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cpp, hip = _sources()
    jobs = min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, cpp + hip))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp,
           f"-L{ROCM}/lib", "-lhiprtc", "-lamdhip64", "-lpthread", "-ldl", f"-Wl,-rpath,{ROCM}/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, LIB)
    _check_direct_kernel()
    if verbose:
        print(f"built {LIB}")
    return LIB


MANIFEST = os.path.join(PKG, "code_objects.txt")


def warm(manifest: str = MANIFEST, threads: int = 0, verbose: bool = False):
    """Compiles every program of `manifest` that the code-object cache lacks
    (conv2d_warm_cache, no GPU needed). Returns (compiled, already cached)."""
    import ctypes
    try:
        import torch  # noqa: F401  (bind torch's HIP runtime, as the package does)
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB)
    lib.conv2d_last_error.restype = ctypes.c_char_p
    lib.conv2d_warm_cache.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_int)]
    done, had = ctypes.c_int(), ctypes.c_int()
    rc = lib.conv2d_warm_cache(manifest.encode(), threads, ctypes.byref(done), ctypes.byref(had))
    if rc != 0:
        raise RuntimeError(f"cache warm-up failed: {lib.conv2d_last_error().decode()}")
    if verbose:
        print(f"code-object cache: {done.value} compiled, {had.value} already present")
    return done.value, had.value


def clean():
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    build(verbose=True)
    if "--warm" in sys.argv[1:]:
        warm(verbose=True)
    sys.exit(0)
