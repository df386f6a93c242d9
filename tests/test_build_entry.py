"""The build entry point's order of loading: the build-time kernel-source check
loads the library before the package is imported, and the package must still
import in the same process (one HIP runtime mapped). Runs in a fresh process."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = """
import sys
sys.path.insert(0, {root!r})
import __graft_entry__ as g
g._load_builder()._check_direct_kernel()
import paper_2407_11488_amd as C
print("ok", C.conv2d_kernel_hash())
"""


def test_kernel_check_then_package_import_in_one_process():
    r = subprocess.run([sys.executable, "-c", SCRIPT.format(root=ROOT)], capture_output=True, text=True,
                       timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.startswith("ok ")


def test_package_refuses_to_load_without_the_hip_library(tmp_path):
    """No CPU fallback: the package without its built HIP library raises on
    import, naming the missing library and how to build it."""
    import shutil
    pkg = os.path.join(ROOT, "paper_2407_11488_amd")
    dst = tmp_path / "paper_2407_11488_amd"
    dst.mkdir()
    for name in os.listdir(pkg):
        if name.endswith(".py"):
            shutil.copy(os.path.join(pkg, name), dst / name)
    code = "import sys; sys.path.insert(0, {!r}); import paper_2407_11488_amd".format(str(tmp_path))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, cwd=str(tmp_path))
    assert r.returncode != 0
    assert "libconv2d.so is missing" in r.stderr
