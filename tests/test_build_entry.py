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
