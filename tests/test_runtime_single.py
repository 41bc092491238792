"""Importing the package before torch leaves one HIP runtime in the process.

torch ships its own HIP runtime; the package loads torch before its library, so
the library binds to that runtime instead of pulling in a second copy (with two,
the library's device calls and torch's tensors and streams would belong to
different runtimes)."""
import subprocess
import sys

CODE = """
import paper_1204_0556_amd, torch
libs = sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l})
print(len(libs))
"""


def test_package_first_loads_one_hip_runtime():
    r = subprocess.run([sys.executable, "-c", CODE], capture_output=True, text=True, timeout=300,
                       cwd=__file__.rsplit("/tests/", 1)[0])
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == "1"
