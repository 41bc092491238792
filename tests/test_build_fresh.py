"""build() on a fresh checkout: no built library in the tree.

The package refuses to import without its library (there is no CPU fallback), so
the build entry point must compile before anything imports the package.  This
copies the sources that build() needs (the package, the header, the oracle and the
build entry point; no shared objects or objects) to a temporary directory and runs
build() there in a fresh interpreter."""
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_build_from_a_tree_without_libraries(tmp_path):
    dst = tmp_path / "repo"
    dst.mkdir()
    skip = shutil.ignore_patterns("*.so", "*.o", "__pycache__")
    for d in ("paper_1204_0556_amd", "include", "oracle"):
        shutil.copytree(os.path.join(ROOT, d), dst / d, ignore=skip)
    shutil.copy2(os.path.join(ROOT, "__graft_entry__.py"), dst / "__graft_entry__.py")
    assert not (dst / "paper_1204_0556_amd" / "liblpdec.so").exists()
    r = subprocess.run([sys.executable, "-c", "import __graft_entry__ as g; g.build()"], cwd=dst,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    assert (dst / "paper_1204_0556_amd" / "liblpdec.so").exists()
    assert (dst / "oracle" / "liblpdec_oracle.so").exists()
