"""build() works from a tree that holds sources only (no prebuilt libraries): the build scripts
are loaded by path, so the package's __init__ (which needs libhcc.so) is not imported before
the library exists."""
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_build_from_sources_only(tmp_path):
    ignore = shutil.ignore_patterns("*.so", "*.so.tmp*", "_build", "__pycache__", "*.o")
    for d in ("paper_2305_16652_amd", "oracle", "include", "workloads"):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d, ignore=ignore)
    shutil.copy(os.path.join(ROOT, "__graft_entry__.py"), tmp_path)
    assert not list(tmp_path.rglob("*.so"))
    r = subprocess.run([sys.executable, "-c", "import __graft_entry__ as g; g.build()"], cwd=tmp_path,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    assert (tmp_path / "paper_2305_16652_amd" / "libhcc.so").exists()
    assert (tmp_path / "oracle" / "liboracle.so").exists()
