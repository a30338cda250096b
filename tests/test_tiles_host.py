"""Host-side checks of the workgroup tiles (plain, transposed targets,
compact): a C++ checker compiled against the table builder, no GPU."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_tiles_bounds_coverage_and_transposed_targets():
    src = os.path.join(ROOT, "tests", "native", "tile_check.cpp")
    tables = os.path.join(ROOT, "paper_2608_20657_amd", "csrc", "tables.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "tile_check")
        subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                        "-I", os.path.join(ROOT, "paper_2608_20657_amd", "csrc"), src, tables, "-o", exe],
                       check=True, capture_output=True, text=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
