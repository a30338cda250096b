"""Host-side checks of the workgroup tiles (plain, transposed targets,
compact): a C++ checker compiled against the table builder, no GPU. It runs
fixed structures and a seeded sweep over small random ones, once as an
optimized build and once under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only: the checker and the table builder, compiled with g++), so
that the builder's index packing (7-bit pattern and 5-bit category fields of
the decode records, 2^32 gather limit, record-slot resizing of compact tiles)
is exercised with bounds and overflow checks on.

A second test draws small structures (N, m, L, d) from a seed and compares
heom_export_layout with the oracle's tables entry by entry."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "tile_check.cpp")
TABLES = os.path.join(ROOT, "paper_2608_20657_amd", "csrc", "tables.cpp")
INC = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2608_20657_amd", "csrc")]
SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=undefined"]


def _run_checker(flags, seed, count, timeout):
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "tile_check")
        subprocess.run(["g++", "-std=c++17", "-ffp-contract=off"] + flags + INC + [SRC, TABLES, "-o", exe],
                       check=True, capture_output=True, text=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        return subprocess.run([exe, str(seed), str(count)], capture_output=True, text=True, timeout=timeout, env=env)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_tiles_bounds_coverage_and_transposed_targets():
    r = _run_checker(["-O2"], seed=1, count=60, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_tiles_under_address_and_ub_sanitizers():
    r = _run_checker(SANITIZE, seed=2, count=25, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]


def test_layout_fuzz_small_structures():
    heom = pytest.importorskip("paper_2608_20657_amd.heom", reason="libheom.so not built")
    from oracle import uvar
    from paper_2608_20657_amd import workloads as W
    from tests.oracle_layout import serialize
    rng = np.random.default_rng(2026)
    for _ in range(40):
        N = int(rng.integers(1, 9))
        m = int(rng.integers(1, 4))
        L = int(rng.integers(0, 6 if m < 3 else 5))
        d = int(rng.integers(0, min(N, 2) + 1))
        p = W.random_problem(N, m, L, d, seed=int(rng.integers(1 << 30)), complex_check=bool(rng.integers(2)))
        lib = heom.Tables(p).export_layout()
        ora = serialize(uvar.UVarSystem(p))
        assert lib.shape == ora.shape and np.array_equal(lib, ora), (N, m, L, d)
