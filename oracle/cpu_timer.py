"""Timed CPU baseline: the oracle's generator run by a compiled RK4 loop
(oracle; test infrastructure only: used by the tests and by the benchmark's
CPU-baseline leg, never by the product).

`build_timer` compiles oracle/csr_rk4.c (plain C, OpenMP, -O3 -march=native
for the host it runs on); `run_rk4` exports one problem's CSR generator M_u
(oracle.uvar, Eq. uvar-propagator) and initial state, runs classical RK4 for
a number of steps on a given number of threads, and returns the final state
with the loop's wall time. The C loop is the same classical RK4 as
oracle/integrate.py (Sec. VII.E); tests/test_cpu_timer.py pins it against
that, step for step.
"""
from __future__ import annotations

import json
import os
import shutil
import subprocess
import tempfile
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csr_rk4.c")


def build_timer(out_dir: Optional[str] = None) -> str:
    """Compile the timer (into out_dir, default oracle/_build) for this host."""
    out_dir = out_dir or os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    exe = os.path.join(out_dir, "csr_rk4")
    cc = shutil.which("gcc") or "cc"
    subprocess.run([cc, "-O3", "-march=native", "-fopenmp", "-std=c11", SRC, "-o", exe, "-lm"], check=True,
                   capture_output=True, text=True)
    return exe


def run_rk4(exe: str, A, y0: np.ndarray, h: float, steps: int, threads: int):
    """Classical RK4 steps of dy/dt = A y from y0 by the compiled timer.
    Returns (final y, dict with seconds, threads used, n, nnz)."""
    A = A.tocsr()
    A.sort_indices()
    with tempfile.TemporaryDirectory() as d:
        np.array([A.shape[0], A.nnz], dtype=np.int64).tofile(os.path.join(d, "n_nnz.i64"))
        A.indptr.astype(np.int64).tofile(os.path.join(d, "indptr.i64"))
        A.indices.astype(np.int64).tofile(os.path.join(d, "indices.i64"))
        A.data.astype(np.complex128).tofile(os.path.join(d, "data.c128"))
        np.ascontiguousarray(y0, dtype=np.complex128).tofile(os.path.join(d, "y0.c128"))
        r = subprocess.run([exe, d, str(int(steps)), repr(float(h)), str(int(threads))], check=True,
                           capture_output=True, text=True)
        y = np.fromfile(os.path.join(d, "y.c128"), dtype=np.complex128)
    return y, json.loads(r.stdout.strip().splitlines()[-1])
