"""Pin of the compiled CPU baseline (oracle/csr_rk4.c): its RK4 loop on the
oracle's generator equals oracle/integrate.py's classical RK4 step for step
(to rounding of the summation order), on one thread and on several."""
import shutil

import numpy as np
import pytest

from oracle import cpu_timer, integrate, uvar
from paper_2608_20657_amd import workloads as W


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_compiled_rk4_matches_oracle_integrator(tmp_path):
    exe = cpu_timer.build_timer(str(tmp_path))
    p = W.random_problem(6, 2, 3, 1, seed=4, loss=True, terminator=True)
    S = uvar.UVarSystem(p)
    A = S.generator()
    y0 = W.random_vector(S.n_var, 3)
    want = y0.copy()
    for _ in range(7):
        want = integrate.rk4_step(A, want, 0.05)
    for threads in (1, 3):
        got, info = cpu_timer.run_rk4(exe, A, y0, 0.05, 7, threads)
        assert info["threads"] == threads and info["n"] == S.n_var and info["steps"] == 7
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
