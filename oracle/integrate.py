"""Classical fourth-order Runge-Kutta (oracle; test infrastructure only).

The paper propagates with a conventional RK4 (Sec. VII.E, remark on work
arrays). For the autonomous linear system dy/dt = A y one step is
    k1 = A y, k2 = A(y + h/2 k1), k3 = A(y + h/2 k2), k4 = A(y + h k3),
    y <- y + h/6 (k1 + 2 k2 + 2 k3 + k4).

Parity: pinned by tests/test_oracle_conventional.py (one step equals the
degree-4 Taylor polynomial of exp(hA); a scalar decay matches the closed form
of the RK4 amplification factor).
"""
from __future__ import annotations

from typing import Callable, List, Optional

import numpy as np


def rk4_step(A, y: np.ndarray, h: float) -> np.ndarray:
    k1 = A @ y
    k2 = A @ (y + 0.5 * h * k1)
    k3 = A @ (y + 0.5 * h * k2)
    k4 = A @ (y + h * k3)
    return y + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def propagate(A, y0: np.ndarray, h: float, nsteps: int, every: int = 1,
              observe: Optional[Callable[[np.ndarray], np.ndarray]] = None):
    """Run nsteps RK4 steps. Returns (final y, list of observe(y) taken at
    step 0 and after every `every` steps)."""
    y = np.array(y0, dtype=np.complex128, copy=True)
    obs: List[np.ndarray] = []
    if observe is not None:
        obs.append(observe(y))
    for s in range(1, nsteps + 1):
        y = rk4_step(A, y, h)
        if observe is not None and s % every == 0:
            obs.append(observe(y))
    return y, obs
