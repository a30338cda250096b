"""Write the oracle's reference trajectories for the GPU parity tests.

Calls only the oracle (and the shared input generators): classical RK4 on
the oracle's unique-variable generator, observables of the tier-0 block every
`every` steps, written as JSON text with full double precision.

    python tests/golden/make_golden.py [name ...]

Workloads:
  localized -- N=64, m=2, L=6, d=1, rho(0)=|e_1><e_1|, dt=0.02, 10000 steps
  saturated -- N=10^4, m=3, L=8, rho(0)=|+><+|, dt=0.02, 10000 steps
  paper_n5_up -- the paper's L=25 single-exponential workload (Sec. VII.A,
      rad/fs units) at N=5, upper-polariton start, dt=0.5 fs, 400 steps
  paper_n3_superposition -- the same at N=3 with one distinguished molecule,
      rho(0) from sqrt(0.3)|e_1> + sqrt(0.7)|c>, dt=0.5 fs, 400 steps
  paper_static_n3_up -- the paper's static-disorder workload (Drude-Lorentz +
      a zero-rate channel, m=2, L=14) at N=3, upper-polariton start,
      dt=0.5 fs, 400 steps
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import integrate, observables, uvar  # noqa: E402
from paper_2608_20657_amd import workloads as W  # noqa: E402

RUNS = {
    "localized": dict(dt=0.02, steps=10000, every=100, state="site1"),
    "saturated": dict(dt=0.02, steps=10000, every=100, state="upper_polariton"),
    "paper_n5_up": dict(dt=W.PAPER_SHAPE_DT, steps=400, every=20, state="upper_polariton",
                        problem=lambda: W.config_paper_shape(5, 0)),
    "paper_n3_superposition": dict(dt=W.PAPER_SHAPE_DT, steps=400, every=20, state="site1_cavity",
                                   problem=lambda: W.config_paper_shape(3, 1)),
    "paper_static_n3_up": dict(dt=W.PAPER_SHAPE_DT, steps=400, every=20, state="upper_polariton",
                               problem=lambda: W.config_paper_static(3, 0)),
}


def amplitude(p, state):
    if state == "site1":
        return lambda i: 1.0 if i == 1 else 0.0
    if state == "photon":
        return lambda i: 1.0 if i == 0 else 0.0
    if state == "site1_cavity":
        return lambda i: math.sqrt(0.7) if i == 0 else (math.sqrt(0.3) if i == 1 else 0.0)
    if state == "upper_polariton":
        th = observables.theta(p.N, p.eps, p.omega_c, p.g)
        return lambda i: math.cos(th) if i == 0 else math.sin(th) / math.sqrt(p.N)
    raise ValueError(state)


def make(name):
    run = RUNS[name]
    p = run["problem"]() if "problem" in run else W.WORKLOADS[name]()
    t0 = time.time()
    S = uvar.UVarSystem(p)
    A = S.generator()
    y0 = S.initial_state(amp=amplitude(p, run["state"]))
    _, obs = integrate.propagate(A, y0, run["dt"], run["steps"], run["every"],
                                 observe=lambda y: observables.from_tier0(S, y))
    out = dict(workload=name, source="oracle: classical RK4 on the unique-variable generator",
               dt=run["dt"], steps=run["steps"], every=run["every"], state=run["state"],
               n_var=S.n_var, observables=[[float(x) for x in o] for o in obs])
    with open(os.path.join(HERE, f"traj_{name}.json"), "w") as f:
        json.dump(out, f)
    print(name, S.n_var, f"{time.time() - t0:.1f}s", flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(RUNS)):
        make(name)
