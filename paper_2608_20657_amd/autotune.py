"""Launch-configuration autotuner for heom_propagate.

Times a few RK4 steps of the caller's problem for each candidate launch
configuration (workgroup tile size, persistent cooperative kernel or one
launch per stage, XCD-contiguous tile mapping) with HIP events on the launch
stream, and leaves the fastest one set on the tables. Every configuration
computes bitwise identical results (one writer per output element and a fixed
summation order per element), so tuning never changes numerics.
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Optional

from . import heom


def candidates(T: "heom.Tables", tiles=(64, 128, 256, 512), persistent=(0, 1), xcd=(1, 0)) -> List[Dict]:
    maxblk = T.max_block()
    out = []
    for tv, pe, xm in itertools.product(tiles, persistent, xcd):
        if tv < maxblk:
            continue
        out.append(dict(tile_vars=tv, persistent=pe, xcd_map=xm))
    return out


def autotune(T: "heom.Tables", torch, tier0, dt: float, steps: int = 40, precision: int = heom.HEOM_FP64,
             cands: Optional[List[Dict]] = None, repeats: int = 2, verbose: bool = False) -> Dict:
    """Pick the fastest launch configuration for propagating this problem.
    Returns {"best": config, "ms_per_step": t, "results": [(config, t), ...]}.
    The tables are left uploaded with the best configuration (T.image)."""
    s = torch.cuda.current_stream()
    cands = cands or candidates(T)
    info = T.info()
    y = torch.empty(info["n_var"], dtype=torch.complex128, device="cuda")
    results = []
    for c in cands:
        T.set_tuning(**c)
        img = torch.empty(T.info()["table_bytes"], dtype=torch.uint8, device="cuda")
        T.upload(img, s)
        wb = T.info()["work_bytes_fp64" if precision == heom.HEOM_FP64 else "work_bytes_fp32"]
        work = torch.empty(wb, dtype=torch.uint8, device="cuda")
        best = float("inf")
        for r in range(repeats + 1):
            T.init_state(tier0, y, s)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            T.propagate(y, work, dt, steps, 0, None, precision, s)
            e1.record(s)
            torch.cuda.synchronize()
            T.work_status(work, s)
            if r > 0:                       # the first run warms up
                best = min(best, e0.elapsed_time(e1) / steps)
        results.append((dict(c), best))
        if verbose:
            print(f"autotune {c}: {best * 1e3:.2f} us/step", flush=True)
    cbest, tbest = min(results, key=lambda x: x[1])
    T.set_tuning(**cbest)
    img = torch.empty(T.info()["table_bytes"], dtype=torch.uint8, device="cuda")
    T.upload(img, s)
    return {"best": cbest, "ms_per_step": tbest, "results": results}
