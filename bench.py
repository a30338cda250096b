#!/usr/bin/env python3
"""Benchmark of the symmetry-adapted HEOM hot path on one MI355X.

One step = one classical RK4 step of the whole hot path (four fused
right-hand-side + combination stages over every unique variable, with the
tier-0 observables every `--obs-every` steps) on the localized workload:
N=64 molecules, m=2 (Debye + one Matsubara term, lam=0.02, gam=0.1,
kT=0.025), L=6, one distinguished molecule (rho(0)=|e_1><e_1|), g=0.01,
eps-omega_c=0.01, kappa=0.005, dt=0.02: 21,105 unique variables. Tables are
built and uploaded before the timed region (the paper's precomputation);
inputs are resident in HBM when timing starts.

Metric: unique-variable RHS updates/s = n_var * 4 * steps / time.

Also reported on the same JSON line:
  roofline      -- the RK4 stage kernel at the largest single-GPU structure
                   (N=10^4, m=4, L=10: 17.3 M variables, 278 MB per FP64
                   vector, above the 256 MB last-level cache): algorithmic
                   bytes per launch / mean launch time from HIP events on the
                   launch stream, against the 8 TB/s HBM peak;
  roofline_main -- the same quantity for the localized workload (its state
                   is cache resident, so it is latency bound, not HBM bound);
  cpu_baseline  -- the CPU oracle (classical RK4 with its sparse generator)
                   on a bounded sample of the same workload, one host core.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_stage_fp64_roofline_probe.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2608_20657_amd", "csrc", "device.hip")


def stage_bytes_per_var(precision: int):
    """Algorithmic state bytes per unique variable, summed over the four
    stages of one RK4 step (each value read or written once; hierarchy
    gathers are reads of values another workgroup also streams, counted
    once):
      FP64: stage 1 reads y, writes w1 (32); stages 2-4 read w, y, write
            w or y (48 each)                                   -> 176
      FP32: stage 1 reads y, writes u1 (24); 2 reads u1 writes u2 (16);
            3 reads u1, u2 writes u3 (24); 4 reads y, u3 writes y' (40) -> 104
    """
    return 176 if precision == 0 else 104


def sha256(path):
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def load_traffic():
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    try:
        rec = json.load(open(PROFILE_TRAFFIC))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != sha256(KERNEL_SRC):
        return None          # kernel changed since the counters were taken
    return rec


def run_solve(T, torch, tier0, dt, steps, obs_every, precision):
    info = T.info()
    s = torch.cuda.current_stream()
    y = torch.empty(info["n_var"], dtype=torch.complex128, device="cuda")
    wb = info["work_bytes_fp64"] if precision == 0 else info["work_bytes_fp32"]
    work = torch.empty(wb, dtype=torch.uint8, device="cuda")
    nobs = steps // obs_every + 1 if obs_every else 1
    obs = torch.zeros(nobs * 10, dtype=torch.float64, device="cuda")
    return y, work, obs, s


def time_propagate(T, torch, tier0, dt, steps, warmup, obs_every, precision):
    """Warm up, then time `steps` RK4 steps from rho(0) with HIP events on the
    launch stream (and wall clock, both bracketed by device syncs)."""
    y, work, obs, s = run_solve(T, torch, tier0, dt, max(steps, warmup), obs_every, precision)
    if warmup:
        T.init_state(tier0, y, s)
        T.propagate(y, work, dt, warmup, obs_every, obs if obs_every else None, precision, s)
        torch.cuda.synchronize()
    T.init_state(tier0, y, s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record(s)
    T.propagate(y, work, dt, steps, obs_every, obs if obs_every else None, precision, s)
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1)
    return ms, wall, y, obs


def cpu_baseline(p, tier0_amp, dt, budget_s):
    """The oracle as it stands (classical RK4 on its sparse generator) on the
    same workload, for as many steps as fit in about budget_s seconds."""
    from oracle import integrate, uvar
    S = uvar.UVarSystem(p)
    A = S.generator()
    y = S.initial_state(amp=tier0_amp)
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        for _ in range(10):
            y = integrate.rk4_step(A, y, dt)
        steps += 10
    el = time.perf_counter() - t0
    return dict(value=S.n_var * 4 * steps / el, unit="unique-variable RHS updates/s", cores=1,
                kind="oracle",
                sample=f"localized workload, first {steps} RK4 steps ({el:.1f} s) of classical RK4 "
                       f"with the oracle's scipy CSR generator ({A.nnz} nonzeros), one thread",
                seconds=round(el, 2), steps=steps)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--obs-every", type=int, default=100)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--roofline-steps", type=int, default=25)
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--roofline-only", action="store_true",
                    help="skip the localized solve (for profiling the roofline kernel alone)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="also run a plain device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus must be 1 "
              "(independent problems shard across GPUs without exchange, see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_2608_20657_amd import heom, workloads as W

    precision = 0 if args.precision == "fp64" else 1
    if args.calibrate_copy_mb:
        nb = args.calibrate_copy_mb << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": nb, "copies": 3}), flush=True)
        del src, dst
    if args.roofline_only:
        args.no_cpu_baseline = True
    p = W.config_localized()
    dt = 0.02
    T = heom.Tables(p)
    tier0 = T.tier0_pure(0.0, 0.0, [1.0])
    tuned = None
    if not args.roofline_only and not args.no_autotune:
        # pick the launch configuration (results are identical for all of them)
        from paper_2608_20657_amd import autotune
        cands = [dict(tile_vars=tv, persistent=0, xcd_map=0, cache_policy=6) for tv in (64, 128, 256)]
        tuned = autotune.autotune(T, torch, tier0, dt, steps=200, precision=precision, cands=cands)
    else:
        img = torch.empty(T.info()["table_bytes"], dtype=torch.uint8, device="cuda")
        T.upload(img, torch.cuda.current_stream())
    info = T.info()
    if args.roofline_only:
        args.steps, args.warmup = 1, 0
    ms, wall, y, obs = time_propagate(T, torch, tier0, dt, args.steps, args.warmup, args.obs_every, precision)
    n = info["n_var"]
    updates = n * 4 * args.steps
    value = updates / (ms / 1e3)
    ob = obs.cpu().numpy().reshape(-1, 10)
    finite = bool(torch.isfinite(y).all().item()) and bool(math.isfinite(float(ob[-1, 0])))

    per_launch_ms = ms / (4 * args.steps)
    bpv = stage_bytes_per_var(precision) / 4.0
    main_bytes = n * bpv + info["table_bytes"]
    roof_main = dict(kernel="stage_kernel (RK4 stage: RHS + combination)", workload="localized",
                     bound="latency", achieved=round(main_bytes / (per_launch_ms * 1e-3) / 1e9, 1),
                     unit="GB/s", mean_launch_us=round(per_launch_ms * 1e3, 3),
                     note="21,105-variable state is cache resident; launch and gather latency bound")

    out = {
        "metric": "unique-variable RHS updates/s",
        "value": value,
        "unit": "unique-variable RHS updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == 0 else "f32-increments/f64-state",
        "data": "synthetic",
        "config": {"workload": "localized: N=64, m=2 (Debye + 1 Matsubara, lam=0.02, gam=0.1, kT=0.025), "
                               "L=6, d=1, g=0.01, eps-omega_c=0.01, kappa=0.005, rho(0)=|e_1><e_1|, dt=0.02",
                   "n_var": n, "patterns": info["n_patterns"], "rhs_per_step": 4,
                   "obs_every": args.obs_every, "precision": args.precision,
                   "parallelism": "single GPU"},
        "wall_s": round(wall, 4),
        "finite": finite,
        "final_observables": [float(x) for x in ob[-1]],
        "roofline_main": roof_main,
        "launch_config": T.tuning(),
        "autotune_us_per_step": {str(c["tile_vars"]): round(t * 1e3, 2) for c, t in tuned["results"]} if tuned else None,
    }

    if not args.no_roofline:
        q = W.config_roofline_probe()
        t0 = time.perf_counter()
        TR = heom.Tables(q)
        build_s = time.perf_counter() - t0
        ri = TR.info()
        img2 = torch.empty(ri["table_bytes"], dtype=torch.uint8, device="cuda")
        TR.upload(img2, torch.cuda.current_stream())
        t0r = TR.tier0_pure(1.0, 0.0, [])
        rms, _, ry, _ = time_propagate(TR, torch, t0r, dt, args.roofline_steps, 3, 0, 0)
        launch_ms = rms / (4 * args.roofline_steps)
        bytes_launch = ri["n_var"] * stage_bytes_per_var(0) / 4.0 + ri["table_bytes"]
        achieved = bytes_launch / (launch_ms * 1e-3) / 1e9
        traffic = load_traffic()
        out["roofline"] = {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic["bytes_per_launch"] if traffic else None,
            "kernel": "stage_kernel, FP64 RK4 stage (RHS + combination); one stage = the lower-tier launch "
                      "plus the top-tier launch; mean over the 4 stages of a step",
            "workload": "roofline probe: N=10^4, m=4, L=10, d=0 (17,347,066 unique variables, "
                        "278 MB per FP64 vector)",
            "algorithmic_bytes_per_launch": int(bytes_launch),
            "bytes_per_var": stage_bytes_per_var(0) / 4.0, "table_bytes": ri["table_bytes"],
            "mean_launch_us": round(launch_ms * 1e3, 2),
            "rhs_updates_per_s": ri["n_var"] * 4 * args.roofline_steps / (rms / 1e3),
            "table_build_s": round(build_s, 2),
        }
        del ry, img2, TR

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, lambda i: 1.0 if i == 1 else 0.0, dt, args.cpu_seconds)
        out["cpu_baseline"]["speedup_gpu_over_cpu"] = round(value / out["cpu_baseline"]["value"], 1)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
