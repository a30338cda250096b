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
                   on a bounded sample of the same workload, one host core;
  batched       -- 512 independent problems drawn with seed 0 (N, m, L, bath,
                   coupling and loss drawn over the batched ranges), RK4 steps of
                   all of them in FP64 and FP32 batches against the plain FP64
                   propagator called once per problem;
  serving       -- a Poisson trace of propagation requests (problems as the
                   batched draw plus a horizon) replayed through the
                   continuous-batching server and through the plain propagator
                   one request at a time: solves/s, p50/p99 latency.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --serve-sweep 0.25,0.5,1,2,10 [--serve-window S] [--serve-deadline S]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

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
      FP32: stage 1 reads y, writes u1 (24); 2 reads u1, writes u2 (16);
            3 reads u2, u1, writes u3 (24); 4 reads u3, u1, y, writes y (48)
                                                               -> 112
    """
    return 176 if precision == 0 else 112


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
    wb = info["work_bytes_fp64"] if (precision & 1) == 0 else info["work_bytes_fp32"]
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


POP_COLS = list(range(1, 9))   # every population of an observable row (cavity ... other sites)


def _rate(ms, n_inst, vars_total, steps):
    sec = ms / 1e3
    return {"ms_per_step": round(ms / steps, 4), "instance_steps_per_s": n_inst * steps / sec,
            "rhs_updates_per_s": vars_total * 4 * steps / sec}


def batched_section(torch, steps, n=512, seed=0, dt=0.02, flag=0, compact=False):
    """Many independent problems at once: the batched launch (every instance
    in one launch per stage and per m) in FP64 and FP32-bulk, against the
    plain per-instance FP64 propagator called once per instance. Time per
    mode = HIP events around `steps` RK4 steps of all instances (each
    instance's tables and state already resident)."""
    from paper_2608_20657_amd import heom, serve as S, workloads as W
    ps = W.draw_batch(n, seed)
    t0 = time.perf_counter()
    structs = {}
    for q in ps:
        k = S.structure_key(q)
        if k not in structs:
            structs[k] = heom.Tables(q)
            if compact:
                structs[k].set_tuning(compact=1)
    build_s = time.perf_counter() - t0
    st = torch.cuda.current_stream()
    imgs = {}
    for k, T in structs.items():
        imgs[k] = torch.empty(S._round(T.info()["table_bytes"]), dtype=torch.uint8, device="cuda")
        T.upload(imgs[k], st)
    inst = []
    for q in ps:
        T = structs[S.structure_key(q)]
        info = T.info()
        params = torch.empty(S._round(T.params_bytes()), dtype=torch.uint8, device="cuda")
        T.upload_params(q, params, st)
        y = torch.empty(info["n_var"], dtype=torch.complex128, device="cuda")
        work = torch.empty(S._round(info["work_bytes_fp64"]), dtype=torch.uint8, device="cuda")
        inst.append((q, T, params, y, work, T.tier0_pure(1.0, 0.0, [0.0] * q.d), info["n_var"]))
    nv = sum(x[6] for x in inst)
    # tables every stage reads: each instance's tiles read its structure's
    # metadata (shared images are re-read per instance)
    tab = sum(x[1].info()["stage_table_bytes"] for x in inst)
    batch = heom.Batch(len(inst))
    obs_bufs = []
    for i, (q, T, params, y, work, t0v, _) in enumerate(inst):
        T.init_state(t0v, y, st)
        obs_bufs.append(torch.zeros(3 * 10, dtype=torch.float64, device="cuda"))
        batch.set_slot(i, T, y, work, dt, params=params, obs=obs_bufs[-1], obs_every=1 + steps)
    batch.commit(torch, st)
    out = {"workload": f"{n} independent problems drawn with seed {seed}: N~U{{4..5000}}, m~U{{1..4}}, "
                       "L~U{3..10}, g~U[0.002,0.03], lam~U[0.005,0.05], gam~U[0.02,0.2], kappa~U[0,0.02], "
                       "kT=0.025, resonant, d=0, rho(0)=|c><c|, dt=0.02",
           "instances": len(inst), "unique_vars_total": nv, "structure_keys": len(structs),
           "largest_instance_vars": max(x[6] for x in inst),
           "median_instance_vars": int(sorted(x[6] for x in inst)[len(inst) // 2]),
           "steps": steps, "table_build_s": round(build_s, 2), "hermitian_ados": bool(flag),
           "table_bytes_read_per_stage": tab}
    for prec, name in ((0, "fp64_batched"), (1, "fp32_batched")):
        for q, T, params, y, work, t0v, _ in inst:
            T.init_state(t0v, y, st)
        batch.propagate(1, prec | flag, st)                # warm-up step
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        batch.propagate(steps, prec | flag, st)
        e1.record(st)
        torch.cuda.synchronize()
        out[name] = _rate(e0.elapsed_time(e1), len(inst), nv, steps)
        # algorithmic bytes of one RK4 step (state as stage_bytes_per_var
        # counts it, plus four stages of table reads) over the step time
        gbs = (nv * stage_bytes_per_var(prec) + 4 * tab) / (out[name]["ms_per_step"] * 1e-3) / 1e9
        out[name]["algorithmic_GBps"] = round(gbs, 1)
        out[name]["hbm_frac"] = round(gbs / HBM_PEAK_GBS, 4)
        out[name]["finite"] = bool(all(torch.isfinite(x[3][:64]).all().item() for x in inst[:64]))
    # every slot recorded its observables after 1 + steps FP64 steps (row 1) and,
    # from the same start, after 1 + steps FP32 steps (row 2)
    ob = np.stack([o.cpu().numpy().reshape(-1, 10) for o in obs_bufs])
    out["max_abs_population_diff_fp32_vs_fp64"] = float(np.abs(ob[:, 2, POP_COLS] - ob[:, 1, POP_COLS]).max())
    del batch
    total_ms = 0.0
    for q, T, params, y, work, t0v, _ in inst:            # plain: one problem at a time
        T.set_params(q)
        T.upload(imgs[S.structure_key(q)], st)
        T.init_state(t0v, y, st)
        T.propagate(y, work, dt, 1, 0, None, flag, st)     # warm-up step
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        T.propagate(y, work, dt, steps, 0, None, flag, st)
        e1.record(st)
        torch.cuda.synchronize()
        total_ms += e0.elapsed_time(e1)
    out["fp64_plain_one_at_a_time"] = _rate(total_ms, len(inst), nv, steps)
    base = out["fp64_plain_one_at_a_time"]["instance_steps_per_s"]
    out["speedup_fp64_batched_vs_plain"] = round(out["fp64_batched"]["instance_steps_per_s"] / base, 3)
    out["speedup_fp32_batched_vs_plain"] = round(out["fp32_batched"]["instance_steps_per_s"] / base, 3)
    del inst, imgs
    torch.cuda.empty_cache()
    return out


def serving_point(torch, rate, window, deadline, seed=1, precision=0, budget_gib=256.0,
                  lanes=(1 << 20,), capacity=(256, 32), fifo=True, flag=0):
    """Poisson arrivals of propagation requests (problems drawn as in the
    batched workload, plus a horizon of U{1000..20000} steps, obs every 100
    steps, dt=0.02). Arrivals in [0, window) are submitted; the run ends at
    `deadline` seconds or when all are done. The continuous-batching server
    (precision as given) and the plain FP64 propagator one request at a time
    (FIFO) replay the same trace."""
    from paper_2608_20657_amd import serve as S, workloads as W
    arr = W.arrival_times(rate, window, seed)
    ps = W.draw_batch(len(arr), seed=seed, with_horizon=True)
    reqs = S.make_requests(ps, arr, dt=0.02, obs_every=100)
    out = {"workload": f"Poisson arrivals at {rate} req/s for {window} s (seed {seed}); problems as the batched "
                       "workload plus horizon U{1000..20000} steps, dt=0.02, observables every 100 steps",
           "rate_req_per_s": rate, "window_s": window, "deadline_s": deadline, "requests": len(reqs),
           "offered_rhs_updates_per_s": None}
    srv = S.Server(torch, int(budget_gib * (1 << 30)), lanes=list(lanes), capacity=list(capacity),
                   precision=precision | flag)
    srv.prepare(ps)
    work = sum(srv.structs[S.structure_key(q)].n_var * 4 * r.horizon for q, r in zip(ps, reqs))
    out["offered_rhs_updates_per_s"] = work / window
    st = srv.run(reqs, window, deadline)
    st["precision"] = "fp32-bulk" if precision == 1 else "fp64"
    st["hermitian_ados"] = bool(flag)
    st["budget_gib"] = budget_gib
    st["lanes_vars_threshold"] = list(lanes)
    out["served"] = st
    if fifo:
        ff = S.Fifo(torch, precision=flag)
        ff.prepare(ps)
        st2 = ff.run(reqs, window, deadline)
        st2["precision"] = "fp64"
        st2["hermitian_ados"] = bool(flag)
        out["plain_fifo"] = st2
        got = {r.rid: r.obs for r in srv.results}
        errs = [float(np.abs(got[r.rid][:, POP_COLS] - r.obs[:, POP_COLS]).max()) for r in ff.results if r.rid in got]
        out["max_abs_population_diff_served_vs_plain_fp64"] = max(errs) if errs else None
        out["compared_requests"] = len(errs)
        if st2["solves_per_s"] > 0:
            out["solves_per_s_ratio_served_over_plain"] = round(st["solves_per_s"] / st2["solves_per_s"], 3)
        del ff
    del srv
    torch.cuda.empty_cache()
    return out


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
    ap.add_argument("--batched-steps", type=int, default=5)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=0.5)
    ap.add_argument("--serve-window", type=float, default=20.0)
    ap.add_argument("--serve-deadline", type=float, default=40.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-precision", choices=["fp64", "fp32"], default="fp64",
                    help="arithmetic of the continuous-batching server (the plain baseline is always FP64)")
    ap.add_argument("--serve-sweep", type=str, default="",
                    help="comma-separated arrival rates: print one serving JSON line per rate and exit")
    ap.add_argument("--general", action="store_true",
                    help="do not assert Hermitian ADOs (every workload here starts from a Hermitian rho_S(0) "
                         "with c_check = conj(c), so by default column gathers of large states read mirrored "
                         "entries; this switch uses the general transposed-copy path)")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="also run a plain device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only; --gpus must be 1 (the path has no multi-GPU "
              "launch: independent problems would shard across GPUs without exchange)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_2608_20657_amd import heom, workloads as W

    precision = 0 if args.precision == "fp64" else 1
    herm = 0 if args.general else heom.HEOM_HERMITIAN
    if args.serve_sweep:
        for r in [float(x) for x in args.serve_sweep.split(",") if x]:
            rec = serving_point(torch, r, args.serve_window, args.serve_deadline,
                                precision=0 if args.serve_precision == "fp64" else 1, flag=herm)
            print(json.dumps({"serving_sweep_point": rec}), flush=True)
        return
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
        # the first candidate would otherwise be timed while the clocks ramp up
        autotune.autotune(T, torch, tier0, dt, steps=2000, precision=precision, cands=cands[:1], repeats=1)
        tuned = autotune.autotune(T, torch, tier0, dt, steps=1000, precision=precision, cands=cands, repeats=3)
    else:
        img = torch.empty(T.info()["table_bytes"], dtype=torch.uint8, device="cuda")
        T.upload(img, torch.cuda.current_stream())
    info = T.info()
    if args.roofline_only:
        args.steps, args.warmup = 1, 0
    ms, wall, y, obs = time_propagate(T, torch, tier0, dt, args.steps, args.warmup, args.obs_every, precision | herm)
    n = info["n_var"]
    updates = n * 4 * args.steps
    value = updates / (ms / 1e3)
    ob = obs.cpu().numpy().reshape(-1, 10)
    finite = bool(torch.isfinite(y).all().item()) and bool(math.isfinite(float(ob[-1, 0])))

    per_launch_ms = ms / (4 * args.steps)
    bpv = stage_bytes_per_var(precision) / 4.0
    main_bytes = n * bpv + info["stage_table_bytes"]
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
                   "obs_every": args.obs_every, "precision": args.precision, "hermitian_ados": not args.general,
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
        if herm:
            TR.set_tuning(compact=1)
        build_s = time.perf_counter() - t0
        ri = TR.info()
        img2 = torch.empty(ri["table_bytes"], dtype=torch.uint8, device="cuda")
        TR.upload(img2, torch.cuda.current_stream())
        t0r = TR.tier0_pure(1.0, 0.0, [])
        rms, _, ry, _ = time_propagate(TR, torch, t0r, dt, args.roofline_steps, 3, 0, herm)
        launch_ms = rms / (4 * args.roofline_steps)
        bytes_launch = ri["n_var"] * stage_bytes_per_var(0) / 4.0 + ri["stage_table_bytes"]
        achieved = bytes_launch / (launch_ms * 1e-3) / 1e9
        traffic = load_traffic()
        out["roofline"] = {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic["bytes_per_launch"] if traffic else None,
            "kernel": "stage_kernel, FP64 RK4 stage (RHS + combination); one stage = the lower-tier launch "
                      "plus the top-tier launch; mean over the 4 stages of a step",
            "tiles": "compact (Hermitian ADOs: upper triangles, mirrored column gathers)" if herm
                     else "full, transposed copy for column gathers",
            "workload": "roofline probe: N=10^4, m=4, L=10, d=0 (17,347,066 unique variables, "
                        "278 MB per FP64 vector)",
            "algorithmic_bytes_per_launch": int(bytes_launch),
            "bytes_per_var": stage_bytes_per_var(0) / 4.0, "table_bytes_read": ri["stage_table_bytes"],
            "mean_launch_us": round(launch_ms * 1e3, 2),
            "rhs_updates_per_s": ri["n_var"] * 4 * args.roofline_steps / (rms / 1e3),
            "table_build_s": round(build_s, 2),
        }
        del ry, img2, TR
        if herm and not args.roofline_only:
            # the same stage on the general path (no Hermitian assertion: full
            # tiles, column gathers from a transposed copy), for reference
            TG = heom.Tables(q)
            img3 = torch.empty(TG.info()["table_bytes"], dtype=torch.uint8, device="cuda")
            TG.upload(img3, torch.cuda.current_stream())
            gms, _, gy, _ = time_propagate(TG, torch, t0r, dt, 10, 3, 0, 0)
            gl = gms / 40.0
            gbytes = ri["n_var"] * stage_bytes_per_var(0) / 4.0 + TG.info()["stage_table_bytes"]
            out["roofline"]["general_path"] = {
                "mean_launch_us": round(gl * 1e3, 2), "algorithmic_bytes_per_launch": int(gbytes),
                "achieved": round(gbytes / (gl * 1e-3) / 1e9, 1),
                "frac": round(gbytes / (gl * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            del gy, img3, TG

    if args.roofline_only:
        args.no_batched = args.no_serve = True
    if not args.no_batched:
        out["batched"] = batched_section(torch, args.batched_steps, flag=herm, compact=bool(herm))
    if not args.no_serve:
        out["serving"] = serving_point(torch, args.serve_rate, args.serve_window, args.serve_deadline,
                                       precision=0 if args.serve_precision == "fp64" else 1, flag=herm)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, lambda i: 1.0 if i == 1 else 0.0, dt, args.cpu_seconds)
        out["cpu_baseline"]["speedup_gpu_over_cpu"] = round(value / out["cpu_baseline"]["value"], 1)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
