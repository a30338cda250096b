#!/usr/bin/env python3
"""Benchmark of the symmetry-adapted HEOM hot path on one MI355X.

Headline (`value`): the batched workload -- 512 independent problems drawn
with seed 0 (N~U{4..5000}, m~U{1..4}, L~U{3..10}, g~U[0.002,0.03],
lam~U[0.005,0.05], gam~U[0.02,0.2], kappa~U[0,0.02], kT=0.025, resonant,
d=0, rho(0)=|c><c|, dt=0.02; 5.3e8 unique variables in all, 8.5 GB per FP64
state). One step = one classical RK4 step of every problem (four fused
right-hand-side + combination stages over every unique variable of every
problem), complex FP64, through heom_batch_propagate. Tables are built and
uploaded before the timed region (the paper's precomputation); every state
is resident in HBM when timing starts. `--warmup` untimed steps, then
`--steps` steps bracketed by device synchronizations and HIP events on the
launch stream.

Metric: unique-variable RHS updates/s = sum of n_var * 4 * steps / time.

Also reported on the same JSON line:
  roofline       -- the batched FP64 step against the 8 TB/s HBM peak:
                    algorithmic bytes of one step (state bytes of the four
                    stages plus the table bytes they read) / step time from the
                    same HIP events; traffic from the committed counter runs;
  roofline_probe -- the RK4 stage kernel alone on the largest structure of the
                    draw (N=10^4, m=4, L=10: 17.3 M variables, 278 MB per FP64
                    vector, above the 256 MB last-level cache);
  batched        -- the same draw in FP32-bulk, and the plain FP64
                    propagator called once per problem;
  localized      -- one small problem (N=64, m=2, L=6, d=1, 21,105 variables;
                    cache resident, launch-latency bound) over 10^4 steps;
  serving        -- Poisson traces of propagation requests (problems as the
                    draw plus a horizon) replayed through the continuous-
                    batching server in FP32 bulk and through the plain FP64
                    propagator one request at a time, at a light and a loaded
                    arrival rate: solves/s, p50/p99 latency, population error;
  cpu_baseline   -- the oracle's generator run by a compiled classical-RK4 loop
                    (C, OpenMP) on the host cores, on a bounded sample of the
                    draw (2000 steps of each of its first problems up to a
                    variable budget), all threads and one thread, plus the
                    localized problem over its full 10^4 steps.

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
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_stage_fp64_roofline_probe.json")
PROFILE_TRAFFIC_BATCH = os.path.join(ROOT, "profiles", "traffic_batch_fp64_batched_draw.json")
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


def progress(msg):
    """One line on stderr per finished section (stdout carries only the JSON line)."""
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def load_traffic(path):
    """Counter-derived HBM bytes per launch from a committed profile summary,
    or None once the kernel source has changed since the counters were
    taken."""
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
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


def element_bytes_per_step(info):
    """FP64 bytes of one RK4 step counted by element: every stage reads the
    input at the distinct positions it reads (own values and gather
    targets), stages 2-4 also the base term at the own entries, every stage
    writes the whole output, plus four stages of table reads. Compact tiles
    read fewer elements than the method-level count assumes; HBM moves
    128-byte lines, and those lines cover nearly the whole state."""
    return (16 * (4 * info["read_entries"] + 3 * info["own_entries"] + 4 * info["n_var"])
            + 4 * info["stage_table_bytes"])


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


_TIMER_DIR = None


def cpu_timer_exe():
    """The CPU baseline's RK4 loop compiled for this host (-march=native),
    in a temporary directory removed when the process ends."""
    global _TIMER_DIR
    from oracle import cpu_timer
    if _TIMER_DIR is None:
        _TIMER_DIR = tempfile.TemporaryDirectory(prefix="heom_cpu_timer_")
    return cpu_timer.build_timer(_TIMER_DIR.name)


def cpu_baseline(dt, var_budget, max_vars, steps=2000, local_steps=10000):
    """The oracle's generator M_u (oracle.uvar) run by the compiled classical
    RK4 loop (oracle/csr_rk4.c, OpenMP) on the host cores: a bounded sample
    of the batched draw -- its first problems in draw order with at most
    `max_vars` unique variables each, up to `var_budget` in all (the oracle
    assembles M_u in Python, which bounds the sample) -- for `steps` steps
    each, on all host threads and on one; and the localized problem over its
    full `local_steps` steps on all threads. Reported in the headline's unit
    (unique-variable RHS updates/s, four per RK4 step)."""
    from oracle import cpu_timer, uvar
    from paper_2608_20657_amd import workloads as W
    exe = cpu_timer_exe()
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    picked, total = [], 0
    t0 = time.perf_counter()
    for i, q in enumerate(W.draw_batch(512, 0)):
        S = uvar.UVarSystem(q)
        if S.n_var > max_vars:
            continue
        if total + S.n_var > var_budget:
            break
        y0 = np.zeros(S.n_var, complex)
        y0[0] = 1.0                        # rho(0) = |c><c|: Z of the empty pattern
        picked.append((i, S.generator(), y0))
        total += S.n_var
    build_s = time.perf_counter() - t0
    out = {}
    for label, th in (("all", threads), ("one", 1)):
        sec = used = 0
        for i, A, y0 in picked:
            _, info = cpu_timer.run_rk4(exe, A, y0, dt, steps, th)
            sec += info["seconds"]
            used = info["threads"]
        out[label] = (total * 4 * steps / sec, sec, used)
    pl = W.config_localized()
    S = uvar.UVarSystem(pl)
    A = S.generator()
    y0 = S.initial_state(amp=lambda i: 1.0 if i == 1 else 0.0)
    _, li = cpu_timer.run_rk4(exe, A, y0, dt, local_steps, threads)
    nnz = sum(A.nnz for _, A, _ in picked)
    return dict(value=out["all"][0], unit="unique-variable RHS updates/s", cores=out["all"][2], kind="oracle",
                sample=f"batched draw (seed 0): the first {len(picked)} problems in draw order with at most "
                       f"{max_vars} unique variables each ({total} variables, {nnz} generator nonzeros), "
                       f"{steps} classical RK4 steps each with the oracle's CSR generator in a compiled C/OpenMP "
                       f"loop, {out['all'][2]} threads ({out['all'][1]:.2f} s)",
                single_thread_value=out["one"][0], single_thread_seconds=round(out["one"][1], 3),
                oracle_assembly_s=round(build_s, 1),
                localized={"value": S.n_var * 4 * local_steps / li["seconds"], "steps": local_steps,
                           "seconds": round(li["seconds"], 3), "threads": li["threads"], "nnz": A.nnz})


def cpu_configs(dt_small=0.05, dt=0.02):
    """The compiled RK4 loop on the oracle's generator for the three
    single-problem workloads at their full step counts on all host threads
    (small: 2,000 steps; localized and saturated: 10^4), and on one thread
    (the saturated workload over a 500-step prefix)."""
    from oracle import cpu_timer, uvar
    from paper_2608_20657_amd import workloads as W
    exe = cpu_timer_exe()
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    out = {}
    for name, p, h, steps, one_steps, amp in (
            ("small", W.config_small(), dt_small, 2000, 2000, lambda i: 1.0 if i == 0 else 0.0),
            ("localized", W.config_localized(), dt, 10000, 10000, lambda i: 1.0 if i == 1 else 0.0),
            ("saturated", W.config_saturated(), dt, 10000, 500, None)):
        t0 = time.perf_counter()
        S = uvar.UVarSystem(p)
        A = S.generator()
        if amp is None:
            import math as _m
            th = 0.5 * _m.atan2(2 * p.g * _m.sqrt(p.N), p.omega_c - p.eps)
            amp = lambda i, c=_m.cos(th), s=_m.sin(th) / _m.sqrt(p.N): c if i == 0 else s
        y0 = S.initial_state(amp=amp)
        asm = time.perf_counter() - t0
        _, all_ = cpu_timer.run_rk4(exe, A, y0, h, steps, threads)
        _, one = cpu_timer.run_rk4(exe, A, y0, h, one_steps, 1)
        out[name] = {"n_var": S.n_var, "nnz": A.nnz, "oracle_assembly_s": round(asm, 1),
                     "all_threads": {"threads": all_["threads"], "steps": steps, "seconds": round(all_["seconds"], 3),
                                     "updates_per_s": S.n_var * 4 * steps / all_["seconds"]},
                     "one_thread": {"steps": one_steps, "seconds": round(one["seconds"], 3),
                                    "updates_per_s": S.n_var * 4 * one_steps / one["seconds"]}}
    return out


POP_COLS = list(range(1, 9))   # every population of an observable row (cavity ... other sites)


def _rate(ms, n_inst, vars_total, steps):
    sec = ms / 1e3
    return {"ms_per_step": round(ms / steps, 4), "instance_steps_per_s": n_inst * steps / sec,
            "rhs_updates_per_s": vars_total * 4 * steps / sec}


def batched_section(torch, steps, warmup, n=512, seed=0, dt=0.02, flag=0, compact=False, tune_tiles=False,
                    tune_shape=False):
    """Many independent problems at once: the batched launch (every instance
    in one launch per stage and per m) in FP64 and FP32-bulk, against the
    plain per-instance FP64 propagator called once per instance. Time per
    mode = HIP events around `steps` RK4 steps of all instances after
    `warmup` untimed ones (each instance's tables and state already
    resident)."""
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
    tiles = {}
    if tune_tiles:
        # tile size per structure, by the single-problem tuner on a problem
        # of that structure (before any parameter block is written for it)
        from paper_2608_20657_amd import autotune
        for k, T in structs.items():
            r = autotune.tune_structure_tiles(T, torch, T.tier0_pure(1.0, 0.0, [0.0] * k[3]), dt, steps=10,
                                              precision=flag)
            tiles[str(k)] = r["best"]["tile_vars"]
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
    elem = sum(element_bytes_per_step(x[1].info()) for x in inst)
    batch = heom.Batch(len(inst))
    obs_bufs = []
    for i, (q, T, params, y, work, t0v, _) in enumerate(inst):
        T.init_state(t0v, y, st)
        obs_bufs.append(torch.zeros(3 * 10, dtype=torch.float64, device="cuda"))
        batch.set_slot(i, T, y, work, dt, params=params, obs=obs_bufs[-1], obs_every=warmup + steps)
    batch.commit(torch, st)
    shape = None
    if tune_shape:
        from paper_2608_20657_amd import autotune
        shape = autotune.autotune_batch(batch, torch, steps=3, precision=flag, merges=(0, 4096, 16384, 65536),
                                        shares=(1, 2), interleaves=(0, 8, 32, 128))
    out = {"workload": f"{n} independent problems drawn with seed {seed}: N~U{{4..5000}}, m~U{{1..4}}, "
                       "L~U{3..10}, g~U[0.002,0.03], lam~U[0.005,0.05], gam~U[0.02,0.2], kappa~U[0,0.02], "
                       "kT=0.025, resonant, d=0, rho(0)=|c><c|, dt=0.02",
           "instances": len(inst), "unique_vars_total": nv, "structure_keys": len(structs),
           "largest_instance_vars": max(x[6] for x in inst),
           "median_instance_vars": int(sorted(x[6] for x in inst)[len(inst) // 2]),
           "steps": steps, "warmup": warmup, "table_build_s": round(build_s, 2), "hermitian_ados": bool(flag),
           "table_bytes_read_per_stage": tab,
           "element_bytes_per_step": elem,
           "tuned_tile_vars": tiles or None,
           "tuned_launch_shape": ({"best": shape["best"], "ms_per_step": {f"merge={c['merge_tiles']},share="
                                   f"{c['share_slots']},interleave={c['interleave']}": round(t, 3)
                                   for c, t in shape["results"]}}
                                  if shape else None)}
    for prec, name in ((0, "fp64_batched"), (1, "fp32_batched")):
        for q, T, params, y, work, t0v, _ in inst:
            T.init_state(t0v, y, st)
        if warmup:
            batch.propagate(warmup, prec | flag, st)       # untimed
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record(st)
        batch.propagate(steps, prec | flag, st)
        e1.record(st)
        torch.cuda.synchronize()
        out[name] = _rate(e0.elapsed_time(e1), len(inst), nv, steps)
        out[name]["wall_s"] = round(time.perf_counter() - w0, 4)
        out[name]["nonfinite_slots"] = int(batch.status(st).sum())
        # algorithmic bytes of one RK4 step (state as stage_bytes_per_var
        # counts it, plus four stages of table reads) over the step time
        gbs = (nv * stage_bytes_per_var(prec) + 4 * tab) / (out[name]["ms_per_step"] * 1e-3) / 1e9
        out[name]["algorithmic_GBps"] = round(gbs, 1)
        out[name]["hbm_frac"] = round(gbs / HBM_PEAK_GBS, 4)
        out[name]["finite"] = bool(all(torch.isfinite(x[3][:64]).all().item() for x in inst[:64]))
    # every slot recorded its observables after warmup + steps FP64 steps (row 1)
    # and, from the same start, after warmup + steps FP32 steps (row 2)
    ob = np.stack([o.cpu().numpy().reshape(-1, 10) for o in obs_bufs])
    out["max_abs_population_diff_fp32_vs_fp64"] = float(np.abs(ob[:, 2, POP_COLS] - ob[:, 1, POP_COLS]).max())
    del batch
    total_ms = 0.0
    for q, T, params, y, work, t0v, _ in inst:            # plain: one problem at a time
        T.set_params(q)
        T.upload(imgs[S.structure_key(q)], st)
        T.init_state(t0v, y, st)
        T.propagate(y, work, dt, max(warmup, 1), 0, None, flag, st)     # untimed
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
                  lanes=(1 << 17, 1 << 20), capacity=(256, 64, 32), fp64_below=1 << 17, fifo=True, flag=0):
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
    # lanes of states below fp64_below variables step in FP64 (launch-latency
    # bound: FP32 bulk saves nothing there), the others in `precision`
    bounds = list(lanes) + [None]
    precs = [(0 if (b is not None and b <= fp64_below) else precision) | flag for b in bounds]
    # both paths first serve one problem of every structure key of the trace
    # for 100 steps (kernels loaded, images uploaded once, allocator and
    # caches warm), then the timed replay
    first = {}
    for q in ps:
        first.setdefault(S.structure_key(q), q)
    warm = S.make_requests(list(first.values()), [0.0] * len(first), dt=0.02, obs_every=100)
    for r in warm:
        r.horizon = 100
    ws = S.Server(torch, int(budget_gib * (1 << 30)), lanes=list(lanes), capacity=list(capacity), precision=precs)
    ws.prepare(list(first.values()))
    ws.run(warm)
    if fifo:
        wf = S.Fifo(torch, precision=flag)
        wf.prepare(list(first.values()))
        wf.run(warm)
        del wf
    del ws
    torch.cuda.synchronize()
    srv = S.Server(torch, int(budget_gib * (1 << 30)), lanes=list(lanes), capacity=list(capacity),
                   precision=precs)
    srv.prepare(ps)
    work = sum(srv.structs[S.structure_key(q)].n_var * 4 * r.horizon for q, r in zip(ps, reqs))
    out["offered_rhs_updates_per_s"] = work / window
    st = srv.run(reqs, window, deadline)
    st["precision"] = ["fp32-bulk" if (p & 1) else "fp64" for p in precs]
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


def copy_bandwidth(torch, mib=2048, reps=10):
    """Achievable HBM bandwidth on this device: a plain device-to-device copy
    of `mib` MiB (read + write bytes per copy / time, HIP events, best of
    `reps`), for context beside the 8 TB/s nominal peak."""
    n = (mib << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    torch.cuda.empty_cache()
    return round(2 * (mib << 20) / (best * 1e-3) / 1e9, 1)


def localized_section(torch, args, precision, herm):
    """The localized problem alone (N=64, m=2, L=6, d=1; 21,105 unique
    variables, cache resident): autotuned launch, then `--local-steps` RK4
    steps timed with HIP events after `--local-warmup` untimed ones."""
    from paper_2608_20657_amd import heom, workloads as W
    p = W.config_localized()
    dt = 0.02
    T = heom.Tables(p)
    tier0 = T.tier0_pure(0.0, 0.0, [1.0])
    tuned = None
    if not args.no_autotune:
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
    ms, wall, y, obs = time_propagate(T, torch, tier0, dt, args.local_steps, args.local_warmup, args.obs_every,
                                      precision | herm)
    n = info["n_var"]
    ob = obs.cpu().numpy().reshape(-1, 10)
    per_launch_ms = ms / (4 * args.local_steps)
    main_bytes = n * stage_bytes_per_var(precision) / 4.0 + info["stage_table_bytes"]
    return {
        "workload": "localized: N=64, m=2 (Debye + 1 Matsubara, lam=0.02, gam=0.1, kT=0.025), L=6, d=1, g=0.01, "
                    "eps-omega_c=0.01, kappa=0.005, rho(0)=|e_1><e_1|, dt=0.02",
        "value": n * 4 * args.local_steps / (ms / 1e3), "unit": "unique-variable RHS updates/s",
        "steps": args.local_steps, "warmup": args.local_warmup, "ms_per_step": ms / args.local_steps,
        "wall_s": round(wall, 4), "n_var": n, "patterns": info["n_patterns"], "obs_every": args.obs_every,
        "finite": bool(torch.isfinite(y).all().item()) and bool(np.isfinite(ob).all()),
        "final_observables": [float(x) for x in ob[-1]],
        "stage_kernel": dict(bound="latency", achieved=round(main_bytes / (per_launch_ms * 1e-3) / 1e9, 1),
                             unit="GB/s", mean_launch_us=round(per_launch_ms * 1e3, 3),
                             note="21,105-variable state is cache resident; launch and gather latency bound"),
        "launch_config": T.tuning(),
        "autotune_us_per_step": {str(c["tile_vars"]): round(t * 1e3, 2) for c, t in tuned["results"]}
        if tuned else None,
    }


def time_rhs(T, torch, y, precision, info, calls=20):
    """heom_rhs alone (dy = M_u y, no RK4 combination) on a resident state:
    mean time per call from HIP events over `calls` calls, in unique-variable
    RHS updates/s and against the HBM peak (reads y, writes dy: 32 B per
    variable, plus the tables)."""
    s = torch.cuda.current_stream()
    dy = torch.empty_like(y)
    for _ in range(3):
        T.rhs(y, dy, s, precision=precision)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(calls):
        T.rhs(y, dy, s, precision=precision)
    e1.record(s)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / calls
    nbytes = 32 * info["n_var"] + info["stage_table_bytes"]
    gbs = nbytes / (us * 1e-6) / 1e9
    del dy
    return {"mean_us": round(us, 2), "rhs_updates_per_s": info["n_var"] / (us * 1e-6),
            "algorithmic_bytes_per_call": int(nbytes), "achieved_GBps": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4), "calls": calls}


def probe_section(torch, args, herm, general=True):
    """The RK4 stage kernel alone on the largest structure of the draw
    (N=10^4, m=4, L=10: 17.3 M variables): mean stage time from HIP events
    over `--roofline-steps` FP64 steps, against the HBM peak."""
    from paper_2608_20657_amd import heom, workloads as W
    q = W.config_roofline_probe()
    dt = 0.02
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
    elem_launch = element_bytes_per_step(ri) / 4.0
    traffic = load_traffic(PROFILE_TRAFFIC)
    out = {
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
        "element_bytes_per_launch": int(elem_launch),
        "frac_element_bytes": round(elem_launch / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "mean_launch_us": round(launch_ms * 1e3, 2),
        "rhs_updates_per_s": ri["n_var"] * 4 * args.roofline_steps / (rms / 1e3),
        "table_build_s": round(build_s, 2),
    }
    out["heom_rhs"] = time_rhs(TR, torch, ry, herm, ri)
    del ry, img2, TR
    if herm and general:
        # the same stage on the general path (no Hermitian assertion: full
        # tiles, column gathers from a transposed copy), for reference
        TG = heom.Tables(q)
        img3 = torch.empty(TG.info()["table_bytes"], dtype=torch.uint8, device="cuda")
        TG.upload(img3, torch.cuda.current_stream())
        gms, _, gy, _ = time_propagate(TG, torch, t0r, dt, 10, 3, 0, 0)
        gl = gms / 40.0
        gbytes = ri["n_var"] * stage_bytes_per_var(0) / 4.0 + TG.info()["stage_table_bytes"]
        out["general_path"] = {
            "mean_launch_us": round(gl * 1e3, 2), "algorithmic_bytes_per_launch": int(gbytes),
            "achieved": round(gbytes / (gl * 1e-3) / 1e9, 1),
            "frac": round(gbytes / (gl * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        del gy, img3, TG
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed RK4 steps of the batched headline")
    ap.add_argument("--warmup", type=int, default=5, help="untimed RK4 steps before them")
    ap.add_argument("--local-steps", type=int, default=10000)
    ap.add_argument("--local-warmup", type=int, default=1000)
    ap.add_argument("--obs-every", type=int, default=100)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64",
                    help="arithmetic of the localized solve")
    ap.add_argument("--roofline-steps", type=int, default=25)
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-var-budget", type=int, default=200000,
                    help="unique variables of the batched draw in the CPU baseline's sample")
    ap.add_argument("--cpu-max-vars", type=int, default=60000)
    ap.add_argument("--cpu-steps", type=int, default=2000, help="RK4 steps per problem of that sample")
    ap.add_argument("--cpu-configs", action="store_true",
                    help="only the CPU baseline on the single-problem workloads at full step counts; print and exit")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the single-structure stage kernel (for profiling it alone)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched headline (for profiling it alone)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tune-tiles", action="store_true",
                    help="tune each structure's tile size for the batched headline (before timing)")
    ap.add_argument("--tune-batch", action="store_true",
                    help="tune the batched headline's launch shape: merge threshold, slots per shared workgroup")
    ap.add_argument("--no-local", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--serve-rates", type=str, default="0.5:20:40,10:10:20",
                    help="serving points rate:window:deadline (seconds), comma separated")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-precision", choices=["fp64", "fp32"], default="fp32",
                    help="arithmetic of the continuous-batching server (the plain baseline is always FP64)")
    ap.add_argument("--serve-sweep", type=str, default="",
                    help="comma-separated arrival rates: print one serving JSON line per rate and exit")
    ap.add_argument("--serve-window", type=float, default=60.0)
    ap.add_argument("--serve-deadline", type=float, default=60.0)
    ap.add_argument("--general", action="store_true",
                    help="do not assert Hermitian ADOs (every workload here starts from a Hermitian rho_S(0) "
                         "with c_check = conj(c), so by default column gathers of large states read mirrored "
                         "entries and tiles are compact; this switch uses the general transposed-copy path)")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="also run a plain device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.cpu_configs:
        print(json.dumps({"cpu_configs": cpu_configs()}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py: measures one GPU only; --gpus must be 1 (the path has no multi-GPU "
              "launch: independent problems would shard across GPUs without exchange)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_2608_20657_amd import heom

    precision = 0 if args.precision == "fp64" else 1
    herm = 0 if args.general else heom.HEOM_HERMITIAN
    serve_prec = 0 if args.serve_precision == "fp64" else 1
    if args.serve_sweep:
        for r in [float(x) for x in args.serve_sweep.split(",") if x]:
            rec = serving_point(torch, r, args.serve_window, args.serve_deadline, precision=serve_prec, flag=herm)
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
        rec = probe_section(torch, args, herm, general=False)
        print(json.dumps({"roofline_probe": rec}), flush=True)
        return

    copy_gbs = copy_bandwidth(torch)
    bt = batched_section(torch, args.steps, args.warmup, flag=herm, compact=bool(herm), tune_tiles=args.tune_tiles,
                         tune_shape=args.tune_batch)
    f64 = bt["fp64_batched"]
    progress(f"batched draw done: {f64['ms_per_step']} ms per FP64 step")
    traffic = load_traffic(PROFILE_TRAFFIC_BATCH)
    step_bytes = bt["unique_vars_total"] * stage_bytes_per_var(0) + 4 * bt["table_bytes_read_per_stage"]
    out = {
        "metric": "unique-variable RHS updates/s",
        "value": f64["rhs_updates_per_s"],
        "unit": "unique-variable RHS updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batched draw: 512 independent problems (seed 0), N~U{4..5000}, m~U{1..4}, "
                               "L~U{3..10}, g~U[0.002,0.03], lam~U[0.005,0.05], gam~U[0.02,0.2], "
                               "kappa~U[0,0.02], kT=0.025, resonant, d=0, rho(0)=|c><c|, dt=0.02",
                   "instances": bt["instances"], "unique_vars_total": bt["unique_vars_total"],
                   "rhs_per_step": 4, "precision": "fp64", "hermitian_ados": bool(herm),
                   "launch": "heom_batch_propagate (grouped and merged stage launches)",
                   "parallelism": "single GPU"},
        "wall_s": f64["wall_s"],
        "finite": f64["finite"] and f64["nonfinite_slots"] == 0,
        "roofline": {
            "bound": "hbm", "achieved": f64["algorithmic_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": f64["hbm_frac"], "traffic": traffic["bytes_per_launch"] if traffic else None,
            "kernel": "batched RK4 stage kernels (batch_stage_*), FP64; one launch = one RK4 step of every "
                      "problem (its four stages, each one launch per group); timed with HIP events on the "
                      "launch stream over the headline's steps",
            "algorithmic_bytes_per_launch": int(step_bytes),
            "state_bytes_per_var_per_step": stage_bytes_per_var(0),
            "table_bytes_per_stage": bt["table_bytes_read_per_stage"],
            "mean_launch_us": round(f64["ms_per_step"] * 1e3, 1),
            "copy_GBps": copy_gbs,
            "frac_of_copy": round(f64["algorithmic_GBps"] / copy_gbs, 4),
            "element_bytes_per_launch": bt["element_bytes_per_step"],
            "frac_element_bytes": round(bt["element_bytes_per_step"] / (f64["ms_per_step"] * 1e-3) / 1e9
                                        / HBM_PEAK_GBS, 4),
        },
        "batched": bt,
    }
    if args.batched_only:
        print(json.dumps(out), flush=True)
        return
    if not args.no_local:
        out["localized"] = localized_section(torch, args, precision, herm)
        progress("localized workload done")
    if not args.no_roofline:
        out["roofline_probe"] = probe_section(torch, args, herm)
        out["roofline_probe"]["frac_of_copy"] = round(out["roofline_probe"]["achieved"] / copy_gbs, 4)
        progress(f"roofline probe done: {out['roofline_probe']['mean_launch_us']} us per stage")
    if not args.no_serve:
        out["serving"] = []
        for spec in [x for x in args.serve_rates.split(",") if x]:
            r, w, d = (float(v) for v in spec.split(":"))
            out["serving"].append(serving_point(torch, r, w, d, precision=serve_prec, flag=herm))
            progress(f"serving point at {r} req/s done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(0.02, args.cpu_var_budget, args.cpu_max_vars, steps=args.cpu_steps)
        out["cpu_baseline"]["speedup_gpu_over_cpu"] = round(out["value"] / out["cpu_baseline"]["value"], 1)
        progress("CPU baseline done")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
