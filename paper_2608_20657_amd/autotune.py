"""Launch-configuration autotuner for heom_propagate and for batches.

`autotune` times a few RK4 steps of the caller's problem for each candidate
launch configuration (workgroup tile size, persistent cooperative kernel or
one launch per stage, XCD-contiguous tile mapping) with HIP events on the
launch stream, and leaves the fastest one set on the tables.
`tune_structure_tiles` does the same over tile sizes for a structure that a
batch will hold, and `autotune_batch` times a committed batch under each
launch shape (merge threshold of its small groups, slots per shared
workgroup) and keeps the fastest. Every configuration computes bitwise
identical results (one writer per output element and a fixed summation order
per element), so tuning never changes numerics.
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


def autotune_batch(batch: "heom.Batch", torch, steps: int = 3, precision: int = heom.HEOM_FP64,
                   merges=(0, 4096, 16384, 65536), shares=(1, 2), interleaves=(32,), repeats: int = 1,
                   verbose: bool = False) -> Dict:
    """Pick the launch shape of a batch: the merge threshold of its small
    groups (heom_batch_set_merge), the slots per shared workgroup
    (heom_batch_set_share) and the chunk in which slots of one structure take
    turns (heom_batch_set_interleave). Times `steps` RK4 steps of every slot for each
    combination with HIP events on the launch stream and keeps the fastest.
    Every shape gives bitwise the same results; tuning advances the states,
    so each slot's state is saved before and restored after, and every slot
    is set again (its step count restarts at 0) and the batch recommitted.
    The slots' buffers are those Batch.set_slot keeps."""
    s = torch.cuda.current_stream()
    saved = {k: (v, v[2].clone()) for k, v in batch._keep.items()}
    dts = dict(batch._dt)
    results = []
    for mg, sh, il in itertools.product(merges, shares, interleaves):
        batch.set_merge(mg)
        batch.set_share(sh)
        batch.set_interleave(il)
        batch.commit(torch, s)
        best = float("inf")
        for r in range(repeats + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            batch.propagate(steps, precision, s)
            e1.record(s)
            torch.cuda.synchronize()
            if r > 0:                       # the first run warms up
                best = min(best, e0.elapsed_time(e1) / steps)
        results.append((dict(merge_tiles=mg, share_slots=sh, interleave=il), best))
        if verbose:
            print(f"autotune_batch merge={mg} share={sh} interleave={il}: {best:.3f} ms/step", flush=True)
    cbest, tbest = min(results, key=lambda x: x[1])
    batch.set_merge(cbest["merge_tiles"])
    batch.set_share(cbest["share_slots"])
    batch.set_interleave(cbest["interleave"])
    for slot, ((tables, params, y, work, obs, every), y0) in saved.items():
        y.copy_(y0)
        batch.set_slot(slot, tables, y, work, dts[slot], params=params, obs=obs, obs_every=every)
    batch.commit(torch, s)
    torch.cuda.synchronize()
    return {"best": cbest, "ms_per_step": tbest, "results": results}


def tune_structure_tiles(tables: "heom.Tables", torch, tier0, dt: float, steps: int = 20,
                         precision: int = heom.HEOM_FP64, tiles=(64, 128, 256, 512)) -> Dict:
    """Tile size of one structure for batches: the single-problem tuner over
    tile sizes with stage launches (a batch runs every structure with stage
    launches), leaving the tables set and uploaded with the fastest size."""
    maxblk = tables.max_block()
    cands = [dict(tile_vars=tv, persistent=0, xcd_map=0) for tv in tiles if tv >= maxblk]
    return autotune(tables, torch, tier0, dt, steps=steps, precision=precision, cands=cands, repeats=1)
