"""GPU tests of batches of independent problems (heom_batch_*).

Each problem's trajectory in a batch must be bitwise the one heom_propagate
gives it alone; problems of one structure key may share one uploaded
structure with their own parameter blocks; slots can be replaced between
steps (continuous batching) without disturbing the others. The solo runs
are themselves parity-tested against the CPU oracle (test_gpu_parity.py);
here one batched problem per kind is also checked against the oracle
directly.
"""
import math

import numpy as np
import pytest

from oracle import integrate, observables as O, uvar
from paper_2608_20657_amd import workloads as W
from tests.gpu_util import gpu_propagate, named_tier0, torch_cuda, upload

pytestmark = pytest.mark.gpu


def make_slot(T, torch, tier0, every, cap):
    info = T.info()
    y = torch.empty(info["n_var"], dtype=torch.complex128, device="cuda")
    T.init_state(tier0, y, torch.cuda.current_stream())
    work = torch.empty(info["work_bytes_fp64"], dtype=torch.uint8, device="cuda")
    obs = torch.zeros(cap * 10, dtype=torch.float64, device="cuda")
    return y, work, obs


def solo(T, torch, tier0, dt, steps, every, precision):
    info = T.info()
    s = torch.cuda.current_stream()
    y = torch.empty(info["n_var"], dtype=torch.complex128, device="cuda")
    T.init_state(tier0, y, s)
    work = torch.empty(info["work_bytes_fp64"], dtype=torch.uint8, device="cuda")
    obs = torch.zeros((steps // every + 1) * 10, dtype=torch.float64, device="cuda")
    T.propagate(y, work, dt, steps, every, obs, precision, s)
    torch.cuda.synchronize()
    return y.cpu().numpy(), obs.cpu().numpy().reshape(-1, 10)


# the last one has launches of its own in a batch (>= 4096 tiles) and runs
# its top tier with the top-tier kernel variant (>= 2048 tiles)
PROBS = [(5, 2, 3, 1, "site1"), (9, 1, 5, 0, "upper_polariton"), (7, 3, 3, 0, "photon"),
         (64, 2, 6, 1, "site1"), (12, 4, 3, 0, "photon"), (4, 1, 2, 2, "site1"), (6, 5, 2, 0, "photon"),
         (10000, 3, 8, 0, "upper_polariton"), (100, 4, 8, 0, "photon")]


@pytest.mark.parametrize("precision,merge", [(0, 16384), (1, 16384), (0, 0), (1, 0), (0, 40)])
def test_batch_equals_solo(precision, merge):
    """merge 16384: the groups with m <= 4 run as one launch per stage, the
    m = 5 group on its own; merge 0: one launch per group; merge 40: only
    the smallest groups are merged."""
    from paper_2608_20657_amd import heom
    import torch
    steps, every = 37, 5
    batch = heom.Batch(len(PROBS) + 2)
    batch.set_merge(merge)
    items = []
    for i, (N, m, L, d, state) in enumerate(PROBS):
        p = W.random_problem(N, m, L, d, seed=i + 1, loss=True)
        T, torch = upload(p)
        t0 = named_tier0(T, p, state)
        dt = 0.02 + 0.005 * i
        y, work, obs = make_slot(T, torch, t0, every, steps // every + 1)
        batch.set_slot((3 * i + 1) % (len(PROBS) + 2), T, y, work, dt, obs=obs, obs_every=every)
        items.append((T, p, t0, dt, y, obs))
    batch.commit(torch, torch.cuda.current_stream())
    batch.propagate(steps, precision, torch.cuda.current_stream())
    torch.cuda.synchronize()
    for T, p, t0, dt, y, obs in items:
        ys, os_ = solo(T, torch, t0, dt, steps, every, precision)
        assert np.array_equal(y.cpu().numpy(), ys)
        ob = obs.cpu().numpy().reshape(-1, 10)
        assert np.array_equal(ob, os_)


def test_batch_shared_structure_params():
    from paper_2608_20657_amd import heom
    import torch
    s = torch.cuda.current_stream()
    base = W.config_saturated()
    base.N = 40                                   # saturated structure (N >= L + 2)
    Tshared, torch = upload(base)
    batch = heom.Batch(3)
    runs = []
    for i, N in enumerate((40, 1000, 10 ** 6)):
        p = W.config_saturated()
        p.N = N
        p.g = 0.005 * (1 + i)
        p.c = [z * (1 + 0.1 * i) for z in p.c]
        p.c_check = [z.conjugate() for z in p.c]
        params = torch.empty(Tshared.params_bytes(), dtype=torch.uint8, device="cuda")
        Tshared.upload_params(p, params, s)
        Tp, _ = upload(p)                         # the same problem with its own tables
        t0 = named_tier0(Tp, p, "upper_polariton")
        y, work, obs = make_slot(Tshared, torch, t0, 4, 6)
        batch.set_slot(i, Tshared, y, work, 0.02, params=params, obs=obs, obs_every=4)
        runs.append((Tp, p, t0, y, obs))
    batch.commit(torch, s)
    batch.propagate(20, 0, s)
    torch.cuda.synchronize()
    for Tp, p, t0, y, obs in runs:
        ys, os_ = solo(Tp, torch, t0, 0.02, 20, 4, 0)
        assert np.array_equal(y.cpu().numpy(), ys)
        assert np.array_equal(obs.cpu().numpy().reshape(-1, 10), os_)


def test_continuous_batching_replace_slots():
    from paper_2608_20657_amd import heom
    import torch
    s = torch.cuda.current_stream()
    batch = heom.Batch(2)
    pa = W.config_localized()
    Ta, torch = upload(pa)
    ta = named_tier0(Ta, pa, "site1")
    ya, wa, oa = make_slot(Ta, torch, ta, 10, 8)
    pb = W.random_problem(6, 3, 3, 0, seed=3)
    Tb, _ = upload(pb)
    tb = named_tier0(Tb, pb, "photon")
    yb, wb, ob = make_slot(Tb, torch, tb, 10, 8)
    batch.set_slot(0, Ta, ya, wa, 0.02, obs=oa, obs_every=10)
    batch.set_slot(1, Tb, yb, wb, 0.02, obs=ob, obs_every=10)
    batch.commit(torch, s)
    batch.propagate(30, 0, s)
    # b finishes; c arrives in its slot while a keeps going
    batch.clear_slot(1)
    pc = W.random_problem(5, 2, 4, 1, seed=4)
    Tc, _ = upload(pc)
    tc = named_tier0(Tc, pc, "site1")
    yc, wc, oc = make_slot(Tc, torch, tc, 10, 8)
    batch.set_slot(1, Tc, yc, wc, 0.03, obs=oc, obs_every=10)
    batch.commit(torch, s)
    batch.propagate(40, 0, s)
    torch.cuda.synchronize()
    assert batch.slot_steps(0) == 70 and batch.slot_steps(1) == 40
    for T, t0, dt, steps, y, obs in ((Ta, ta, 0.02, 70, ya, oa), (Tb, tb, 0.02, 30, yb, ob), (Tc, tc, 0.03, 40, yc, oc)):
        ys, os_ = solo(T, torch, t0, dt, steps, 10, 0)
        assert np.array_equal(y.cpu().numpy(), ys)
        got = obs.cpu().numpy().reshape(-1, 10)
        assert np.array_equal(got[:steps // 10 + 1], os_)


def test_batch_slot_against_oracle():
    from paper_2608_20657_amd import heom
    import torch
    s = torch.cuda.current_stream()
    p = W.random_problem(8, 2, 4, 1, seed=12, loss=True)
    T, torch = upload(p)
    t0 = named_tier0(T, p, "site1")
    y, work, obs = make_slot(T, torch, t0, 10, 21)
    batch = heom.Batch(1)
    batch.set_slot(0, T, y, work, 0.02, obs=obs, obs_every=10)
    batch.commit(torch, s)
    batch.propagate(200, 0, s)
    torch.cuda.synchronize()
    S = uvar.UVarSystem(p)
    y0 = np.zeros(S.n_var, complex)
    y0[:t0.size] = t0
    _, ref = integrate.propagate(S.generator(), y0, 0.02, 200, 10, observe=lambda v: O.from_tier0(S, v))
    ref = np.array(ref)
    got = obs.cpu().numpy().reshape(-1, 10)
    for j in range(9):
        assert np.abs(got[:, j] - ref[:, j]).max() <= 1e-10 * max(np.abs(ref[:, j]).max(), 1e-300)


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replays_equal_direct_launches(precision):
    """Steps replayed from a captured HIP graph give bitwise the states and
    observable rows of direct launches: several replays in a row with other
    device work and synchronizations between them, a remainder launched
    directly, and a re-capture after a slot changes."""
    from paper_2608_20657_amd import heom
    import torch
    stream = torch.cuda.Stream()
    shapes = [(5, 2, 3, 1, "site1"), (9, 1, 5, 0, "upper_polariton"), (64, 2, 6, 1, "site1"), (7, 3, 3, 0, "photon")]
    every, cap = 3, 40
    runs = []
    for graph in (4, 0):
        b = heom.Batch(len(shapes) + 1)
        b.set_graph(graph)
        slots = []
        with torch.cuda.stream(stream):
            for i, (N, m, L, d, state) in enumerate(shapes):
                p = W.random_problem(N, m, L, d, seed=40 + i, loss=True)
                T, _ = upload(p)
                t0 = named_tier0(T, p, state)
                y, work, obs = make_slot(T, torch, t0, every, cap)
                b.set_slot(i, T, y, work, 0.02, obs=obs, obs_every=every)
                slots.append((T, y, obs))
        torch.cuda.synchronize()
        b.commit(torch, stream)
        runs.append((b, slots))
    scratch = torch.ones(1 << 20, dtype=torch.float64, device="cuda")
    for rep in range(3):
        for b, _ in runs:
            b.propagate(9, precision, stream)          # two replays of four steps and one direct step
        stream.synchronize()
        scratch.mul_(1.5).add_(rep)                    # other device work between the replays
        torch.cuda.synchronize()
        for sa, sb in zip(runs[0][1], runs[1][1]):
            assert np.array_equal(sa[1].cpu().numpy(), sb[1].cpu().numpy()), rep
            assert np.array_equal(sa[2].cpu().numpy(), sb[2].cpu().numpy()), rep
    # a new slot: both batches re-commit (the graph is captured again) and go on
    p = W.random_problem(6, 2, 4, 0, seed=77, loss=True)
    extra = []
    for b, slots in runs:
        T, _ = upload(p)
        t0 = named_tier0(T, p, "photon")
        with torch.cuda.stream(stream):
            y, work, obs = make_slot(T, torch, t0, every, cap)
        torch.cuda.synchronize()
        b.set_slot(len(shapes), T, y, work, 0.03, obs=obs, obs_every=every)
        b.commit(torch, stream)
        b.propagate(13, precision, stream)
        extra.append((y, obs))
    stream.synchronize()
    for sa, sb in zip(runs[0][1], runs[1][1]):
        assert np.array_equal(sa[1].cpu().numpy(), sb[1].cpu().numpy())
        assert np.array_equal(sa[2].cpu().numpy(), sb[2].cpu().numpy())
    assert np.array_equal(extra[0][0].cpu().numpy(), extra[1][0].cpu().numpy())
    assert np.array_equal(extra[0][1].cpu().numpy(), extra[1][1].cpu().numpy())
    assert runs[0][0].slot_steps(2) == 40 and runs[0][0].slot_steps(len(shapes)) == 13
    # the graph-replayed trajectory is the solo one
    T, y, obs = runs[0][1][1]
    t0 = named_tier0(T, T.problem, "upper_polariton")
    ys, os_ = solo(T, torch, t0, 0.02, 40, every, precision)
    assert np.array_equal(y.cpu().numpy(), ys)
    assert np.array_equal(obs.cpu().numpy().reshape(-1, 10)[:40 // every + 1], os_)


def test_commit_resolves_retuned_tables_and_refuses_stale_params():
    """A slot's tables re-tuned and re-uploaded into a new buffer after
    heom_batch_set_slot: commit takes the new image (slot without its own
    parameter block), refuses a parameter block written for the old tiles
    (E_STATE), accepts it once written again; the results then equal solo
    runs bitwise."""
    from paper_2608_20657_amd import heom
    torch = torch_cuda()
    s = torch.cuda.current_stream()
    p = W.config_localized()
    steps, dt = 12, 0.02
    T = heom.Tables(p)
    T.set_tuning(tile_vars=64)
    img = torch.empty(T.info()["table_bytes"], dtype=torch.uint8, device="cuda")
    T.upload(img, s)
    t0 = T.tier0_pure(0.0, 0.0, [1.0])
    params = torch.empty(4096 * ((T.params_bytes() + 4095) // 4096), dtype=torch.uint8, device="cuda")
    q = W.config_localized()
    q.N, q.g = 300, 0.013
    T.upload_params(q, params, s)
    b = heom.Batch(2)
    ys = []
    for i, prm in enumerate((None, params)):
        y = torch.empty(T.info()["n_var"], dtype=torch.complex128, device="cuda")
        T.init_state(t0, y, s)
        work = torch.empty(2 * T.info()["work_bytes_fp64"], dtype=torch.uint8, device="cuda")
        b.set_slot(i, T, y, work, dt, params=prm)
        ys.append((y, work))
    # re-tune (new tiles, new layout) and upload into a new buffer; the old one is freed
    T.set_tuning(tile_vars=256)
    img2 = torch.empty(T.info()["table_bytes"], dtype=torch.uint8, device="cuda")
    T.upload(img2, s)
    del img
    torch.cuda.empty_cache()
    with pytest.raises(heom.HeomError) as e:
        b.commit(torch, s)
    assert e.value.code == -7
    T.upload_params(q, params, s)
    b.commit(torch, s)
    b.propagate(steps, 0, s)
    torch.cuda.synchronize()
    # solo runs on the re-tuned tables: the tables' own parameters, then q's
    want0, _ = gpu_propagate(T, torch, t0, dt, steps, 0)
    T.set_params(q)
    img3 = torch.empty(T.info()["table_bytes"], dtype=torch.uint8, device="cuda")
    T.upload(img3, s)
    want1, _ = gpu_propagate(T, torch, t0, dt, steps, 0)
    assert np.array_equal(ys[0][0].cpu().numpy(), want0)
    assert np.array_equal(ys[1][0].cpu().numpy(), want1)


def test_hermitian_flag_checked_per_slot():
    """HEOM_HERMITIAN on a batch whose slot parameters have c_check != conj(c)
    is refused (E_INVAL), as heom_propagate refuses it."""
    from paper_2608_20657_amd import heom
    torch = torch_cuda()
    s = torch.cuda.current_stream()
    p = W.random_problem(5, 2, 3, 1, seed=2, complex_check=False)
    bad = W.random_problem(5, 2, 3, 1, seed=2, complex_check=True)
    T = heom.Tables(p)
    img = torch.empty(T.info()["table_bytes"], dtype=torch.uint8, device="cuda")
    T.upload(img, s)
    params = torch.empty(4096 * ((T.params_bytes() + 4095) // 4096), dtype=torch.uint8, device="cuda")
    T.upload_params(bad, params, s)
    b = heom.Batch(2)
    keep = []
    for i, prm in enumerate((None, params)):
        y = torch.empty(T.info()["n_var"], dtype=torch.complex128, device="cuda")
        T.init_state(T.tier0_pure(0.0, 0.0, [1.0]), y, s)
        work = torch.empty(T.info()["work_bytes_fp64"], dtype=torch.uint8, device="cuda")
        b.set_slot(i, T, y, work, 0.02, params=prm)
        keep.append((y, work))
    b.commit(torch, s)
    with pytest.raises(heom.HeomError) as e:
        b.propagate(2, heom.HEOM_HERMITIAN, s)
    assert e.value.code == -1
    b.propagate(2, 0, s)                 # the general path is fine
    b.clear_slot(1)
    b.commit(torch, s)
    b.propagate(2, heom.HEOM_HERMITIAN, s)
    torch.cuda.synchronize()


@pytest.mark.parametrize("share,interleave", [(1, 0), (2, 0), (1, 3), (2, 3)])
def test_shared_structure_slots_equal_solo(share, interleave):
    """Slots on one uploaded structure with their own parameter blocks
    (different N beyond saturation, couplings, loss; every other slot without
    observables), computed in pairs side by side (one tile's metadata staged
    once for both halves of a workgroup) with an odd slot out, or one
    workgroup per slot with the slots of a structure taking turns three tiles
    at a time, beside slots of another structure: every slot equals its
    heom_propagate run bitwise, FP64 and FP32 increments, plain and compact
    tiles."""
    from paper_2608_20657_amd import heom
    torch = torch_cuda()
    s = torch.cuda.current_stream()
    steps, every, dt = 9, 3, 0.02
    base = [W.config_localized(), W.config_saturated()]
    for compact in (0, 1):
        for precision in (0, 1):
            flag = precision | (heom.HEOM_HERMITIAN if compact else 0)
            b = heom.Batch(8)
            b.set_merge(0)
            b.set_share(share)
            b.set_interleave(interleave)
            keep, want = [], []
            structs = []
            for bp in base:
                T = heom.Tables(bp)
                T.set_tuning(compact=compact)
                img = torch.empty(T.info()["table_bytes"], dtype=torch.uint8, device="cuda")
                T.upload(img, s)
                structs.append((T, img))
            slot = 0
            for si, (T, img) in enumerate(structs):
                for j in range(4 if si == 0 else 3):
                    q = (W.config_localized if si == 0 else W.config_saturated)()
                    q.N = q.N + 37 * j
                    q.g = q.g * (1 + 0.1 * j)
                    q.kappa = 0.003 * j
                    params = torch.empty(4096 * ((T.params_bytes() + 4095) // 4096), dtype=torch.uint8,
                                         device="cuda")
                    T.upload_params(q, params, s)
                    t0 = T.tier0_pure(0.0, 0.0, [1.0]) if si == 0 else T.tier0_pure(0.6, 0.8 / math.sqrt(q.N))
                    info = T.info()
                    y = torch.empty(info["n_var"], dtype=torch.complex128, device="cuda")
                    T.init_state(t0, y, s)
                    work = torch.empty(info["work_bytes_fp64"], dtype=torch.uint8, device="cuda")
                    ev = every if slot % 2 == 0 else 0
                    obs = torch.zeros((steps // every + 1) * 10, dtype=torch.float64, device="cuda")
                    b.set_slot(slot, T, y, work, dt, params=params, obs=obs if ev else None, obs_every=ev)
                    keep.append((y, obs, params))
                    # solo: the same problem on its own tables
                    Ts = heom.Tables(q)
                    Ts.set_tuning(compact=compact)
                    imgs = torch.empty(Ts.info()["table_bytes"], dtype=torch.uint8, device="cuda")
                    Ts.upload(imgs, s)
                    wy, wo = gpu_propagate(Ts, torch, t0, dt, steps, ev, flag)
                    want.append((wy, wo if ev else np.zeros((steps // every + 1, 10))))
                    slot += 1
            b.commit(torch, s)
            b.propagate(steps, flag, s)
            torch.cuda.synchronize()
            for (y, obs, _), (wy, wo) in zip(keep, want):
                assert np.array_equal(y.cpu().numpy().view(np.float64), wy.view(np.float64)), (compact, precision)
                assert np.array_equal(obs.cpu().numpy().reshape(-1, 10), wo), (compact, precision)


def test_one_slot_batch_across_calls_and_graph():
    """A batch of one slot (its own parameter block, observable rows every 5
    steps) runs heom_propagate's launches: bitwise the solo run, across calls
    of 7 and 8 steps; then graph replays of the batch kernels continue the
    same trajectory and rows; then a second slot joins (commit) and the first
    keeps going, still bitwise the solo run."""
    from paper_2608_20657_amd import heom
    torch = torch_cuda()
    s = torch.cuda.current_stream()
    base = W.config_localized()
    q = W.config_localized()
    q.N, q.g, q.kappa = 200, 0.012, 0.002
    T = heom.Tables(base)
    img = torch.empty(T.info()["table_bytes"], dtype=torch.uint8, device="cuda")
    T.upload(img, s)
    params = torch.empty(4096 * ((T.params_bytes() + 4095) // 4096), dtype=torch.uint8, device="cuda")
    T.upload_params(q, params, s)
    t0 = T.tier0_pure(0.0, 0.0, [1.0])
    info = T.info()
    total, every = 7 + 8 + 8 + 6, 5
    y = torch.empty(info["n_var"], dtype=torch.complex128, device="cuda")
    T.init_state(t0, y, s)
    work = torch.empty(info["work_bytes_fp64"], dtype=torch.uint8, device="cuda")
    obs = torch.zeros((total // every + 1) * 10, dtype=torch.float64, device="cuda")
    b = heom.Batch(2)
    b.set_slot(0, T, y, work, 0.02, params=params, obs=obs, obs_every=every)
    b.commit(torch, s)
    b.propagate(7, 0, s)
    b.propagate(8, 0, s)
    b.set_graph(4)
    b.propagate(8, 0, s)                      # two graph replays of the batch kernels
    b.set_graph(0)
    y2 = torch.empty(info["n_var"], dtype=torch.complex128, device="cuda")
    T.init_state(t0, y2, s)
    work2 = torch.empty(info["work_bytes_fp64"], dtype=torch.uint8, device="cuda")
    b.set_slot(1, T, y2, work2, 0.02)
    b.commit(torch, s)
    b.propagate(6, 0, s)
    torch.cuda.synchronize()
    Tq = heom.Tables(q)
    imgq = torch.empty(Tq.info()["table_bytes"], dtype=torch.uint8, device="cuda")
    Tq.upload(imgq, s)
    wy, wo = gpu_propagate(Tq, torch, t0, 0.02, total, every)
    assert b.slot_steps(0) == total
    assert np.array_equal(y.cpu().numpy().view(np.float64), wy.view(np.float64))
    assert np.array_equal(obs.cpu().numpy().reshape(-1, 10), wo)


def test_autotune_batch_restores_states_and_keeps_results():
    """autotune_batch tries merge thresholds, shared workgroups and slot
    interleaving on the committed batch, then restores every slot's state
    and step count: the batch afterwards equals the slots' solo runs
    bitwise."""
    from paper_2608_20657_amd import autotune, heom
    torch = torch_cuda()
    s = torch.cuda.current_stream()
    b = heom.Batch(6)
    keep, want = [], []
    steps, every = 9, 3
    for i, (N, m, L, d) in enumerate([(5, 2, 3, 1), (7, 3, 3, 0), (5, 2, 3, 1), (64, 2, 6, 1), (64, 2, 6, 1)]):
        p = W.random_problem(N, m, L, d, seed=40 + i, loss=True)
        T, _ = upload(p)
        t0 = named_tier0(T, p, "site1" if d else "photon")
        want.append(gpu_propagate(T, torch, t0, 0.02, steps, every))
        info = T.info()
        y = torch.empty(info["n_var"], dtype=torch.complex128, device="cuda")
        T.init_state(t0, y, s)
        work = torch.empty(info["work_bytes_fp64"], dtype=torch.uint8, device="cuda")
        obs = torch.zeros((steps // every + 1) * 10, dtype=torch.float64, device="cuda")
        b.set_slot(i, T, y, work, 0.02, obs=obs, obs_every=every)
        keep.append((T, y, obs))
    b.commit(torch, s)
    res = autotune.autotune_batch(b, torch, steps=2, merges=(0, 64), shares=(1, 2), interleaves=(0, 1))
    assert len(res["results"]) == 8 and res["best"] in [c for c, _ in res["results"]]
    b.propagate(steps, 0, s)
    torch.cuda.synchronize()
    for (T, y, obs), (wy, wo) in zip(keep, want):
        assert np.array_equal(y.cpu().numpy().view(np.float64), wy.view(np.float64))
        assert np.array_equal(obs.cpu().numpy().reshape(-1, 10), wo)
