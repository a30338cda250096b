"""GPU tests of the transposed copies (heom_tuning.transposed).

With the copies on, every stage also writes its output with each block's
category matrix transposed, and the column-molecule moves gather from that
copy. The copy holds the same values and every variable sums its terms in
the same order, so right-hand sides and trajectories must be bitwise those
without copies; one right-hand side per case is also checked against the
CPU oracle directly.
"""
import numpy as np
import pytest

from oracle import uvar
from paper_2608_20657_amd import workloads as W
from tests.gpu_util import gpu_propagate, gpu_rhs, named_tier0, rhs_bound, torch_cuda

pytestmark = pytest.mark.gpu

CASES = [(5, 2, 3, 1, "site1", False), (7, 3, 3, 0, "photon", True), (4, 1, 2, 2, "site1", True),
         (6, 5, 2, 0, "photon", False), (64, 2, 6, 1, "site1", False), (3, 2, 4, 1, "site1", True)]


def tables(p, transposed, tile_vars=0):
    torch = torch_cuda()
    from paper_2608_20657_amd import heom
    T = heom.Tables(p)
    kw = {"transposed": transposed}
    if tile_vars:
        kw["tile_vars"] = tile_vars
    T.set_tuning(**kw)
    info = T.info()
    if transposed >= 0:
        assert info["transposed"] == transposed
    assert info["rhs_work_bytes"] == (16 * info["n_var"] if info["transposed"] else 0)
    buf = torch.empty(info["table_bytes"], dtype=torch.uint8, device="cuda")
    T.upload(buf, torch.cuda.current_stream())
    return T, torch


def problem(N, m, L, d, cc):
    return W.random_problem(N, m, L, d, seed=N * 7 + m + L, complex_check=cc, loss=True, terminator=True)


@pytest.mark.parametrize("N,m,L,d,state,cc", CASES)
def test_rhs_transposed_bitwise_and_vs_oracle(N, m, L, d, state, cc):
    p = problem(N, m, L, d, cc)
    S = uvar.UVarSystem(p)
    y = W.random_vector(S.n_var, seed=N + L)
    T0, torch = tables(p, 0, tile_vars=64)
    T1, _ = tables(p, 1, tile_vars=64)
    a, b = gpu_rhs(T0, torch, y), gpu_rhs(T1, torch, y)
    assert np.array_equal(a.view(np.float64), b.view(np.float64))
    A = S.generator()
    assert np.all(np.abs(b - A @ y) <= rhs_bound(A, y))


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("N,m,L,d,state,cc", CASES)
def test_propagate_transposed_bitwise(N, m, L, d, state, cc, precision):
    p = problem(N, m, L, d, cc)
    out = []
    for tr in (0, 1):
        T, torch = tables(p, tr, tile_vars=64)
        out.append(gpu_propagate(T, torch, named_tier0(T, p, state), 0.05, 23, 5, precision))
    (y0, o0), (y1, o1) = out
    assert np.array_equal(y0.view(np.float64), y1.view(np.float64))
    assert np.array_equal(o0, o1)


@pytest.mark.parametrize("precision", [0, 1])
def test_large_state_default_copies_bitwise(precision):
    """1.56 M variables: copies on by default, top tier in its own launch."""
    p = W.random_problem(100, 4, 8, 0, seed=3)
    T1, torch = tables(p, -1)
    assert T1.info()["transposed"] == 1 and T1.info()["n_tiles"] >= 2048
    T0, _ = tables(p, 0)
    t0 = named_tier0(T1, p, "photon")
    y1, o1 = gpu_propagate(T1, torch, t0, 0.02, 6, 3, precision)
    y0, o0 = gpu_propagate(T0, torch, t0, 0.02, 6, 3, precision)
    assert np.array_equal(y0.view(np.float64), y1.view(np.float64))
    assert np.array_equal(o0, o1)
    yr = W.random_vector(T1.info()["n_var"], seed=5)
    assert np.array_equal(gpu_rhs(T0, torch, yr).view(np.float64), gpu_rhs(T1, torch, yr).view(np.float64))


def test_batch_mixes_slots_with_and_without_copies():
    """A batch of slots with and without copies equals their solo runs."""
    from paper_2608_20657_amd import heom
    torch = torch_cuda()
    s = torch.cuda.current_stream()
    probs = [(5, 2, 3, 1, "site1", False, 1), (7, 3, 3, 0, "photon", True, 0), (64, 2, 6, 1, "site1", False, 1)]
    steps, every, dt = 17, 4, 0.05
    for precision in (0, 1):
        b = heom.Batch(len(probs))
        keep, want = [], []
        for i, (N, m, L, d, state, cc, tr) in enumerate(probs):
            p = problem(N, m, L, d, cc)
            T, _ = tables(p, tr, tile_vars=64)
            t0 = named_tier0(T, p, state)
            want.append(gpu_propagate(T, torch, t0, dt, steps, every, precision))
            info = T.info()
            y = torch.empty(info["n_var"], dtype=torch.complex128, device="cuda")
            T.init_state(t0, y, s)
            work = torch.empty(info["work_bytes_fp64"], dtype=torch.uint8, device="cuda")
            obs = torch.zeros((steps // every + 1) * 10, dtype=torch.float64, device="cuda")
            b.set_slot(i, T, y, work, dt, obs=obs, obs_every=every)
            keep.append((T, y, work, obs))
        b.commit(torch, s)
        b.propagate(steps, precision, s)
        torch.cuda.synchronize()
        for (T, y, work, obs), (wy, wo) in zip(keep, want):
            assert np.array_equal(y.cpu().numpy().view(np.float64), wy.view(np.float64))
            assert np.array_equal(obs.cpu().numpy().reshape(-1, 10), wo)


# Hermitian ADOs (HEOM_HERMITIAN): column gathers read the conjugated mirrored
# entry of the row-major state itself. The mirrored entries are computed by
# different threads, so results agree with the general path to rounding.
HERM = [(5, 2, 3, 1, "site1"), (7, 3, 3, 0, "photon"), (4, 1, 2, 2, "site1"), (64, 2, 6, 1, "upper_polariton"),
        (6, 5, 2, 0, "photon")]


def herm_problem(N, m, L, d):
    return W.random_problem(N, m, L, d, seed=N * 5 + m + L, complex_check=False, loss=True, terminator=True)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("N,m,L,d,state", HERM)
def test_hermitian_mirror_matches_general(N, m, L, d, state, precision):
    from paper_2608_20657_amd import heom
    p = herm_problem(N, m, L, d)
    Tg, torch = tables(p, 0, tile_vars=64)
    Th, _ = tables(p, 1, tile_vars=64)
    t0 = named_tier0(Tg, p, state)
    yg, og = gpu_propagate(Tg, torch, t0, 0.05, 23, 5, precision)
    yh, oh = gpu_propagate(Th, torch, t0, 0.05, 23, 5, precision | heom.HEOM_HERMITIAN)
    tol = 1e-12 if precision == 0 else 1e-6
    scale = np.abs(yg).max()
    assert np.abs(yh - yg).max() <= tol * scale
    assert np.abs(oh - og).max() <= tol * max(1.0, np.abs(og).max())
    # the flag is ignored by tables without transposed copies: bitwise the general path
    yn, on = gpu_propagate(Tg, torch, t0, 0.05, 23, 5, precision | heom.HEOM_HERMITIAN)
    assert np.array_equal(yn.view(np.float64), yg.view(np.float64)) and np.array_equal(on, og)


def two_steps_from_random_hermitian(p, variants, seed=7, dt=0.02):
    """Two RK4 steps from the same seeded random Hermitian state (every tier
    populated, entries of order one) on several table variants; returns the
    initial state and each variant's result (variants: (tuning, precision))."""
    from tests.gpu_util import hermitian_vector
    torch = torch_cuda()
    S = uvar.UVarSystem(p)
    y0 = hermitian_vector(S, seed)
    s = torch.cuda.current_stream()
    out = []
    for tuning, prec in variants:
        from paper_2608_20657_amd import heom
        T = heom.Tables(p)
        T.set_tuning(**tuning)
        info = T.info()
        img = torch.empty(info["table_bytes"], dtype=torch.uint8, device="cuda")
        T.upload(img, s)
        y = torch.from_numpy(y0).to("cuda")
        work = torch.empty(info["work_bytes_fp64"], dtype=torch.uint8, device="cuda")
        T.propagate(y, work, dt, 2, 0, None, prec, s)
        T.work_status(work, s)
        out.append(y.cpu().numpy())
        del img, y, work
    return y0, out


def assert_close_per_element(a, b, y0, rel):
    """|a - b| <= rel (|b| + |y0|) entry by entry: rounding differences of a
    few RK4 stages from an order-one start; a wrong term of any tier moves
    its entries by far more."""
    err = np.abs(a - b)
    bound = rel * (np.abs(b) + np.abs(y0))
    assert np.all(err <= bound), f"worst ratio {(err / bound).max():.3g}"


def test_hermitian_mirror_large_state():
    """1.56 M variables (transposed targets by default, top tier in its own
    launch): from a random Hermitian state, two steps with mirrored column
    gathers equal two general steps (transposed copy) entry by entry, FP64
    and FP32 increments."""
    from paper_2608_20657_amd import heom
    p = W.random_problem(100, 4, 8, 0, seed=3)
    for prec, rel in ((0, 1e-12), (1, 1e-6)):
        y0, (yg, yh) = two_steps_from_random_hermitian(
            p, [(dict(transposed=1), prec), (dict(transposed=1), prec | heom.HEOM_HERMITIAN)])
        assert_close_per_element(yh, yg, y0, rel)


def test_hermitian_flag_needs_adjoint_preserving_bath():
    from paper_2608_20657_amd import heom
    p = W.random_problem(5, 2, 3, 1, seed=2, complex_check=True)
    T, torch = tables(p, 1, tile_vars=64)
    with pytest.raises(heom.HeomError) as e:
        gpu_propagate(T, torch, named_tier0(T, p, "site1"), 0.05, 3, 1, heom.HEOM_HERMITIAN)
    assert e.value.code == -1


def test_batch_hermitian_equals_solo():
    """Batch slots with and without transposed tables, Hermitian flag: each
    equals its own heom_propagate run with the flag, bitwise."""
    from paper_2608_20657_amd import heom
    torch = torch_cuda()
    s = torch.cuda.current_stream()
    probs = [(5, 2, 3, 1, "site1", 1), (7, 3, 3, 0, "photon", 0), (64, 2, 6, 1, "site1", 1)]
    steps, every, dt = 17, 4, 0.05
    for precision in (0, 1):
        flag = precision | heom.HEOM_HERMITIAN
        b = heom.Batch(len(probs))
        keep, want = [], []
        for i, (N, m, L, d, state, tr) in enumerate(probs):
            p = herm_problem(N, m, L, d)
            T, _ = tables(p, tr, tile_vars=64)
            t0 = named_tier0(T, p, state)
            want.append(gpu_propagate(T, torch, t0, dt, steps, every, flag))
            info = T.info()
            y = torch.empty(info["n_var"], dtype=torch.complex128, device="cuda")
            T.init_state(t0, y, s)
            work = torch.empty(info["work_bytes_fp64"], dtype=torch.uint8, device="cuda")
            obs = torch.zeros((steps // every + 1) * 10, dtype=torch.float64, device="cuda")
            b.set_slot(i, T, y, work, dt, obs=obs, obs_every=every)
            keep.append((T, y, work, obs))
        b.commit(torch, s)
        b.propagate(steps, flag, s)
        torch.cuda.synchronize()
        for (T, y, work, obs), (wy, wo) in zip(keep, want):
            assert np.array_equal(y.cpu().numpy().view(np.float64), wy.view(np.float64))
            assert np.array_equal(obs.cpu().numpy().reshape(-1, 10), wo)


# Compact tiles (heom_tuning.compact): threads cover only each block's upper
# triangle and T_q, write the mirrored entry as the conjugate, and take the
# column sums as conjugates of the row sums. Hermitian ADOs only.
def compact_tables(p, tile_vars=0):
    torch = torch_cuda()
    from paper_2608_20657_amd import heom
    T = heom.Tables(p)
    kw = {"compact": 1}
    if tile_vars:
        kw["tile_vars"] = tile_vars
    T.set_tuning(**kw)
    info = T.info()
    assert info["compact"] == 1 and info["transposed"] == 1 and info["rhs_work_bytes"] == 0
    buf = torch.empty(info["table_bytes"], dtype=torch.uint8, device="cuda")
    T.upload(buf, torch.cuda.current_stream())
    return T, torch


@pytest.mark.parametrize("tile_vars", [64, 256])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("N,m,L,d,state", HERM)
def test_compact_matches_general(N, m, L, d, state, precision, tile_vars):
    from paper_2608_20657_amd import heom
    p = herm_problem(N, m, L, d)
    Tg, torch = tables(p, 0, tile_vars=64)
    Tc, _ = compact_tables(p, tile_vars=tile_vars)
    t0 = named_tier0(Tg, p, state)
    yg, og = gpu_propagate(Tg, torch, t0, 0.05, 23, 5, precision)
    yc, oc = gpu_propagate(Tc, torch, t0, 0.05, 23, 5, precision | heom.HEOM_HERMITIAN)
    tol = 1e-12 if precision == 0 else 1e-6
    assert np.abs(yc - yg).max() <= tol * np.abs(yg).max()
    assert np.abs(oc - og).max() <= tol * max(1.0, np.abs(og).max())


def test_compact_large_state():
    """1.56 M variables on compact tiles (>= 2048 tiles, split top tier): two
    steps from a random Hermitian state equal two general steps entry by
    entry, FP64 and FP32 increments."""
    from paper_2608_20657_amd import heom
    p = W.random_problem(100, 4, 8, 0, seed=3)
    for prec, rel in ((0, 1e-12), (1, 1e-6)):
        y0, (yg, yc) = two_steps_from_random_hermitian(
            p, [(dict(transposed=1), prec), (dict(compact=1), prec | heom.HEOM_HERMITIAN)])
        assert_close_per_element(yc, yg, y0, rel)


def test_compact_needs_hermitian_flag():
    from paper_2608_20657_amd import heom
    p = herm_problem(5, 2, 3, 1)
    Tc, torch = compact_tables(p, tile_vars=64)
    t0 = named_tier0(Tc, p, "site1")
    with pytest.raises(heom.HeomError) as e:
        gpu_propagate(Tc, torch, t0, 0.05, 3, 1, 0)
    assert e.value.code == -7
    with pytest.raises(heom.HeomError) as e:
        gpu_rhs(Tc, torch, W.random_vector(Tc.info()["n_var"], seed=1))
    assert e.value.code == -7


def test_batch_compact_equals_solo():
    """Compact and full slots in one batch, Hermitian flag: each slot equals
    its own heom_propagate run, bitwise."""
    from paper_2608_20657_amd import heom
    torch = torch_cuda()
    s = torch.cuda.current_stream()
    probs = [(5, 2, 3, 1, "site1", "compact"), (7, 3, 3, 0, "photon", "full"),
             (64, 2, 6, 1, "site1", "compact"), (6, 5, 2, 0, "photon", "transposed")]
    steps, every, dt = 17, 4, 0.05
    for precision in (0, 1):
        flag = precision | heom.HEOM_HERMITIAN
        b = heom.Batch(len(probs))
        keep, want = [], []
        for i, (N, m, L, d, state, kind) in enumerate(probs):
            p = herm_problem(N, m, L, d)
            T, _ = compact_tables(p, 64) if kind == "compact" else tables(p, 1 if kind == "transposed" else 0, 64)
            t0 = named_tier0(T, p, state)
            want.append(gpu_propagate(T, torch, t0, dt, steps, every, flag))
            info = T.info()
            y = torch.empty(info["n_var"], dtype=torch.complex128, device="cuda")
            T.init_state(t0, y, s)
            work = torch.empty(info["work_bytes_fp64"], dtype=torch.uint8, device="cuda")
            obs = torch.zeros((steps // every + 1) * 10, dtype=torch.float64, device="cuda")
            b.set_slot(i, T, y, work, dt, obs=obs, obs_every=every)
            keep.append((T, y, work, obs))
        b.commit(torch, s)
        with pytest.raises(heom.HeomError):
            b.propagate(1, precision, s)        # compact slots need the flag
        b.propagate(steps, flag, s)
        torch.cuda.synchronize()
        for (T, y, work, obs), (wy, wo) in zip(keep, want):
            assert np.array_equal(y.cpu().numpy().view(np.float64), wy.view(np.float64))
            assert np.array_equal(obs.cpu().numpy().reshape(-1, 10), wo)


def test_compact_probe_size_matches_general():
    """At the roofline probe's full size (17.3 M variables), the benchmarked
    configuration: two FP64 steps on compact tiles under HEOM_HERMITIAN from a
    random Hermitian state (every tier populated) equal two general steps
    (full tiles, transposed copy) entry by entry."""
    from paper_2608_20657_amd import heom
    p = W.config_roofline_probe()
    y0, (yg, yc) = two_steps_from_random_hermitian(
        p, [(dict(transposed=1), 0), (dict(compact=1), heom.HEOM_HERMITIAN)], seed=9)
    assert np.isfinite(yg).all()
    assert_close_per_element(yc, yg, y0, 1e-12)
