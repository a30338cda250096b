"""Linear reconstruction of general initial operators (Sec. VI.C, Table II).

The oracle's explicit relabeling sum (oracle.relabel) is pinned on the CPU:
the relabeled responses of the symmetry-adapted oracle's representative
propagations add up to the conventional dense HEOM propagated from the same
arbitrary rho_S(0) (no symmetry used at all), and the |c><e_1| response is
the adjoint of the |e_1><c| one exactly when c_check = conj(c). On the GPU,
heom_reconstruct_dense is compared with that oracle entry by entry, and the
whole reconstruction (representatives propagated through the C ABI, dense
output formed on the device) with the conventional oracle.
"""
import numpy as np
import pytest

from oracle import conventional as C, integrate, relabel, uvar
from paper_2608_20657_amd import reconstruct as RC
from paper_2608_20657_amd import workloads as W


def oracle_tier0_trajectory(q, R0, dt, nsteps, every):
    """Representative propagation by the symmetry-adapted oracle; returns the
    slot matrix of its tier-0 block at each output time."""
    S = uvar.UVarSystem(q)
    blk = S.tier0_block()
    y0 = S.initial_state(rho=lambda i, j: R0[i, j])
    ns = q.d + 3

    pa, pb = q.d + 1, q.d + 2

    def slots(y):
        R = np.zeros((ns, ns), dtype=np.complex128)
        for idx, a, b in S.variables(blk):
            R[S.molecule_index(blk, a), S.molecule_index(blk, b)] = y[idx]
        # the second pool molecule has the first one's entries (pool invariance)
        if q.N - q.d >= 1:
            for x in range(ns):
                if x not in (pa, pb):
                    R[pb, x], R[x, pb] = R[pa, x], R[x, pa]
            R[pb, pb] = R[pa, pa]
            R[pb, pa] = R[pa, pb]
        return R

    _, obs = integrate.propagate(S.generator(), y0, dt, nsteps, every, observe=slots)
    return obs


def conventional_rho(p, rho0, dt, nsteps, every):
    A, labels = C.generator(p)
    D = p.N + 1
    y0 = C.initial_vector(rho0, len(labels))
    _, obs = integrate.propagate(A, y0, dt, nsteps, every, observe=lambda v: v[:D * D].reshape(D, D).copy())
    return np.array(obs)


def random_rho(N, seed, hermitian=True):
    rng = np.random.default_rng(seed)
    M = rng.normal(size=(N + 1, N + 1)) + 1j * rng.normal(size=(N + 1, N + 1))
    if hermitian:
        M = M @ M.conj().T
        M /= np.trace(M).real
    return M


def oracle_responses(p, dt, nsteps, every):
    """Slot-matrix trajectories of all five representatives (oracle)."""
    return {name: oracle_tier0_trajectory(RC.with_d(p, d), RC.slot_matrix(d, a, b), dt, nsteps, every)
            for name, d, (a, b) in RC.REPRESENTATIVES if d <= p.N}


@pytest.mark.parametrize("N,m,L,complex_check,hermitian", [
    (3, 1, 3, False, True),
    (4, 2, 2, False, True),
    (3, 1, 3, True, False),
    (2, 1, 4, False, False),
    (1, 1, 3, True, False),
])
def test_oracle_reconstruction_matches_conventional(N, m, L, complex_check, hermitian):
    p = W.random_problem(N, m, L, 0, seed=7 + N + m, complex_check=complex_check, loss=True)
    rho0 = random_rho(N, seed=N * 10 + L, hermitian=hermitian)
    dt, nsteps, every = 0.05, 40, 10
    ref = conventional_rho(p, rho0, dt, nsteps, every)
    resp = oracle_responses(p, dt, nsteps, every)
    scale = np.abs(ref).max()
    for k in range(nsteps // every + 1):
        got = relabel.dense(rho0, {name: tr[k] for name, tr in resp.items()})
        assert np.abs(got - ref[k]).max() <= 1e-12 * scale


@pytest.mark.parametrize("complex_check", [False, True])
def test_oracle_adjoint_response(complex_check):
    """Eq. adjoint-preservation on the oracle: with c_check = conj(c) the
    response to |c><e_1| is the adjoint of the response to |e_1><c|; with an
    independent c_check it is not."""
    p = W.random_problem(3, 2, 3, 1, seed=11, complex_check=complex_check, loss=True)
    ec = oracle_tier0_trajectory(p, RC.slot_matrix(1, 1, 0), 0.05, 30, 10)
    ce = oracle_tier0_trajectory(p, RC.slot_matrix(1, 0, 1), 0.05, 30, 10)
    dev = max(np.abs(b - a.conj().T).max() for a, b in zip(ec, ce))
    if complex_check:
        assert dev > 1e-6
    else:
        assert dev <= 1e-13
    assert RC.adjoint_preserved(p) == (not complex_check)


def test_plan_skips_absent_operator_types():
    p = W.random_problem(3, 1, 2, 0, seed=1)
    rho0 = np.zeros((4, 4), dtype=complex)
    rho0[2, 2] = 1.0                       # a localized excitation only
    need = RC.plan(p, rho0)
    assert {k for k, v in need.items() if v} == {"ee"}
    full = random_rho(3, seed=2, hermitian=False)
    need = RC.plan(p, full)
    assert all(need[k] for k in ("cc", "ec", "ce", "ee", "e12")) and need["ec_for_ce"]
    q = W.random_problem(3, 1, 2, 0, seed=1, complex_check=True)
    assert "ec_for_ce" not in RC.plan(q, full)
    one = np.zeros((2, 2), dtype=complex)
    one[1, 1] = 1.0
    assert not RC.plan(W.random_problem(1, 1, 2, 0, seed=1), one)["e12"]   # N = 1: no pair


def test_pack_slots_layout():
    """The five slot matrices are packed as (re, im) pairs, row-major, in the
    order cc (3x3), ec, ce, ee (4x4), e12 (5x5); absent ones as zeros."""
    rng = np.random.default_rng(0)
    resp = {n: rng.normal(size=(k, k)) + 1j * rng.normal(size=(k, k)) for n, k, _ in RC.PACK}
    R = RC.pack_slots(resp)
    assert R.size == 164
    off = 0
    for name, n, _ in RC.PACK:
        blk = R[off:off + 2 * n * n]
        assert np.array_equal(blk[0::2].reshape(n, n), resp[name].real)
        assert np.array_equal(blk[1::2].reshape(n, n), resp[name].imag)
        off += 2 * n * n
    R2 = RC.pack_slots({"ee": resp["ee"]})
    assert np.count_nonzero(R2[:82]) == 0 and np.count_nonzero(R2[114:]) == 0
    with pytest.raises(ValueError):
        RC.pack_slots({"cc": np.zeros((4, 4))})


def test_reconstruct_dense_argument_errors():
    """Argument errors come back before anything is launched (no GPU needed:
    the pointers below are never dereferenced)."""
    heom = pytest.importorskip("paper_2608_20657_amd.heom", reason="libheom.so not built")
    import ctypes
    R = np.zeros(164)
    dummy = ctypes.c_void_p(16)
    dp = R.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    lib = heom.LIB
    assert heom.reconstruct_work_bytes(0) == 0 and heom.reconstruct_work_bytes(4097) == 0
    assert heom.reconstruct_work_bytes(5) == 16 * (2 * 5 + 4)
    assert lib.heom_reconstruct_dense(0, dummy, dp, 1, dummy, 1 << 20, dummy, None) == -1
    assert lib.heom_reconstruct_dense(4097, dummy, dp, 1, dummy, 1 << 30, dummy, None) == -1
    assert lib.heom_reconstruct_dense(5, None, dp, 1, dummy, 1 << 20, dummy, None) == -1
    assert lib.heom_reconstruct_dense(5, dummy, dp, 64, dummy, 1 << 20, dummy, None) == -1       # unknown bit
    assert lib.heom_reconstruct_dense(5, dummy, dp, 2 | 32, dummy, 1 << 20, dummy, None) == -1   # adjoint without ce
    assert lib.heom_reconstruct_dense(5, dummy, dp, 1, dummy, 16 * 13, dummy, None) == -3        # work too small
    odd = ctypes.c_void_p(24)
    assert lib.heom_reconstruct_dense(5, odd, dp, 1, dummy, 1 << 20, dummy, None) == -1         # misaligned


def random_slots(rng, scale=1.0):
    return {n: scale * (rng.normal(size=(k, k)) + 1j * rng.normal(size=(k, k))) for n, k, _ in RC.PACK}


def gpu_dense(N, rho0, resp, mask):
    import torch
    from paper_2608_20657_amd import heom
    rd = torch.from_numpy(np.ascontiguousarray(rho0)).to("cuda")
    work = torch.empty(heom.reconstruct_work_bytes(N), dtype=torch.uint8, device="cuda")
    out = torch.full((N + 1, N + 1), complex("nan"), dtype=torch.complex128, device="cuda")
    heom.reconstruct_dense(N, rd, RC.pack_slots(resp), mask, work, out, torch.cuda.current_stream())
    return out.cpu().numpy()


def masked(rho0, mask):
    """rho0 with the entries of the types absent from `mask` zeroed (the
    oracle then sums only the present types)."""
    r = rho0.copy()
    D = r.shape[0]
    for a in range(D):
        for b in range(D):
            name, _ = relabel.representative(a, b)
            bit = next(bt for n, _, bt in RC.PACK if n == name)
            if not mask & bit:
                r[a, b] = 0
    return r


@pytest.mark.gpu
@pytest.mark.parametrize("N", [1, 2, 5, 20])
@pytest.mark.parametrize("mask", [31, 1, 2 | 8, 16, 4, 4 | 32, 31 | 32])
def test_reconstruct_dense_vs_oracle(N, mask):
    """heom_reconstruct_dense against the oracle's explicit relabeling sum,
    every entry (N = 20: 441 entries, two workgroups with a ragged tail)."""
    from tests.gpu_util import torch_cuda
    torch_cuda()
    rng = np.random.default_rng(N * 100 + mask)
    rho0 = random_rho(N, seed=N + mask, hermitian=False)
    resp = random_slots(rng)
    want_resp = dict(resp)
    if mask & 32:
        want_resp["ce"] = resp["ec"].conj().T        # the adjoint form; R's ce block must not be read
        resp["ce"] = np.full((4, 4), 1e30 + 1e30j)
    got = gpu_dense(N, rho0, resp, mask)
    ref = relabel.dense(masked(rho0, mask), want_resp)
    bound = 1e-13 * (N + 1) ** 2 * np.abs(rho0).max() * max(np.abs(v).max() for v in want_resp.values())
    assert np.abs(got - ref).max() <= bound


@pytest.mark.gpu
def test_reconstruct_dense_large_sampled():
    """N = 400 (the column sums span two workgroups, the entries 629 with a
    ragged tail): sampled entries, edges and diagonal included, against the
    oracle's sum over all 160,801 terms of each."""
    from tests.gpu_util import torch_cuda
    torch_cuda()
    N = 400
    rng = np.random.default_rng(5)
    rho0 = (rng.normal(size=(N + 1, N + 1)) + 1j * rng.normal(size=(N + 1, N + 1))) / (N + 1)
    resp = random_slots(rng)
    got = gpu_dense(N, rho0, resp, 31)
    picks = [(0, 0), (0, 1), (0, N), (1, 0), (N, 0), (1, 1), (N, N), (1, 2), (2, 1), (N - 1, N), (N, N - 1),
             (255, 256), (256, 255), (256, 256), (399, 3)]
    picks += [tuple(int(v) for v in rng.integers(0, N + 1, 2)) for _ in range(9)]
    for i, j in picks:
        ref = relabel.entry(rho0, resp, i, j)
        assert abs(got[i, j] - ref) <= 1e-12 * N, (i, j, got[i, j], ref)


@pytest.mark.gpu
@pytest.mark.parametrize("N,m,L,complex_check,hermitian", [
    (3, 1, 3, False, True),
    (3, 1, 3, True, False),
    (2, 1, 4, False, False),
])
def test_reconstruct_oracle_trajectories_on_gpu(N, m, L, complex_check, hermitian):
    """The product's reconstruction from the oracle's representative
    propagations (the dense output formed by heom_reconstruct_dense) against
    the conventional oracle; four propagations when the adjoint relation
    holds, five otherwise."""
    from tests.gpu_util import torch_cuda
    torch_cuda()
    p = W.random_problem(N, m, L, 0, seed=7 + N + m, complex_check=complex_check, loss=True)
    rho0 = random_rho(N, seed=N * 10 + L, hermitian=hermitian)
    dt, nsteps, every = 0.05, 40, 10
    ref = conventional_rho(p, rho0, dt, nsteps, every)
    got = RC.reconstruct(p, rho0, dt, nsteps, every, tier0_trajectory=oracle_tier0_trajectory)
    assert np.abs(got["rho"] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert len(got["propagations"]) == (5 if complex_check else 4)
    assert got["adjoint_reduction"] == (not complex_check)
    loc = np.zeros((N + 1, N + 1), dtype=complex)
    loc[2, 2] = 1.0
    got = RC.reconstruct(p, loc, dt, 10, 5, tier0_trajectory=oracle_tier0_trajectory)
    assert got["propagations"] == ["ee"]
    assert np.abs(got["rho"] - conventional_rho(p, loc, dt, 10, 5)).max() <= 1e-12


@pytest.mark.gpu
@pytest.mark.parametrize("complex_check", [False, True])
def test_reconstruction_on_gpu(complex_check):
    from tests.gpu_util import torch_cuda
    torch_cuda()
    p = W.random_problem(4, 2, 3, 0, seed=21, complex_check=complex_check, loss=True)
    rho0 = random_rho(4, seed=5, hermitian=not complex_check)
    dt, nsteps, every = 0.05, 60, 20
    ref = conventional_rho(p, rho0, dt, nsteps, every)
    got = RC.reconstruct(p, rho0, dt, nsteps, every)
    assert np.abs(got["rho"] - ref).max() <= 1e-10 * np.abs(ref).max()
    assert len(got["propagations"]) == (5 if complex_check else 4)


@pytest.mark.parametrize("N,d", [(5, 0), (5, 1), (6, 2), (3, 2), (1, 1), (2, 2)])
def test_tier0_operator_and_expand_vs_oracle(N, d):
    """heom_tier0_operator writes the oracle's tier-0 block of the same
    operator (exact copies of the entries) and heom_tier0_expand inverts it."""
    from paper_2608_20657_amd import heom
    p = W.random_problem(N, 2, 3, d, seed=N + d)
    T = heom.Tables(p)
    rng = np.random.default_rng(N * 3 + d)
    ns = d + 3
    R = rng.normal(size=(ns, ns)) + 1j * rng.normal(size=(ns, ns))
    pa, pb = d + 1, d + 2
    for x in range(ns):                 # make R pool-invariant, as the operator is
        if x not in (pa, pb):
            R[pb, x], R[x, pb] = R[pa, x], R[x, pa]
    R[pb, pb], R[pb, pa] = R[pa, pa], R[pa, pb]
    npool = N - d
    if npool < 2:                       # no pair of pool molecules
        R[pa, pb] = R[pb, pa] = 0
    if npool < 1:
        R[pa, :] = R[:, pa] = R[pb, :] = R[:, pb] = 0
    t0 = T.tier0_operator(R)
    S = uvar.UVarSystem(p)
    ref = S.initial_state(rho=lambda i, j: R[i, j])[:t0.size]
    assert np.array_equal(t0, ref)
    assert np.array_equal(T.tier0_expand(t0), R)
