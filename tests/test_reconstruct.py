"""Linear reconstruction of general initial operators (Sec. VI.C, Table II).

The relabeling algebra of paper_2608_20657_amd.reconstruct is checked on the
CPU with representative propagations run by the symmetry-adapted oracle,
against the conventional dense HEOM oracle started from the same arbitrary
rho_S(0) (no symmetry used at all). The GPU test runs the representatives
through the C ABI.
"""
import numpy as np
import pytest

from oracle import conventional as C, integrate, uvar
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


@pytest.mark.parametrize("N,m,L,complex_check,hermitian", [
    (3, 1, 3, False, True),
    (4, 2, 2, False, True),
    (3, 1, 3, True, False),
    (2, 1, 4, False, False),
])
def test_reconstruction_matches_conventional(N, m, L, complex_check, hermitian):
    p = W.random_problem(N, m, L, 0, seed=7 + N + m, complex_check=complex_check, loss=True)
    rho0 = random_rho(N, seed=N * 10 + L, hermitian=hermitian)
    dt, nsteps, every = 0.05, 40, 10
    ref = conventional_rho(p, rho0, dt, nsteps, every)
    got = RC.reconstruct(p, rho0, dt, nsteps, every, tier0_trajectory=oracle_tier0_trajectory)
    scale = np.abs(ref).max()
    assert np.abs(got["rho"] - ref).max() <= 1e-12 * scale
    # four propagations when the adjoint relation holds (Eq. adjoint-preservation), five otherwise
    assert len(got["propagations"]) == (5 if complex_check else 4)
    assert got["adjoint_reduction"] == (not complex_check)


def test_plan_skips_absent_operator_types():
    p = W.random_problem(3, 1, 2, 0, seed=1)
    rho0 = np.zeros((4, 4), dtype=complex)
    rho0[2, 2] = 1.0                       # a localized excitation only
    got = RC.reconstruct(p, rho0, 0.05, 10, 5, tier0_trajectory=oracle_tier0_trajectory)
    assert got["propagations"] == ["ee"]
    ref = conventional_rho(p, rho0, 0.05, 10, 5)
    assert np.abs(got["rho"] - ref).max() <= 1e-12


def test_dense_relabel_sums_by_brute_force():
    """The closed-form weighted sums equal explicit relabelings of a random
    slot matrix (each relabeled operator written out entry by entry)."""
    rng = np.random.default_rng(3)
    N = 5
    R1 = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    R2 = rng.normal(size=(5, 5)) + 1j * rng.normal(size=(5, 5))
    w = rng.normal(size=N) + 1j * rng.normal(size=N)
    Wm = rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))
    np.fill_diagonal(Wm, 0)

    def relabeled(R, dist):
        """Dense operator with slot matrix R where slot 1+a is molecule dist[a]."""
        d = len(dist)
        D = np.zeros((N + 1, N + 1), dtype=complex)
        def slot(i):
            return 0 if i == 0 else (1 + dist.index(i) if i in dist else d + 1)
        for i in range(N + 1):
            for j in range(N + 1):
                si, sj = slot(i), slot(j)
                if si == d + 1 and sj == d + 1 and i != j:
                    sj = d + 2
                D[i, j] = R[si, sj]
        return D

    ref1 = sum(w[i - 1] * relabeled(R1, [i]) for i in range(1, N + 1))
    assert np.allclose(RC._dense_d1(R1, w), ref1, rtol=0, atol=1e-12)
    ref2 = sum(Wm[i - 1, j - 1] * relabeled(R2, [i, j]) for i in range(1, N + 1) for j in range(1, N + 1) if i != j)
    assert np.allclose(RC._dense_d2(R2, Wm), ref2, rtol=0, atol=1e-12)


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
