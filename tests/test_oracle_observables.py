"""Pins of the oracle's observables and initial states.

Against: the definitions evaluated on dense matrices (Eqs. Pcav-uvar ...
Pminus-uvar as matrix elements), and the paper's printed initial values
(Eqs. cavity-initial-uvar, bright-initial-uvar, upper-polariton-initial,
lower-polariton-initial, localized-initial-TC-populations,
superposition-initial-TC-populations, site1-cavity-initial-elements).
"""
import math

import numpy as np
import pytest

from oracle import conventional, observables as O, uvar
from paper_2608_20657_amd.workloads import Problem


def prob(N, d, eps=0.0, wc=0.0, g=0.1):
    return Problem(N=N, m=1, L=2, d=d, c=[0.01 - 0.02j], c_check=[0.01 + 0.02j], nu=[0.1],
                   eps=eps, omega_c=wc, g=g)


@pytest.mark.parametrize("N,d,eps,wc", [(3, 0, 0, 0), (5, 1, 0.2, -0.1), (4, 2, -0.3, 0.1), (6, 1, 0, 0)])
def test_from_tier0_matches_dense(N, d, eps, wc):
    p = prob(N, d, eps, wc)
    S = uvar.UVarSystem(p)
    labs = conventional.labels(N, 1, 2)
    rng = np.random.default_rng(N + d)
    u = rng.standard_normal(S.n_var) + 1j * rng.standard_normal(S.n_var)
    rho = S.expand(u, labs)[:(N + 1) ** 2].reshape(N + 1, N + 1)
    rho = 0.5 * (rho + rho.conj().T)              # Hermitian part
    u0 = S.compress(np.r_[rho.reshape(-1), np.zeros(len(labs[1:]) * (N + 1) ** 2)], labs)
    assert np.abs(O.from_tier0(S, u0) - O.dense(rho, N, eps, wc, p.g)).max() < 1e-13


def tier0(S):
    b = S.blocks[0]
    return b


@pytest.mark.parametrize("N", [2, 5, 10, 10 ** 4])
def test_symmetric_initial_states(N):
    p = prob(N, 0, eps=0.05, wc=-0.02, g=0.03)
    S = uvar.UVarSystem(p)
    b = tier0(S)
    th = O.theta(N, p.eps, p.omega_c, p.g)
    s, c = math.sin(th), math.cos(th)
    Z, Y0, X0, P0, T0 = b.mat(0, 0), b.mat(0, 1), b.mat(1, 0), b.mat(1, 1), b.T(0)
    states = {
        "photon": (lambda i: 1.0 if i == 0 else 0.0, dict(Z=1, X=0, Y=0, P=0, T=0)),
        "bright": (lambda i: 0.0 if i == 0 else 1 / math.sqrt(N), dict(Z=0, X=0, Y=0, P=1 / N, T=1 / N)),
        "UP": (lambda i: c if i == 0 else s / math.sqrt(N),
               dict(Z=c * c, X=s * c / math.sqrt(N), Y=s * c / math.sqrt(N), P=s * s / N, T=s * s / N)),
        "LP": (lambda i: -s if i == 0 else c / math.sqrt(N),
               dict(Z=s * s, X=-s * c / math.sqrt(N), Y=-s * c / math.sqrt(N), P=c * c / N, T=c * c / N)),
    }
    for name, (amp, want) in states.items():
        y = S.initial_state(amp=amp)
        for key, idx in dict(Z=Z, X=X0, Y=Y0, P=P0, T=T0).items():
            assert abs(y[idx] - want[key]) < 1e-15, (name, key)
        assert np.count_nonzero(y[b.size:]) == 0
        o = O.from_tier0(S, y)
        assert abs(o[0] - 1) < 1e-12
    up = O.from_tier0(S, S.initial_state(amp=states["UP"][0]))
    assert abs(up[5] - 1) < 1e-12 and abs(up[6]) < 1e-12
    lp = O.from_tier0(S, S.initial_state(amp=states["LP"][0]))
    assert abs(lp[6] - 1) < 1e-12 and abs(lp[5]) < 1e-12


@pytest.mark.parametrize("N", [5, 10, 25, 100, 10 ** 3, 10 ** 6])
def test_localized_initial_populations(N):
    p = prob(N, 1, g=0.01)
    S = uvar.UVarSystem(p)
    o = O.from_tier0(S, S.initial_state(amp=lambda i: 1.0 if i == 1 else 0.0))
    assert abs(o[5] - 1 / (2 * N)) < 1e-13 and abs(o[6] - 1 / (2 * N)) < 1e-13
    assert abs(o[4] - (1 - 1 / N)) < 1e-13
    assert o[7] == 1.0 and o[8] == 0.0


@pytest.mark.parametrize("N", [5, 10, 25, 100, 10 ** 3])
def test_superposition_initial_populations(N):
    p = prob(N, 1, g=0.01)
    S = uvar.UVarSystem(p)
    amp = lambda i: math.sqrt(0.7) if i == 0 else (math.sqrt(0.3) if i == 1 else 0.0)
    y = S.initial_state(amp=amp)
    b = S.blocks[0]
    assert abs(y[b.mat(1, 1)] - 0.3) < 1e-15 and abs(y[b.mat(0, 0)] - 0.7) < 1e-15
    assert abs(y[b.mat(1, 0)] - math.sqrt(0.21)) < 1e-15 and abs(y[b.mat(0, 1)] - math.sqrt(0.21)) < 1e-15
    o = O.from_tier0(S, y)
    assert abs(o[4] - 0.3 * (1 - 1 / N)) < 1e-13
    assert abs(o[5] - 0.5 * (math.sqrt(0.7) + math.sqrt(0.3 / N)) ** 2) < 1e-13
    assert abs(o[6] - 0.5 * (math.sqrt(0.7) - math.sqrt(0.3 / N)) ** 2) < 1e-13


def bath_free_hamiltonian(N, eps, wc, g):
    """H_S of Eq. HS on {|c>, |e_1>..|e_N>}, written out here (independent
    of the oracle's own builder)."""
    H = np.diag([wc] + [eps] * N).astype(np.complex128)
    H[0, 1:] = g
    H[1:, 0] = g
    return H


@pytest.mark.parametrize("N,eps,wc,g", [(3, 0.05, -0.02, 0.03), (3, -0.05, 0.02, 0.03),
                                        (5, 0.3, 0.0, 0.01), (5, 0.0, 0.3, 0.01),
                                        (4, 0.2, -0.1, 0.2), (6, 0.0, 0.0, 0.05)])
def test_polaritons_are_the_bright_eigenvectors(N, eps, wc, g):
    """Eqs. Rabi-splitting and polariton-states under detuning of either
    sign: the two eigenvectors of H_S with a cavity component are the
    polaritons, the higher one |+>. A state prepared in the upper eigenvector
    has P_+ = 1, P_- = 0, and in the lower one P_- = 1, P_+ = 0; the
    compressed tier-0 form gives the same numbers. The eigenvectors come from
    numpy's eigh, not from the oracle's angle."""
    H = bath_free_hamiltonian(N, eps, wc, g)
    w, V = np.linalg.eigh(H)
    bright = [j for j in range(N + 1) if abs(V[0, j]) > 1e-8]
    assert len(bright) == 2                       # the N-1 dark states have no cavity part
    lo, hi = sorted(bright, key=lambda j: w[j])
    # the splitting of the two is sqrt(Omega_R^2 + Delta^2), Omega_R = 2 g sqrt(N)
    assert abs((w[hi] - w[lo]) - math.sqrt(4 * g * g * N + (wc - eps) ** 2)) < 1e-12
    p = prob(N, 0, eps, wc, g)
    S = uvar.UVarSystem(p)
    labs = conventional.labels(N, 1, 2)
    for j, plus in ((hi, 1.0), (lo, 0.0)):
        v = V[:, j]
        rho = np.outer(v, v.conj())
        o = O.dense(rho, N, eps, wc, g)
        assert abs(o[5] - plus) < 1e-12 and abs(o[6] - (1.0 - plus)) < 1e-12
        assert abs(o[0] - 1.0) < 1e-12 and abs(o[3] + o[1] - 1.0) < 1e-12   # all weight in {c, B}
        u0 = S.compress(np.r_[rho.reshape(-1), np.zeros(len(labs[1:]) * (N + 1) ** 2)], labs)
        assert np.abs(O.from_tier0(S, u0) - o).max() < 1e-13
