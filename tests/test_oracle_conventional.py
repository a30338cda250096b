"""Pins of the conventional dense HEOM oracle and of the RK4 integrator.

Against: closed-form dynamics of special cases (bath switched off:
collective Rabi oscillation at sqrt(N) g, Eq. Rabi-splitting; with cavity
loss: the exact non-Hermitian two-level evolution; pure dephasing with g = 0:
the second-cumulant result exp(-int int C), which the hierarchy reaches as L
grows), invariants (trace and Hermiticity of rho_S without loss, dTr/dt =
-kappa Z with loss), and the definition of RK4 for a linear system (one
step equals the degree-4 Taylor polynomial of exp(hA)).
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import conventional, integrate
from paper_2608_20657_amd.workloads import Problem, random_problem


def run(p, rho0, h, steps, every=1):
    A, labs = conventional.generator(p)
    y0 = conventional.initial_vector(rho0, len(labs))
    D = p.N + 1
    _, obs = integrate.propagate(A, y0, h, steps, every,
                                 observe=lambda y: y[:D * D].reshape(D, D).copy())
    return obs


def bath_off(N, m=1, **kw):
    return Problem(N=N, m=m, L=2, d=0, c=[0j] * m, c_check=[0j] * m, nu=[0.1] * m, **kw)


@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_rabi_resonant(N):
    g, h = 0.05, 0.05
    p = bath_off(N, g=g)
    rho0 = np.zeros((N + 1, N + 1), complex)
    rho0[0, 0] = 1
    obs = run(p, rho0, h, 400, 10)
    for s, rho in enumerate(obs):
        t = s * 10 * h
        assert abs(rho[0, 0].real - math.cos(math.sqrt(N) * g * t) ** 2) < 1e-9


def test_rabi_detuned_with_loss():
    N, g, eps, wc, kappa, h = 3, 0.04, 0.03, -0.02, 0.01, 0.02
    p = bath_off(N, g=g, eps=eps, omega_c=wc, kappa=kappa)
    rho0 = np.zeros((N + 1, N + 1), complex)
    rho0[0, 0] = 1
    obs = run(p, rho0, h, 1000, 50)
    Om = g * math.sqrt(N)
    Heff = np.array([[wc - 0.5j * kappa, Om], [Om, eps]])
    for s, rho in enumerate(obs):
        t = s * 50 * h
        psi = sla.expm(-1j * Heff * t) @ np.array([1, 0], complex)
        assert abs(rho[0, 0].real - abs(psi[0]) ** 2) < 1e-9
        # <B|rho|B>
        B = np.r_[0, np.ones(N) / math.sqrt(N)]
        assert abs((B @ rho @ B).real - abs(psi[1]) ** 2) < 1e-9


def pure_dephasing_x(c, nu, delta, t):
    gt = sum(ck / nk ** 2 * (math.exp(-nk * t) + nk * t - 1.0) for ck, nk in zip(c, nu))
    return 0.5 * np.exp(-1j * delta * t - gt)


@pytest.mark.parametrize("m", [1, 2])
def test_pure_dephasing_converges_with_depth(m):
    from paper_2608_20657_amd.workloads import debye_matsubara, debye_high_temperature
    if m == 1:
        c, cc, nu = debye_high_temperature(0.02, 0.1, 0.025)
    else:
        c, cc, nu = debye_matsubara(0.02, 0.1, 0.025, 2)
    eps, wc, h, steps = 0.01, 0.0, 0.05, 600
    errs = []
    for L in (1, 3, 6):
        p = Problem(N=1, m=m, L=L, d=0, c=c, c_check=cc, nu=nu, eps=eps, omega_c=wc, g=0.0)
        rho0 = 0.5 * np.ones((2, 2), complex)
        obs = run(p, rho0, h, steps, steps)
        t = steps * h
        errs.append(abs(obs[-1][1, 0] - pure_dephasing_x(c, nu, eps - wc, t)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-6
    # the molecule-cavity coherence pairs with C(t), the cavity-molecule one
    # with its conjugate
    Y = obs[-1][0, 1]
    assert abs(Y - np.conj(pure_dephasing_x(c, nu, eps - wc, t))) < 1e-6


def test_trace_and_hermiticity():
    p = random_problem(3, 2, 3, 0, seed=5, loss=False)
    rng = np.random.default_rng(0)
    psi = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    psi /= np.linalg.norm(psi)
    rho0 = np.outer(psi, psi.conj())
    for rho in run(p, rho0, 0.01, 200, 20):
        assert abs(np.trace(rho) - 1.0) < 1e-12
        assert np.abs(rho - rho.conj().T).max() < 1e-12


def test_trace_decay_with_loss():
    p = random_problem(2, 1, 3, 0, seed=7, loss=True)
    A, labs = conventional.generator(p)
    rng = np.random.default_rng(3)
    y = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    dy = A @ y
    D = p.N + 1
    rho, drho = y[:D * D].reshape(D, D), dy[:D * D].reshape(D, D)
    assert abs(np.trace(drho) - (-p.kappa * rho[0, 0])) < 1e-12


def test_rk4_is_taylor_degree4():
    rng = np.random.default_rng(11)
    A = (rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12))) * 0.3
    y = rng.standard_normal(12) + 1j * rng.standard_normal(12)
    h = 0.37
    want = y.copy()
    term = y.copy()
    for j in range(1, 5):
        term = (h * A @ term) / j
        want = want + term
    got = integrate.rk4_step(A, y, h)
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()


def test_rk4_scalar_amplification():
    lam, h = -0.8 + 0.3j, 0.25
    z = lam * h
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    got = integrate.rk4_step(np.array([[lam]]), np.array([1.0 + 0j]), h)[0]
    assert abs(got - R) < 1e-15


def test_terminator_pure_dephasing_closed_form():
    """The terminator (Sec. VII.A, Ishizaki-Tanimura form) under pure
    dephasing (g = 0): -Delta sum_i [Q_i,[Q_i, rho]] multiplies a
    molecule-cavity coherence by exp(-Delta t) and a coherence between two
    molecules by exp(-2 Delta t), and leaves populations alone. Against
    X(t) = X(0) exp(-i(eps - omega_c) t - g(t) - Delta t) at N = 1 and
    S_12(t) = S_12(0) exp(-g(t) - conj(g(t)) - 2 Delta t) at N = 2, with
    g(t) = sum_k c_k/nu_k^2 (exp(-nu_k t) + nu_k t - 1), which the hierarchy
    reaches to rounding at these depths."""
    from paper_2608_20657_amd.workloads import debye_high_temperature
    c, cc, nu = debye_high_temperature(0.02, 0.1, 0.025)
    eps, wc, h, steps, delta = 0.01, -0.004, 0.05, 600, 0.013
    t = steps * h
    gt = sum(ck / nk ** 2 * (math.exp(-nk * t) + nk * t - 1.0) for ck, nk in zip(c, nu))
    p1 = Problem(N=1, m=1, L=12, d=0, c=c, c_check=cc, nu=nu, eps=eps, omega_c=wc, g=0.0,
                 terminator=delta)
    rho1 = run(p1, 0.5 * np.ones((2, 2), complex), h, steps, steps)[-1]
    want_x = 0.5 * np.exp(-1j * (eps - wc) * t - gt - delta * t)
    assert abs(rho1[1, 0] - want_x) < 1e-9
    assert abs(rho1[0, 1] - np.conj(want_x)) < 1e-9
    assert abs(rho1[1, 1] - 0.5) < 1e-13 and abs(rho1[0, 0] - 0.5) < 1e-13
    p2 = Problem(N=2, m=1, L=8, d=0, c=c, c_check=cc, nu=nu, eps=eps, omega_c=wc, g=0.0,
                 terminator=delta)
    psi = np.array([0.0, 1.0, 1.0]) / math.sqrt(2.0)
    rho2 = run(p2, np.outer(psi, psi).astype(complex), h, steps, steps)[-1]
    want_s = 0.5 * np.exp(-gt - np.conj(gt) - 2.0 * delta * t)
    assert abs(rho2[1, 2] - want_s) < 1e-9 and abs(rho2[2, 1] - want_s) < 1e-9
    assert abs(rho2[1, 1] - 0.5) < 1e-13 and abs(rho2[2, 2] - 0.5) < 1e-13
    # the factor really is the terminator's: without it the same runs miss
    # the closed form by far more than the tolerance
    assert abs(want_x * math.exp(delta * t) - want_x) > 1e-2
