"""Seeded synthetic inputs for the symmetry-adapted HEOM hot path.

This module is the only code shared by the GPU path and the CPU oracle. It
holds problem parameters and random draws, and none of the method's
arithmetic: no hierarchy, no pattern, no right-hand side.

Problem statement (paper Sec. II, Eqs. HS, BCF-exp, scaled-HEOM): N identical
two-level molecules in one cavity mode, single-excitation basis
{|c>, |e_1>..|e_N>}, m exponentials per local bath (c_k, c_check_k, nu_k),
hierarchy depth L, d distinguished molecules (Sec. V.B), energies eps and
omega_c, single-molecule coupling g, cavity loss rate kappa.

Bath coefficients come from the Drude-Lorentz spectral density of the
paper's Eq. Drude_Lorentz, decomposed into the exact Debye term plus
Matsubara terms (the paper allows any such decomposition, Sec. II.B).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Problem:
    """One HTC-HEOM problem. Units: hbar = 1, dimensionless energies."""
    N: int
    m: int
    L: int
    d: int
    c: List[complex]                 # c_k, k = 0..m-1 (Eq. BCF-exp)
    c_check: List[complex]           # c_check_k (Eq. BCF-exp)
    nu: List[float]                  # real decay rates nu_k >= 0
    eps: float = 0.0                 # molecular transition energy (Eq. HS)
    omega_c: float = 0.0             # cavity frequency (Eq. HS)
    g: float = 0.0                   # single-molecule coupling (Eq. HS)
    kappa: float = 0.0               # cavity loss rate
    terminator: float = 0.0          # Ishizaki-Tanimura Delta (0 = off)

    def structure_key(self):
        """Tables depend on N only below the saturation point N = L + d + 2."""
        return (min(self.N, self.L + self.d + 2), self.m, self.L, self.d)


def debye_high_temperature(lam: float, gam: float, kT: float):
    """Single Debye exponential in the high-temperature form
    c = lam*gam*(2kT/gam - i), nu = gam."""
    c = complex(lam * gam * (2.0 * kT / gam), -lam * gam)
    return [c], [c.conjugate()], [gam]


def debye_matsubara(lam: float, gam: float, kT: float, m: int):
    """Drude-Lorentz BCF as the exact Debye term plus m-1 Matsubara terms.

    k = 0: c_0 = lam*gam*(cot(gam/(2kT)) - i), nu_0 = gam.
    k >= 1: nu_k = 2*pi*k*kT, c_k = 4*lam*gam*kT*nu_k/(nu_k^2 - gam^2) (real).
    All rates are real, so c_check_k = conj(c_k) (Sec. II.B).
    """
    beta = 1.0 / kT
    c = [complex(lam * gam / math.tan(beta * gam / 2.0), -lam * gam)]
    nu = [gam]
    for k in range(1, m):
        vk = 2.0 * math.pi * k * kT
        c.append(complex(4.0 * lam * gam * kT * vk / (vk * vk - gam * gam), 0.0))
        nu.append(vk)
    return c, [z.conjugate() for z in c], nu


# ---------------------------------------------------------------- workloads
KT = 0.025


def config_small() -> Problem:
    """N=2, m=1, L=3, resonant, g=0.02, kappa=0; high-temperature Debye bath
    with lam=0.02, gam=0.1, kT=0.025. rho(0)=|c><c|, dt=0.05, 2000 steps."""
    c, cc, nu = debye_high_temperature(0.02, 0.1, KT)
    return Problem(N=2, m=1, L=3, d=0, c=c, c_check=cc, nu=nu,
                   eps=0.0, omega_c=0.0, g=0.02, kappa=0.0)


def config_localized() -> Problem:
    """N=64, m=2 (Debye + one Matsubara), L=6, d=1 (molecule 1 distinguished),
    lam=0.02, gam=0.1, kT=0.025, g=0.01, eps-omega_c=0.01, kappa=0.005.
    rho(0)=|e_1><e_1|, dt=0.02, 10000 steps."""
    c, cc, nu = debye_matsubara(0.02, 0.1, KT, 2)
    return Problem(N=64, m=2, L=6, d=1, c=c, c_check=cc, nu=nu,
                   eps=0.01, omega_c=0.0, g=0.01, kappa=0.005)


def config_saturated() -> Problem:
    """N=10^4, m=3, L=8, lam=0.03, gam=0.05, kT=0.025, g=0.005, kappa=0.01,
    resonant, rho(0)=|+><+|, dt=0.02, 10000 steps."""
    c, cc, nu = debye_matsubara(0.03, 0.05, KT, 3)
    return Problem(N=10000, m=3, L=8, d=0, c=c, c_check=cc, nu=nu,
                   eps=0.0, omega_c=0.0, g=0.005, kappa=0.01)


def config_roofline_probe() -> Problem:
    """Largest structure of the batched draw: N=10^4, m=4, L=10, d=0, the
    saturated workload's bath family with three Matsubara terms, resonant,
    rho(0)=|c><c|. 17.3 M unique variables: one FP64 vector exceeds the
    256 MB last-level cache, so its streaming rate is set by HBM."""
    c, cc, nu = debye_matsubara(0.03, 0.05, KT, 4)
    return Problem(N=10000, m=4, L=10, d=0, c=c, c_check=cc, nu=nu,
                   eps=0.0, omega_c=0.0, g=0.005, kappa=0.01)


CM_TO_RAD_PER_FS = 2.0 * math.pi * 2.99792458e-5   # E[cm^-1] -> omega[rad/fs]


def config_paper_shape(N: int, d: int = 0) -> Problem:
    """The paper's single-exponential runs (Sec. VII.A), in rad/fs and fs:
    omega_cav = eps = 10000 cm^-1, collective Rabi splitting 500 cm^-1 held
    fixed with g = Omega_R / (2 sqrt N) (Eq. g-fixed-Rabi), Drude-Lorentz
    bath lam = 50 cm^-1, gam = 18 cm^-1, kT = 208 cm^-1 (300 K), one
    exponential (the exact Debye term c = lam gam (cot(gam/2kT) - i),
    nu = gam) and the Ishizaki-Tanimura terminator for the omitted
    Matsubara terms, Delta = sum_k c_k/nu_k = 2 lam kT/gam - lam cot(gam/2kT);
    L = 25, no loss. The time step is 0.5 fs (PAPER_SHAPE_DT). d = 0 for
    symmetric starts (upper polariton), d = 1 for the localized and
    cavity-site superposition starts."""
    f = CM_TO_RAD_PER_FS
    lam, gam, kT = 50.0 * f, 18.0 * f, 208.0 * f
    c = complex(lam * gam / math.tan(gam / (2.0 * kT)), -lam * gam)
    delta = 2.0 * lam * kT / gam - lam / math.tan(gam / (2.0 * kT))
    omega_r = 500.0 * f
    return Problem(N=N, m=1, L=25, d=d, c=[c], c_check=[c.conjugate()], nu=[gam],
                   eps=10000.0 * f, omega_c=10000.0 * f, g=omega_r / (2.0 * math.sqrt(N)),
                   kappa=0.0, terminator=delta)


PAPER_SHAPE_DT = 0.5


def config_paper_static(N: int, d: int = 0) -> Problem:
    """The paper's static-disorder runs (Sec. VII.D, static energetic
    disorder), in rad/fs: Gaussian site disorder sigma = 25 cm^-1 as a
    non-decaying channel (c = sigma^2, nu = 0) beside the Drude-Lorentz
    channel of config_paper_shape (with its terminator), m = 2, L = 14,
    Omega_R = 100 cm^-1 with g = Omega_R / (2 sqrt N), resonant at
    10000 cm^-1, dt = 0.5 fs."""
    f = CM_TO_RAD_PER_FS
    base = config_paper_shape(N, d)
    s2 = complex((25.0 * f) ** 2, 0.0)
    return Problem(N=N, m=2, L=14, d=d, c=[base.c[0], s2], c_check=[base.c_check[0], s2],
                   nu=[base.nu[0], 0.0], eps=base.eps, omega_c=base.omega_c,
                   g=100.0 * f / (2.0 * math.sqrt(N)), kappa=0.0, terminator=base.terminator)


def _matsubara_pole_too_close(gam: float, m: int, kT: float) -> bool:
    """gamma within 5% of a Matsubara rate nu_k = 2 pi k kT (k >= 1): there
    cot(gamma / 2kT) in the Debye coefficient diverges, whatever m, and so
    does the Matsubara coefficient c_k if the bath keeps that term."""
    k = 1
    while 2.0 * math.pi * k * kT <= gam / 0.95:
        vk = 2.0 * math.pi * k * kT
        if abs(gam / vk - 1.0) < 0.05:
            return True
        k += 1
    return False


def draw_batch(n: int = 512, seed: int = 0,
               with_horizon: bool = False) -> List[Problem]:
    """Seeded ragged batch: N~U{4..5000}, m~U{1..4}, L~U{3..10},
    g~U[0.002,0.03], lam~U[0.005,0.05], gam~U[0.02,0.2], kappa~U[0,0.02],
    kT=0.025, resonant, d=0. A gamma within 5% of a Matsubara rate 2 pi k kT
    (k >= 1; there the Debye coefficient's cot and the k-th Matsubara
    coefficient diverge) is redrawn, whatever m. With with_horizon, each
    problem carries a step count U{1000..20000} as attribute `horizon`."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        N = int(rng.integers(4, 5001))
        m = int(rng.integers(1, 5))
        L = int(rng.integers(3, 11))
        g = float(rng.uniform(0.002, 0.03))
        lam = float(rng.uniform(0.005, 0.05))
        gam = float(rng.uniform(0.02, 0.2))
        while _matsubara_pole_too_close(gam, m, KT):
            gam = float(rng.uniform(0.02, 0.2))
        kappa = float(rng.uniform(0.0, 0.02))
        c, cc, nu = debye_matsubara(lam, gam, KT, m)
        p = Problem(N=N, m=m, L=L, d=0, c=c, c_check=cc, nu=nu,
                    eps=0.0, omega_c=0.0, g=g, kappa=kappa)
        if with_horizon:
            p.horizon = int(rng.integers(1000, 20001))
        out.append(p)
    return out


def arrival_times(rate: float, window_s: float, seed: int = 0) -> np.ndarray:
    """Poisson arrival times (seconds) in [0, window_s)."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= window_s:
            return np.asarray(out)
        out.append(t)


def random_problem(N: int, m: int, L: int, d: int, seed: int,
                   complex_check: bool = False, loss: bool = True,
                   detuning: bool = True, terminator: bool = False) -> Problem:
    """Random parameters of unit-ish size for structural parity tests.

    With complex_check, c_check is drawn independently of conj(c) (the
    equations then have no Hermiticity symmetry, which exposes sign and
    conjugation mistakes)."""
    rng = np.random.default_rng(seed)
    c = [complex(rng.uniform(-1, 1), rng.uniform(-1, 1)) * 0.3 for _ in range(m)]
    if complex_check:
        cc = [complex(rng.uniform(-1, 1), rng.uniform(-1, 1)) * 0.3 for _ in range(m)]
    else:
        cc = [z.conjugate() for z in c]
    nu = [float(rng.uniform(0.05, 1.0)) for _ in range(m)]
    return Problem(N=N, m=m, L=L, d=d, c=c, c_check=cc, nu=nu,
                   eps=float(rng.uniform(-0.5, 0.5)) if detuning else 0.0,
                   omega_c=float(rng.uniform(-0.5, 0.5)) if detuning else 0.0,
                   g=float(rng.uniform(0.05, 0.5)),
                   kappa=float(rng.uniform(0.0, 0.3)) if loss else 0.0,
                   terminator=float(rng.uniform(0.0, 0.2)) if terminator else 0.0)


def random_vector(n: int, seed: int) -> np.ndarray:
    """Complex128 vector with entries uniform in the unit square."""
    rng = np.random.default_rng(seed)
    return (rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)).astype(np.complex128)


WORKLOADS = {
    "small": config_small,
    "localized": config_localized,
    "saturated": config_saturated,
    "roofline_probe": config_roofline_probe,
}
