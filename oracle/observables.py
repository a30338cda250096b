"""Populations of the reduced density operator (oracle; test infrastructure
only).

Output order (10 real numbers), shared by convention with the library's
observable vector:
    0 Tr rho_S                     (Eq. trace-uvar)
    1 P_cav = <c|rho|c>            (Eq. Pcav-uvar)
    2 P_exc = sum_i <e_i|rho|e_i>  (Eq. Pexc-uvar)
    3 P_B = <B|rho|B>              (Eq. PB-uvar, |B> of Eq. bright)
    4 P_D = Tr(rho P_D)            (Eq. PD-uvar, P_D of Eq. dark-projector)
    5 P_+ = <+|rho|+>              (Eq. Pplus-uvar)
    6 P_- = <-|rho|->              (Eq. Pminus-uvar)
    7 <e_1|rho|e_1>                (site 1; Sec. VII.B)
    8 sum_{i>1} <e_i|rho|e_i>      (other sites; Sec. VII.B)
    9 Im Tr rho_S                  (zero for a Hermitian rho_S)

Polariton angle (Eq. polariton-states): tan(2 theta) = Omega_R / Delta with
Omega_R = 2 g sqrt(N) (Eq. Rabi-splitting), Delta = omega_c - eps and
theta in [0, pi/2]; read as theta = atan2(Omega_R, Delta) / 2.

`dense` evaluates the definitions on a full (N+1)x(N+1) matrix.
`from_tier0` evaluates them from the tier-0 unique variables by summing the
identical entries of each category with its multiplicity (any d); for d = 0
these are the paper's formulas Eqs. trace-uvar ... Pminus-uvar.

Parity: tests/test_oracle_observables.py checks from_tier0 against dense on
expanded random Hermitian states, and both against the paper's printed
initial values (Eqs. cavity-initial-uvar ... superposition-initial-TC-
populations).
"""
from __future__ import annotations

import math

import numpy as np

NOBS = 10


def theta(N: int, eps: float, omega_c: float, g: float) -> float:
    return 0.5 * math.atan2(2.0 * g * math.sqrt(N), omega_c - eps)


def dense(rho: np.ndarray, N: int, eps: float, omega_c: float, g: float) -> np.ndarray:
    D = N + 1
    assert rho.shape == (D, D)
    c = np.zeros(D, dtype=np.complex128)
    c[0] = 1.0
    B = np.zeros(D, dtype=np.complex128)
    B[1:] = 1.0 / math.sqrt(N)
    th = theta(N, eps, omega_c, g)
    up = math.sin(th) * B + math.cos(th) * c
    lp = math.cos(th) * B - math.sin(th) * c
    Pd = np.zeros((D, D), dtype=np.complex128)
    Pd[1:, 1:] = np.eye(N)
    Pd -= np.outer(B, B.conj())
    tr = np.trace(rho)
    out = np.zeros(NOBS)
    out[0] = tr.real
    out[1] = rho[0, 0].real
    out[2] = np.trace(rho[1:, 1:]).real
    out[3] = (B.conj() @ rho @ B).real
    out[4] = np.trace(rho @ Pd).real
    out[5] = (up.conj() @ rho @ up).real
    out[6] = (lp.conj() @ rho @ lp).real
    out[7] = rho[1, 1].real
    out[8] = np.trace(rho[2:, 2:]).real
    out[9] = tr.imag
    return out


def from_tier0(sys, y: np.ndarray) -> np.ndarray:
    """Observables from the tier-0 block of a unique-variable vector."""
    p = sys.p
    N = p.N
    blk = sys.blocks[0]
    cats = blk.cats
    G = blk.G
    Z = y[blk.mat(0, 0)]
    X = [y[blk.mat(q + 1, 0)] for q in range(G)]
    Y = [y[blk.mat(0, q + 1)] for q in range(G)]
    P = [y[blk.mat(q + 1, q + 1)] for q in range(G)]
    M = [float(c.mult) for c in cats]
    pexc = sum(M[q] * P[q] for q in range(G))
    tr = Z + pexc
    # sum_{ij} rho_ij over molecules, grouped by category pairs
    tot = pexc
    for q in range(G):
        if cats[q].mult >= 2:
            tot += M[q] * (M[q] - 1.0) * y[blk.T(q)]
        for r in range(G):
            if r != q:
                tot += M[q] * M[r] * y[blk.mat(q + 1, r + 1)]
    pb = tot / N
    bc = sum(M[q] * X[q] for q in range(G)) / math.sqrt(N)   # <B|rho|c>
    cb = sum(M[q] * Y[q] for q in range(G)) / math.sqrt(N)   # <c|rho|B>
    th = theta(N, p.eps, p.omega_c, p.g)
    s, c = math.sin(th), math.cos(th)
    out = np.zeros(NOBS)
    out[0] = tr.real
    out[1] = Z.real
    out[2] = pexc.real
    out[3] = pb.real
    out[4] = (pexc - pb).real
    out[5] = (Z * c * c + pb * s * s + s * c * (bc + cb)).real
    out[6] = (Z * s * s + pb * c * c - s * c * (bc + cb)).real
    site1 = None
    for q, cat in enumerate(cats):
        if cat.dist_label == 0:
            site1 = P[q]
    if site1 is None:
        # molecule 1 is a pool molecule: it lies in the zero category
        site1 = P[G - 1]
    out[7] = site1.real
    out[8] = (pexc - site1).real
    out[9] = tr.imag
    return out
