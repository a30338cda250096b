"""Conventional scaled HEOM with dense ADOs (oracle; test infrastructure only).

Follows the paper's Eq. scaled-HEOM term by term, on the single-excitation
basis of Eq. basis and the Hamiltonian of Eq. HS:

    d rho_n/dt = -i[H_S, rho_n] - Gamma_n rho_n
                 - i sum_{i,k} sqrt((n_ik+1)|c_k|) [Q_i, rho_{n+e_ik}]        (|n| < L)
                 - i sum_{i,k} sqrt(n_ik/|c_k|) (c_k Q_i rho_{n-e_ik}
                                                 - cc_k rho_{n-e_ik} Q_i)    (n_ik > 0)

with Gamma_n = sum n_ik nu_k (Eq. tier-damping), Q_i = |e_i><e_i| and the hard
cutoff |n| <= L (Sec. II.C). Two additions act on every ADO:

* cavity loss, Lindblad form kappa(a rho a^+ - {a^+ a, rho}/2) with
  a = |G><c|; the jump term leaves the single-excitation block, so the block
  equation gains -(kappa/2){|c><c|, rho_n};
* the optional Ishizaki-Tanimura terminator, -Delta sum_i [Q_i,[Q_i, rho_n]].

A channel with |c_k| = 0 is switched off (both coefficients zero).

Vector layout: ADO-major in label order, each ADO row-major over the basis
{c, e_1..e_N} (index 0 = cavity). Super-operators act on row-major vec(rho):
A rho -> (A kron I) vec, rho B -> (I kron B^T) vec.

Parity: pinned by tests/test_oracle_conventional.py (bath-off Rabi
oscillation, pure-dephasing closed form, trace and Hermiticity, ADO count).
"""
from __future__ import annotations

import itertools
import math
from typing import Dict, List, Tuple

import numpy as np
import scipy.sparse as sp


def labels(N: int, m: int, L: int) -> List[Tuple[int, ...]]:
    """Every label n (flattened molecule-major, n[i*m+k]) with |n| <= L,
    in order of increasing tier, then lexicographic."""
    out = []
    for tier in range(L + 1):
        for combo in itertools.combinations_with_replacement(range(N * m), tier):
            n = [0] * (N * m)
            for j in combo:
                n[j] += 1
            out.append(tuple(n))
    # each multiset of (i,k) directions is produced exactly once; sort within
    # a tier for a deterministic order (label 0 is the zero label)
    out.sort(key=lambda n: (sum(n), tuple(-x for x in n)))
    return out


def hamiltonian(N: int, eps: float, omega_c: float, g: float) -> np.ndarray:
    D = N + 1
    H = np.zeros((D, D), dtype=np.complex128)
    H[0, 0] = omega_c
    for i in range(1, D):
        H[i, i] = eps
        H[0, i] = g
        H[i, 0] = g
    return H


def _proj(D: int, i: int) -> sp.csr_matrix:
    return sp.csr_matrix(([1.0 + 0j], ([i], [i])), shape=(D, D))


def generator(p) -> Tuple[sp.csr_matrix, List[Tuple[int, ...]]]:
    """Sparse generator of the conventional scaled HEOM for problem p."""
    N, m, L = p.N, p.m, p.L
    D = N + 1
    D2 = D * D
    I = sp.identity(D, dtype=np.complex128, format="csr")
    H = sp.csr_matrix(hamiltonian(N, p.eps, p.omega_c, p.g))
    comm_H = (sp.kron(H, I) - sp.kron(I, H.T)).tocsr()
    Pc = _proj(D, 0)
    loss = (sp.kron(Pc, I) + sp.kron(I, Pc.T)).tocsr() * (0.5 * p.kappa)
    Q = [_proj(D, i + 1) for i in range(N)]
    QL = [sp.kron(q, I).tocsr() for q in Q]          # Q_i rho
    QR = [sp.kron(I, q.T).tocsr() for q in Q]        # rho Q_i
    term = sp.csr_matrix((D2, D2), dtype=np.complex128)
    if p.terminator != 0.0:
        for i in range(N):
            QQ = (QL[i] @ QL[i] - 2.0 * (QL[i] @ QR[i]) + QR[i] @ QR[i])
            term = term + QQ
        term = term * p.terminator
    a = [abs(complex(ck)) for ck in p.c]

    labs = labels(N, m, L)
    index: Dict[Tuple[int, ...], int] = {n: j for j, n in enumerate(labs)}
    rows, cols, vals = [], [], []

    def put(bi: int, bj: int, M: sp.spmatrix):
        M = M.tocoo()
        rows.append(M.row + bi * D2)
        cols.append(M.col + bj * D2)
        vals.append(M.data)

    base = (-1j) * comm_H - loss - term
    for j, n in enumerate(labs):
        gam = sum(n[i * m + k] * p.nu[k] for i in range(N) for k in range(m))
        put(j, j, base - gam * sp.identity(D2, dtype=np.complex128, format="csr"))
        tier = sum(n)
        for i in range(N):
            for k in range(m):
                nik = n[i * m + k]
                if a[k] == 0.0:
                    continue
                if tier < L:
                    up = list(n)
                    up[i * m + k] += 1
                    coef = -1j * math.sqrt((nik + 1) * a[k])
                    put(j, index[tuple(up)], (QL[i] - QR[i]) * coef)
                if nik > 0:
                    dn = list(n)
                    dn[i * m + k] -= 1
                    w = math.sqrt(nik / a[k])
                    M = (QL[i] * complex(p.c[k]) - QR[i] * complex(p.c_check[k])) * (-1j * w)
                    put(j, index[tuple(dn)], M)
    dim = len(labs) * D2
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(dim, dim))
    A.sum_duplicates()
    return A, labs


def ado_count(N: int, m: int, L: int) -> int:
    """Closed form C(Nm+L, L) (Eq. direct-ado-count)."""
    return math.comb(N * m + L, L)


def initial_vector(rho0: np.ndarray, n_ado: int) -> np.ndarray:
    """Factorized initial condition (Eq. factorized-initial-*): tier 0 holds
    rho_S(0), every other ADO is zero."""
    D2 = rho0.size
    y = np.zeros(n_ado * D2, dtype=np.complex128)
    y[:D2] = rho0.reshape(-1)
    return y
