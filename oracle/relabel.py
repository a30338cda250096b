"""Linear reconstruction by explicit relabelings (oracle; test infrastructure only).

Sec. VI.C: the reduced map G_t is linear in rho_S(0) (Eq. Gt-linearity) and
commutes with relabelings U of the molecules (Eq. Gt-covariance). Writing
rho_S(0) as sum over (a, b) of rho0[a][b] |a><b| (index 0 = cavity, 1..N =
molecules), each |a><b| is the relabeling of one representative of Table II:

    (0, 0): |c><c|        d = 0, no molecule distinguished
    (k, 0): |e_1><c|      d = 1, molecule k in the place of e_1
    (0, k): |c><e_1|      d = 1
    (k, k): |e_1><e_1|    d = 1
    (k, l): |e_1><e_2|    d = 2, k in the place of e_1 and l in that of e_2

so rho_S(t) = sum over (a, b) of rho0[a][b] U_ab G_t[representative] U_ab^+.
A representative's response is given by its slot matrix R (slots: cavity,
the distinguished molecules, two pool molecules; heom_tier0_expand's form).
The relabeled response is written out entry by entry: an entry (i, j) takes
R at the slots of i and j (cavity, the distinguished slot that i or j was
relabeled into, else a pool molecule; two different pool molecules take the
two pool slots), as pool invariance requires. Every term of the double sum
over (a, b) is added on its own: no closed-form weight sums.

Parity: pinned by tests/test_reconstruct.py (the sum of relabeled oracle
responses equals the conventional dense HEOM propagated from the same
rho_S(0); the |c><e_1| response is the adjoint of the |e_1><c| one when
c_check = conj(c), Eq. adjoint-preservation).
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np


def representative(a: int, b: int) -> Tuple[str, List[int]]:
    """Name of the representative of |a><b| and the molecules relabeled into
    its distinguished slots e_1 (, e_2)."""
    if a == 0 and b == 0:
        return "cc", []
    if b == 0:
        return "ec", [a]
    if a == 0:
        return "ce", [b]
    if a == b:
        return "ee", [a]
    return "e12", [a, b]


def slots(i: int, j: int, dist: List[int]) -> Tuple[int, int]:
    """Slots of the basis states i and j in a response whose distinguished
    slots hold the molecules `dist`."""
    d = len(dist)

    def one(x):
        if x == 0:
            return 0
        if x in dist:
            return 1 + dist.index(x)
        return d + 1

    si, sj = one(i), one(j)
    if si == d + 1 and sj == d + 1 and i != j:
        sj = d + 2          # two different pool molecules
    return si, sj


def entry(rho0: np.ndarray, resp: Dict[str, np.ndarray], i: int, j: int) -> complex:
    """Entry (i, j) of sum over (a, b) of rho0[a][b] U_ab G[rep] U_ab^+."""
    D = rho0.shape[0]
    total = 0j
    for a in range(D):
        for b in range(D):
            w = rho0[a, b]
            if w == 0:
                continue
            name, dist = representative(a, b)
            si, sj = slots(i, j, dist)
            total += w * resp[name][si, sj]
    return complex(total)


def dense(rho0: np.ndarray, resp: Dict[str, np.ndarray]) -> np.ndarray:
    """The whole (N+1) x (N+1) reconstruction (small N: N^4 terms)."""
    D = rho0.shape[0]
    out = np.empty((D, D), dtype=np.complex128)
    for i in range(D):
        for j in range(D):
            out[i, j] = entry(rho0, resp, i, j)
    return out
