"""General initial density operators by linear reconstruction (Sec. VI.C).

The reduced map G_t is linear in rho_S(0) (Eq. Gt-linearity) and covariant
under molecular relabelings (Eq. Gt-covariance). Any single-excitation
operator splits into five ordered operator types (Eq.
arbitrary-initial-expansion), and every operator of one type is a
relabeling of one representative (Table II):

    |c><c|       d = 0        |e_1><c|   d = 1        |c><e_1|   d = 1
    |e_1><e_1|   d = 1        |e_1><e_2| d = 2

so rho_S(t) for any rho_S(0) follows from at most five propagations whose
sizes do not depend on N. The response to |c><e_1| is the adjoint of the
response to |e_1><c| when the map preserves adjoints (Eq.
adjoint-preservation); with the real decay rates of this library that holds
when c_check_k = conj(c_k) for every channel, and then four propagations
suffice. Otherwise the fifth one is run.

Each representative runs on the device through the C ABI (its own tables
with d distinguished molecules); its tier-0 block at every output time is
read back and turned into the representative's slot matrix R (cavity,
distinguished molecules, two pool molecules; heom_tier0_expand). The dense
rho_S(t) is then the weighted sum of the relabeled responses, formed in
closed form per entry: for the d=1 representatives with weights w_i,

    [c,c] = W R_cc     [c,k] = w_k R_c1 + (W - w_k) R_cp     (W = sum_i w_i)
    [k,k] = w_k R_11 + (W - w_k) R_pp
    [k,l] = w_k R_1p + w_l R_p1 + (W - w_k - w_l) R_pq          (k != l)

and similarly for the ordered pairs of the d=2 representative. The dense
output has (N+1)^2 entries per time (the quadratic cost of the requested
output, not of the propagation).
"""
from __future__ import annotations

import copy
from typing import Callable, Dict, List, Optional

import numpy as np

# representative operators: (name, d, (row slot, column slot)) with slots
# 0 = cavity, 1..d = distinguished molecules e_1..e_d
REPRESENTATIVES = [
    ("cc", 0, (0, 0)),
    ("ec", 1, (1, 0)),
    ("ce", 1, (0, 1)),
    ("ee", 1, (1, 1)),
    ("e12", 2, (1, 2)),
]

MAX_DENSE_N = 4096


def with_d(problem, d: int):
    q = copy.copy(problem)
    q.d = d
    return q


def adjoint_preserved(problem) -> bool:
    """Eq. adjoint-preservation for real decay rates: every c_check_k is the
    complex conjugate of c_k (then the equations map an ADO hierarchy onto
    its adjoint)."""
    cc = problem.c_check if problem.c_check is not None else [complex(z).conjugate() for z in problem.c]
    return all(complex(b) == complex(a).conjugate() for a, b in zip(problem.c, cc))


def slot_matrix(d: int, a: int, b: int) -> np.ndarray:
    R = np.zeros((d + 3, d + 3), dtype=np.complex128)
    R[a, b] = 1.0
    return R


def gpu_tier0_trajectory(problem, R0: np.ndarray, dt: float, nsteps: int, every: int,
                         precision: int = 0) -> List[np.ndarray]:
    """Propagate the operator with slot matrix R0 (its tables have
    problem.d distinguished molecules) on the device and return its slot
    matrix after 0, every, 2 every, ... steps."""
    import torch
    from . import heom
    T = heom.Tables(problem)
    info = T.info()
    s = torch.cuda.current_stream()
    img = torch.empty(info["table_bytes"], dtype=torch.uint8, device="cuda")
    T.upload(img, s)
    y = torch.empty(info["n_var"], dtype=torch.complex128, device="cuda")
    T.init_state(T.tier0_operator(R0), y, s)
    work = torch.empty(info["work_bytes_fp64"], dtype=torch.uint8, device="cuda")
    n0 = info["tier0_size"]
    out = [T.tier0_expand(y[:n0].cpu().numpy())]
    done = 0
    while done < nsteps:
        k = min(every, nsteps - done)
        T.propagate(y, work, dt, k, 0, None, precision, s)
        done += k
        out.append(T.tier0_expand(y[:n0].cpu().numpy()))
    return out


def _dense_d0(R: np.ndarray, N: int) -> np.ndarray:
    D = np.empty((N + 1, N + 1), dtype=np.complex128)
    D[0, 0] = R[0, 0]
    D[0, 1:] = R[0, 1]
    D[1:, 0] = R[1, 0]
    D[1:, 1:] = R[1, 2]
    idx = np.arange(1, N + 1)
    D[idx, idx] = R[1, 1]
    return D


def _dense_d1(R: np.ndarray, w: np.ndarray) -> np.ndarray:
    """sum_i w_i U_i G[A] U_i^+ with R the slot matrix of G[A] (slots c, e_1,
    p, q) and U_i a relabeling taking molecule 1 to i."""
    N = w.size
    W = w.sum()
    D = np.empty((N + 1, N + 1), dtype=np.complex128)
    D[0, 0] = W * R[0, 0]
    D[0, 1:] = w * R[0, 1] + (W - w) * R[0, 2]
    D[1:, 0] = w * R[1, 0] + (W - w) * R[2, 0]
    D[1:, 1:] = (w[:, None] * R[1, 2] + w[None, :] * R[2, 1]
                 + (W - w[:, None] - w[None, :]) * R[2, 3])
    idx = np.arange(1, N + 1)
    D[idx, idx] = w * R[1, 1] + (W - w) * R[2, 2]
    return D


def _dense_d2(R: np.ndarray, Wm: np.ndarray) -> np.ndarray:
    """sum_{i != j} Wm_ij U_ij G[A] U_ij^+ with R the slot matrix of G[A]
    (slots c, e_1, e_2, p, q) and U_ij taking molecules (1, 2) to (i, j)."""
    N = Wm.shape[0]
    r, s = Wm.sum(axis=1), Wm.sum(axis=0)
    W = Wm.sum()
    rest = W - r - s
    D = np.empty((N + 1, N + 1), dtype=np.complex128)
    D[0, 0] = W * R[0, 0]
    D[0, 1:] = r * R[0, 1] + s * R[0, 2] + rest * R[0, 3]
    D[1:, 0] = r * R[1, 0] + s * R[2, 0] + rest * R[3, 0]
    WT = Wm.T
    D[1:, 1:] = (Wm * R[1, 2] + WT * R[2, 1]
                 + (r[:, None] - Wm) * R[1, 3] + (s[:, None] - WT) * R[2, 3]
                 + (r[None, :] - WT) * R[3, 1] + (s[None, :] - Wm) * R[3, 2]
                 + (W - r[:, None] - s[:, None] - r[None, :] - s[None, :] + Wm + WT) * R[3, 4])
    idx = np.arange(1, N + 1)
    D[idx, idx] = r * R[1, 1] + s * R[2, 2] + rest * R[3, 3]
    return D


def plan(problem, rho0: np.ndarray) -> Dict[str, bool]:
    """Which representatives the reconstruction of rho0 propagates."""
    N = int(problem.N)
    off = rho0[1:, 1:] - np.diag(np.diag(rho0[1:, 1:]))
    need = {
        "cc": rho0[0, 0] != 0,
        "ec": bool(np.any(rho0[1:, 0] != 0)),
        "ce": bool(np.any(rho0[0, 1:] != 0)),
        "ee": bool(np.any(np.diag(rho0)[1:] != 0)),
        "e12": N >= 2 and bool(np.any(off != 0)),
    }
    if need["ce"] and adjoint_preserved(problem):
        need["ec_for_ce"] = True
    return need


def reconstruct(problem, rho0: np.ndarray, dt: float, nsteps: int, every: int,
                tier0_trajectory: Optional[Callable] = None, precision: int = 0) -> Dict:
    """rho_S(t) after 0, every, 2 every, ... RK4 steps (nsteps a multiple of
    every) for an arbitrary single-excitation rho_S(0) (dense (N+1)x(N+1),
    index 0 = cavity, 1..N = molecules). problem.d is ignored (each
    representative sets its own). Returns {"rho": (n_times, N+1, N+1),
    "propagations": names of the representatives propagated}."""
    N = int(problem.N)
    if N > MAX_DENSE_N:
        raise ValueError(f"dense output for N > {MAX_DENSE_N} is not supported")
    rho0 = np.asarray(rho0, dtype=np.complex128)
    if rho0.shape != (N + 1, N + 1):
        raise ValueError("rho0 must be (N+1)x(N+1)")
    if every < 1 or nsteps % every:
        raise ValueError("nsteps must be a multiple of every")
    run = tier0_trajectory or (lambda q, R0, dt_, n_, e_: gpu_tier0_trajectory(q, R0, dt_, n_, e_, precision))
    need = plan(problem, rho0)
    adj = need.pop("ec_for_ce", False)
    traj: Dict[str, List[np.ndarray]] = {}
    for name, d, (a, b) in REPRESENTATIVES:
        want = need[name] or (name == "ec" and adj and need["ce"])
        if not want or (name == "ce" and adj):
            continue
        traj[name] = run(with_d(problem, d), slot_matrix(d, a, b), dt, nsteps, every)
    if adj and need["ce"]:
        traj["ce"] = [R.conj().T for R in traj["ec"]]
    nt = nsteps // every + 1
    w_ec, w_ce, w_ee = rho0[1:, 0], rho0[0, 1:], np.diag(rho0)[1:]
    Wm = rho0[1:, 1:] - np.diag(w_ee)
    out = np.zeros((nt, N + 1, N + 1), dtype=np.complex128)
    for k in range(nt):
        if need["cc"]:
            out[k] += rho0[0, 0] * _dense_d0(traj["cc"][k], N)
        if need["ec"]:
            out[k] += _dense_d1(traj["ec"][k], w_ec)
        if need["ce"]:
            out[k] += _dense_d1(traj["ce"][k], w_ce)
        if need["ee"]:
            out[k] += _dense_d1(traj["ee"][k], w_ee)
        if need["e12"]:
            out[k] += _dense_d2(traj["e12"][k], Wm)
    propagated = [n for n in traj if not (n == "ce" and adj)]
    return {"rho": out, "propagations": propagated, "adjoint_reduction": bool(adj and need["ce"])}
