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
read back and turned into the representative's slot matrix (cavity,
distinguished molecules, two pool molecules; heom_tier0_expand). The dense
rho_S(t) of each output time, the weighted sum of the relabeled responses,
is formed on the device by heom_reconstruct_dense from rho_S(0) and the
five slot matrices: one pass over the (N+1)^2 entries, the quadratic cost
of the requested output, not of the propagation.
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


# packing of the five slot matrices for heom_reconstruct_dense: (name,
# slots, mask bit), in the order of REPRESENTATIVES
PACK = [("cc", 3, 1), ("ec", 4, 2), ("ce", 4, 4), ("ee", 4, 8), ("e12", 5, 16)]


def pack_slots(resp: Dict[str, np.ndarray]) -> np.ndarray:
    """The responses present in `resp` packed as heom_reconstruct_dense reads
    them (absent ones as zeros)."""
    out = []
    for name, n, _ in PACK:
        R = resp.get(name)
        R = np.zeros((n, n), dtype=np.complex128) if R is None else np.asarray(R, dtype=np.complex128)
        if R.shape != (n, n):
            raise ValueError(f"slot matrix {name} must be {n}x{n}")
        out.append(np.ascontiguousarray(R).view(np.float64).ravel())
    return np.concatenate(out)


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
    import torch
    from . import heom
    run = tier0_trajectory or (lambda q, R0, dt_, n_, e_: gpu_tier0_trajectory(q, R0, dt_, n_, e_, precision))
    need = plan(problem, rho0)
    adj = need.pop("ec_for_ce", False)
    traj: Dict[str, List[np.ndarray]] = {}
    for name, d, (a, b) in REPRESENTATIVES:
        want = need[name] or (name == "ec" and adj and need["ce"])
        if not want or (name == "ce" and adj):
            continue
        traj[name] = run(with_d(problem, d), slot_matrix(d, a, b), dt, nsteps, every)
    mask = sum(bit for name, _, bit in PACK if need[name])
    if adj and need["ce"]:
        mask |= heom.HEOM_RECON_CE_ADJOINT
    nt = nsteps // every + 1
    s = torch.cuda.current_stream()
    rho0_dev = torch.from_numpy(np.ascontiguousarray(rho0)).to("cuda")
    work = torch.empty(heom.reconstruct_work_bytes(N), dtype=torch.uint8, device="cuda")
    dense = torch.empty((N + 1, N + 1), dtype=torch.complex128, device="cuda")
    out = np.zeros((nt, N + 1, N + 1), dtype=np.complex128)
    for k in range(nt):
        R = pack_slots({name: tr[k] for name, tr in traj.items()})
        heom.reconstruct_dense(N, rho0_dev, R, mask, work, dense, s)
        out[k] = dense.cpu().numpy()
    propagated = list(traj)
    return {"rho": out, "propagations": propagated, "adjoint_reduction": bool(adj and need["ce"])}
