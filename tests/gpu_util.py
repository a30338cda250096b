"""Helpers for the GPU tests: device memory through torch, calls through the
C ABI binding."""
import math

import numpy as np


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def upload(p):
    """Build tables for problem p and upload them; returns (tables, torch)."""
    torch = torch_cuda()
    from paper_2608_20657_amd import heom
    T = heom.Tables(p)
    info = T.info()
    buf = torch.empty(info["table_bytes"], dtype=torch.uint8, device="cuda")
    T.upload(buf, torch.cuda.current_stream())
    return T, torch


def gpu_rhs(T, torch, y: np.ndarray) -> np.ndarray:
    yd = torch.from_numpy(np.ascontiguousarray(y)).to("cuda")
    dy = torch.empty_like(yd)
    T.rhs(yd, dy, torch.cuda.current_stream())
    torch.cuda.synchronize()
    return dy.cpu().numpy()


def gpu_propagate(T, torch, tier0: np.ndarray, dt: float, steps: int, every: int, precision: int = 0,
                  check_status: bool = True):
    info = T.info()
    s = torch.cuda.current_stream()
    y = torch.empty(info["n_var"], dtype=torch.complex128, device="cuda")
    T.init_state(tier0, y, s)
    wbytes = info["work_bytes_fp64"] if precision == 0 else info["work_bytes_fp32"]
    work = torch.empty(wbytes, dtype=torch.uint8, device="cuda")
    nobs = steps // every + 1 if every > 0 else 0
    obs = torch.zeros(max(nobs, 1) * 10, dtype=torch.float64, device="cuda")
    T.propagate(y, work, dt, steps, every, obs if every > 0 else None, precision, s)
    if check_status:
        T.work_status(work, s)        # raises if a grid barrier timed out
    torch.cuda.synchronize()
    return y.cpu().numpy(), obs.cpu().numpy().reshape(-1, 10)[:nobs]


def rhs_bound(A, y: np.ndarray, c: float = 1e-13) -> np.ndarray:
    """Elementwise rounding-error scale of A @ y: c * (|A| @ |y|)."""
    return c * (abs(A) @ np.abs(y)) + 1e-300


def named_tier0(T, p, state: str) -> np.ndarray:
    if state == "photon":
        return T.tier0_pure(1.0, 0.0, [0.0] * p.d)
    if state == "site1":
        return T.tier0_pure(0.0, 0.0, [1.0] + [0.0] * (p.d - 1))
    if state == "upper_polariton":
        th = 0.5 * math.atan2(2 * p.g * math.sqrt(p.N), p.omega_c - p.eps)
        return T.tier0_pure(math.cos(th), math.sin(th) / math.sqrt(p.N), [math.sin(th) / math.sqrt(p.N)] * p.d)
    raise ValueError(state)


def mirror_permutation(S) -> np.ndarray:
    """For every unique variable of the oracle system S, the index of the
    entry with row and column categories exchanged (Z, P_q and T_q map to
    themselves): the conjugate partner of the entry in a Hermitian ADO."""
    perm = np.arange(S.n_var)
    by_G = {}
    for b in S.blocks:
        by_G.setdefault(b.G, []).append(b.offset)
    for G, offs in by_G.items():
        G1 = G + 1
        A, B = np.divmod(np.arange(G1 * G1), G1)
        offs = np.asarray(offs, dtype=np.int64)[:, None]
        perm[(offs + np.arange(G1 * G1)[None, :]).ravel()] = (offs + (B * G1 + A)[None, :]).ravel()
    return perm


def hermitian_vector(S, seed: int) -> np.ndarray:
    """Seeded random state whose every ADO is Hermitian: entry (A,B) is the
    conjugate of entry (B,A); diagonal entries and T_q are real."""
    from paper_2608_20657_amd import workloads as W
    y = W.random_vector(S.n_var, seed)
    return 0.5 * (y + np.conj(y[mirror_permutation(S)]))


def gpu_rhs_prec(T, torch, y: np.ndarray, precision: int) -> np.ndarray:
    """heom_rhs at the given precision flags: complex128 in/out (FP64) or
    complex64 in/out (FP32)."""
    dt = np.complex64 if (precision & 1) else np.complex128
    yd = torch.from_numpy(np.ascontiguousarray(y.astype(dt))).to("cuda")
    dy = torch.empty_like(yd)
    T.rhs(yd, dy, torch.cuda.current_stream(), precision=precision)
    torch.cuda.synchronize()
    return dy.cpu().numpy()
