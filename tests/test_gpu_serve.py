"""GPU tests of the continuous-batching server.

Each request's observable trajectory must be the same alone, in the mix
(other requests admitted and retired around it, a byte budget that makes
admission wait) and through the plain one-at-a-time heom_propagate path:
bitwise in FP64, and in FP32-bulk bitwise between alone and mix, within
1e-5 absolute of FP64 on populations. One served request is checked against
the CPU oracle directly.
"""
import copy

import numpy as np
import pytest

from oracle import integrate, observables as O, uvar
from paper_2608_20657_amd import workloads as W
from tests.gpu_util import torch_cuda

pytestmark = pytest.mark.gpu

# (N, m, L, d); N=20 and N=50 at (m, L, d) = (2, 4, 0) share a structure key
SHAPES = [(20, 2, 4, 0), (50, 2, 4, 0), (5, 1, 3, 1), (64, 2, 6, 1), (9, 3, 3, 0), (4, 1, 2, 2),
          (12, 1, 5, 0), (30, 2, 4, 0), (7, 4, 3, 0), (16, 2, 5, 1)]
POPS = [1, 2, 4, 5, 6]       # population columns of the observable rows (cavity, excitonic, bright, dark, ...)


def requests(every=20):
    from paper_2608_20657_amd import serve as S
    rng = np.random.default_rng(5)
    out = []
    for i, (N, m, L, d) in enumerate(SHAPES):
        p = W.random_problem(N, m, L, d, seed=100 + i, loss=True)
        p.g *= 0.2
        h = every * int(rng.integers(2, 9))
        out.append(S.Request(i, p, h, 0.01 + 0.002 * i, every, arrival=0.02 * i))
    return out


def run_server(reqs, precision, budget=None, lanes=(2000,), capacity=(3, 2)):
    torch = torch_cuda()
    from paper_2608_20657_amd import serve as S
    srv = S.Server(torch, budget or (64 << 30), lanes=lanes, capacity=list(capacity), precision=precision,
                   target_ms=1.0)
    srv.prepare([r.problem for r in reqs])
    st = srv.run(reqs)
    return {r.rid: r for r in srv.results}, st, srv


def tight_budget(reqs):
    """A budget that holds any single request with its image but not all of them."""
    torch = torch_cuda()
    from paper_2608_20657_amd import serve as S
    srv = S.Server(torch, 1 << 40)
    need = []
    for r in reqs:
        nb, s = srv.footprint(r)
        need.append(nb + s.table_bytes)
    return max(need) + sorted(need)[-2] // 2, sum(need)


@pytest.mark.parametrize("precision", [0, 1])
def test_served_equals_alone(precision):
    reqs = requests()
    budget, total = tight_budget(reqs)
    assert budget < total
    res, st, srv = run_server(reqs, precision, budget=budget)
    assert st["completed"] == len(reqs) and st["rejected"] == 0 and st["outstanding"] == 0
    assert st["peak_bytes"] <= budget
    assert st["peak_in_flight"] < len(reqs)          # admission waited for memory or slots
    for r in reqs:
        alone, st1, _ = run_server([copy.copy(r)], precision)
        a = alone[r.rid].obs
        b = res[r.rid].obs
        assert a.shape == (r.horizon // r.obs_every + 1, 10)
        assert np.array_equal(a, b), f"request {r.rid} differs alone vs in the mix"


def test_served_equals_plain_fifo_fp64():
    torch = torch_cuda()
    from paper_2608_20657_amd import serve as S
    reqs = requests()
    res, st, _ = run_server(reqs, 0)
    fifo = S.Fifo(torch, precision=0, chunk=40)
    fifo.prepare([r.problem for r in reqs])
    st2 = fifo.run(reqs)
    assert st2["completed"] == len(reqs)
    for r in fifo.results:
        assert np.array_equal(r.obs, res[r.rid].obs), f"request {r.rid}: served != plain"


def test_served_fp32_within_tolerance_of_fp64():
    reqs = requests()
    r64, _, _ = run_server(reqs, 0)
    r32, _, _ = run_server(reqs, 1)
    for r in reqs:
        a, b = r64[r.rid].obs, r32[r.rid].obs
        assert np.abs(a[:, POPS] - b[:, POPS]).max() <= 1e-5


def test_served_request_against_oracle():
    reqs = requests()
    res, _, _ = run_server(reqs, 0)
    r = reqs[2]                                    # (5, 1, 3, 1)
    S = uvar.UVarSystem(r.problem)
    y0 = S.initial_state(amp=lambda i: 1.0 if i == 0 else 0.0)
    _, ref = integrate.propagate(S.generator(), y0, r.dt, r.horizon, r.obs_every,
                                 observe=lambda v: O.from_tier0(S, v))
    ref = np.array(ref)
    got = res[r.rid].obs
    for j in range(9):
        assert np.abs(got[:, j] - ref[:, j]).max() <= 1e-10 * max(np.abs(ref[:, j]).max(), 1e-300)


def test_rejects_what_cannot_fit():
    torch = torch_cuda()
    from paper_2608_20657_amd import serve as S
    reqs = requests()[:2]
    srv = S.Server(torch, 4096)
    st = srv.run(reqs)
    assert st["completed"] == 0 and st["rejected"] == 2


def test_served_hermitian_compact_equals_fifo_and_matches_general():
    """Under HEOM_HERMITIAN the server and the FIFO build compact tiles; the
    requests (Hermitian rho_S(0), c_check = conj(c)) then agree bitwise
    between served and plain, and with the general path to rounding."""
    torch = torch_cuda()
    from paper_2608_20657_amd import heom, serve as S
    reqs = requests()
    herm = heom.HEOM_HERMITIAN
    res_h, st, srv = run_server(reqs, herm)
    assert st["completed"] == len(reqs)
    assert all(s.tables.info()["compact"] == 1 for s in srv.structs.values())
    fifo = S.Fifo(torch, precision=herm, chunk=40)
    fifo.prepare([r.problem for r in reqs])
    assert fifo.run(reqs)["completed"] == len(reqs)
    for r in fifo.results:
        assert np.array_equal(r.obs, res_h[r.rid].obs), f"request {r.rid}: served != plain"
    res_g, _, _ = run_server(reqs, 0)
    for r in reqs:
        a, b = res_g[r.rid].obs, res_h[r.rid].obs
        assert np.abs(a - b).max() <= 1e-12 * max(1.0, np.abs(a).max())
