"""Host-side rules of the continuous-batching server: lane choice, request
footprints, admission against slots and a byte budget, chunk length."""
import numpy as np
import pytest

from paper_2608_20657_amd import serve as S


def test_lane_of_thresholds():
    th = [100, 10_000]
    assert S.lane_of(1, th) == 0
    assert S.lane_of(99, th) == 0
    assert S.lane_of(100, th) == 1
    assert S.lane_of(9_999, th) == 1
    assert S.lane_of(10_000, th) == 2
    assert S.lane_of(5, []) == 0


def test_request_bytes_counts_every_buffer():
    # 46 variables (the two-molecule workload): state 736 B, work, params, 21 observable rows
    nb = S.request_bytes(46, 131_328 + 46 * 32, 4096, 2000, 100)
    assert nb == S._round(736) + S._round(131_328 + 1472) + 4096 + S._round(21 * 10 * 8)
    assert nb % S.ALIGN == 0


def test_structure_key_saturates():
    class P:
        pass
    a, b, c = P(), P(), P()
    for x, N in ((a, 40), (b, 10 ** 6), (c, 7)):
        x.N, x.m, x.L, x.d = N, 3, 8, 0
    assert S.structure_key(a) == S.structure_key(b) == (10, 3, 8, 0)
    assert S.structure_key(c) == (7, 3, 8, 0)


def test_admission_fifo_on_memory():
    tb = {"A": 500, "B": 600}
    w = [(0, 0, 100, "A"), (1, 1, 50, "B"), (2, 0, 10, "A")]
    # request 1 does not fit after 0: it blocks 2 although 2 would fit
    adm, ev = S.plan_admission(w, {0: 2, 1: 2}, 1000, {}, [], tb, 2000)
    assert adm == [0] and ev == []
    # enough memory: everything in arrival order, each image counted once
    adm, ev = S.plan_admission(w, {0: 2, 1: 2}, 1260, {}, [], tb, 2000)
    assert adm == [0, 1, 2]


def test_admission_slots_let_other_lanes_pass():
    tb = {"A": 0, "B": 0}
    w = [(0, 0, 10, "A"), (1, 0, 10, "A"), (2, 1, 10, "B")]
    adm, _ = S.plan_admission(w, {0: 1, 1: 1}, 10 ** 6, {}, [], tb, 10 ** 9)
    assert adm == [0, 2]
    adm, _ = S.plan_admission(w, {0: 0, 1: 0}, 10 ** 6, {}, [], tb, 10 ** 9)
    assert adm == []


def test_admission_evicts_unused_images_lru():
    tb = {"A": 400, "B": 400, "C": 400}
    # A and B resident and unused (A least recently used); C needs 400 + 100
    adm, ev = S.plan_admission([(7, 0, 100, "C")], {0: 1}, 150, {"A": 400, "B": 400}, ["A", "B"], tb, 2000)
    assert adm == [7] and ev == ["A"]
    # a resident image is reused without its bytes
    adm, ev = S.plan_admission([(8, 0, 100, "A")], {0: 1}, 150, {"A": 400}, ["A"], tb, 2000)
    assert adm == [8] and ev == []


def test_admission_skips_what_can_never_fit():
    adm, _ = S.plan_admission([(0, 0, 5000, "A"), (1, 0, 10, "A")], {0: 2}, 100, {}, [], {"A": 20}, 1000)
    assert adm == [1]


def test_chunk_steps():
    assert S.chunk_steps([], None, 25.0) == 0
    assert S.chunk_steps([100, 40], None, 25.0, first=8) == 8
    assert S.chunk_steps([100, 40], 0.5, 25.0) == 40          # never past the nearest horizon
    assert S.chunk_steps([1000], 0.5, 25.0) == 50
    assert S.chunk_steps([1000], 100.0, 25.0) == 1            # at least one step
    assert S.chunk_steps([10 ** 6], 1e-6, 25.0, cap=4096) == 4096


def test_make_requests_rounds_horizon():
    class P:
        pass
    ps = []
    for h in (1000, 1234, 19_999):
        p = P()
        p.horizon = h
        ps.append(p)
    rs = S.make_requests(ps, [0.0, 0.5, 1.0], dt=0.02, obs_every=100)
    assert [r.horizon for r in rs] == [1000, 1300, 20_000]
    assert [r.arrival for r in rs] == [0.0, 0.5, 1.0]


def test_summarize_percentiles():
    rs = [S.Result(i, 0.0, 0.0, float(i + 1), None, 1) for i in range(100)]
    st = S.summarize(rs, 103, 50.0, outstanding=3)
    assert st["completed"] == 100 and st["outstanding"] == 3
    assert st["solves_per_s"] == pytest.approx(2.0)
    assert st["p50_latency_s"] == pytest.approx(50.5)
    assert st["p99_latency_s"] == pytest.approx(99.01)


def test_summarize_censors_unfinished_requests():
    # two finished after 1 s, two never finished in a 10 s run (arrived at 0 and 4 s)
    rs = [S.Result(0, 0.0, 0.0, 1.0, None, 1), S.Result(1, 2.0, 2.0, 3.0, None, 1)]
    st = S.summarize(rs, [(0, 0.0), (1, 2.0), (2, 0.0), (3, 4.0)], 10.0, outstanding=2)
    assert st["submitted"] == 4 and st["completed"] == 2
    assert st["p50_latency_s"] == pytest.approx(1.0)
    # all latencies: 1, 1, 10, 6 -> median 3.5
    assert st["p50_latency_all_lower_bound_s"] == pytest.approx(3.5)


def test_predicted_step_time_scales_up_only():
    assert S.predicted_ms_per_step(None, 0, 100) is None
    assert S.predicted_ms_per_step(2.0, 1000, 1000) == 2.0
    assert S.predicted_ms_per_step(2.0, 1000, 500) == 2.0          # fewer variables: keep (shorter chunks)
    assert S.predicted_ms_per_step(2.0, 1000, 50_000) == pytest.approx(100.0)
    # a 17 M-variable request joining small ones: its first chunk is sized
    # for its own step time, not for 4096 small steps
    k = S.chunk_steps([20_000], S.predicted_ms_per_step(0.02, 20_000, 17_000_000), 25.0)
    assert k == 1


def test_hermitian_request_rule():
    from paper_2608_20657_amd import workloads as W
    ok = W.random_problem(5, 2, 3, 1, seed=1, complex_check=False)
    bad = W.random_problem(5, 2, 3, 1, seed=1, complex_check=True)
    assert S.hermitian_request_ok(ok, None)
    assert not S.hermitian_request_ok(bad, None)
    R = np.array([[0.7, 0.2 + 0.1j, 0, 0], [0.2 - 0.1j, 0.3, 0, 0], [0, 0, 0, 0], [0, 0, 0, 0]])
    assert S.hermitian_request_ok(ok, R)
    R2 = R.copy()
    R2[0, 1] = 0.2 - 0.1j                  # |c><e_1| coherence not matched by its adjoint
    assert not S.hermitian_request_ok(ok, R2)
