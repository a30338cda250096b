"""Seeded workload generators: the batched draw keeps its decay rates away
from the poles of the Drude-Lorentz coefficients (Sec. II.B)."""
import math

from paper_2608_20657_amd import workloads as W


def test_batched_draw_avoids_matsubara_poles():
    # cot(gamma / 2kT) in the Debye coefficient diverges at gamma = 2 pi k kT
    # for every k >= 1, whether or not the bath keeps a Matsubara term there
    ps = W.draw_batch(512, 0)
    assert any(q.m == 1 for q in ps)
    for q in ps:
        gam = q.nu[0]
        assert 0.02 <= gam <= 0.2
        for k in range(1, 4):
            vk = 2.0 * math.pi * k * W.KT
            assert abs(gam / vk - 1.0) >= 0.05, (gam, q.m)
        # x = gamma / 2kT lies in [0.4, 4] and 5% away from pi, so
        # |cot x| <= 1 / |sin x| <= 1 / sin(0.05 pi); lambda <= 0.05
        assert abs(q.c[0].real) <= 0.05 * gam / math.sin(0.05 * math.pi)
        for k in range(1, q.m):
            assert q.nu[k] == 2.0 * math.pi * k * W.KT


def test_batched_draw_is_seeded():
    a, b = W.draw_batch(16, 3), W.draw_batch(16, 3)
    assert [(q.N, q.m, q.L, q.g, q.nu[0]) for q in a] == [(q.N, q.m, q.L, q.g, q.nu[0]) for q in b]
    assert [(q.N, q.nu[0]) for q in a] != [(q.N, q.nu[0]) for q in W.draw_batch(16, 4)]
