"""Pins of the oracle's pattern enumeration and unique-variable layout.

Against: the paper's printed hierarchy sizes (Table I and Sec. VII.E,
tests/golden/table1_counts.json), the closed forms of Eqs. direct-ado-count,
canonical-count-one, uvar-count and ordering-count, the saturation thresholds
of Eqs. first-saturation, second-saturation and distinguished-thresholds,
the worked examples of Sec. IV-V, and brute-force orbit counts of the
molecule-resolved hierarchy under the relabelings that fix the distinguished
molecules.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import conventional, patterns as P

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_counts.json")))


def sig3(x):
    return float(f"{x:.2e}")


def counts(N, m, L, d):
    blocks, _, nv = P.build_layout(N, m, L, d)
    return len(blocks), nv


@pytest.mark.parametrize("row", GOLD["rounded_rows"], ids=lambda r: f"N{r['N']}")
def test_table1_rounded(row):
    N = row["N"]
    ncan, nvar = counts(min(N, 40), 1, 25, 0)
    assert sig3(ncan) == row["canonical"]
    assert sig3(nvar) == row["unique"]
    assert sig3(16 * nvar / 1e9) == row["unique_gb"]
    naive = conventional.ado_count(N, 1, 25)
    assert sig3(naive) == row["naive_ado"]
    assert sig3(16 * (N + 1) ** 2 * naive / 1e9) == row["naive_gb"]
    assert sig3(naive * (N + 1) ** 2 / nvar) == row["R"]


def test_table1_exact_symmetric():
    ex = GOLD["exact_symmetric"]
    for N, want in ex["unique"].items():
        ncan, nvar = counts(int(N), 1, 25, 0)
        assert ncan == ex["canonical_N_ge_25"]
        assert nvar == want


def test_localized_exact():
    ex = GOLD["exact_localized"]
    ncan26, nvar26 = counts(26, 1, 25, 1)
    ncan28, nvar28 = counts(28, 1, 25, 1)
    assert ncan26 == ncan28 == ex["canonical_N_ge_26"]
    assert nvar28 == ex["unique_N_ge_28"]
    assert round(16 * nvar28 / 1e6, 2) == ex["mb"]
    assert round(nvar28 / counts(28, 1, 25, 0)[1], 2) == ex["ratio_to_symmetric"]


@pytest.mark.parametrize("N,L", [(1, 4), (2, 5), (3, 6), (5, 5), (7, 10), (12, 9)])
def test_canonical_count_closed_form(N, L):
    ncan, _ = counts(N, 1, L, 0)
    assert ncan == P.canonical_count_m1(N, L)
    # per tier: restricted partition numbers p_N(l)
    pats = P.enumerate_patterns(N, 1, L, 0)
    for l in range(L + 1):
        assert sum(1 for p in pats if p.tier == l) == P.partitions_at_most(l, N)


def test_partition_numbers_textbook():
    # p(n) for n = 0..15 (OEIS A000041)
    want = [1, 1, 2, 3, 5, 7, 11, 15, 22, 30, 42, 56, 77, 101, 135, 176]
    assert [P.partitions_at_most(n, n) for n in range(16)] == want
    # partitions of 10 into at most 3 parts: 14
    assert P.partitions_at_most(10, 3) == 14


@pytest.mark.parametrize("m,L,d", [(1, 4, 0), (1, 5, 1), (2, 3, 0), (2, 3, 1), (3, 2, 2), (1, 3, 2)])
def test_saturation_thresholds(m, L, d):
    seq = {N: counts(N, m, L, d) for N in range(max(d, 1), L + d + 6)}
    for N in seq:
        if N >= L + d:
            assert seq[N][0] == seq[L + d][0]          # patterns saturate
        if N >= L + d + 2:
            assert seq[N][1] == seq[L + d + 2][1]      # unique variables saturate
    # and not before (the thresholds are sharp for these structures)
    if L + d - 1 >= max(d, 1):
        assert seq[L + d - 1][0] < seq[L + d][0]
    assert seq[L + d + 1][1] < seq[L + d + 2][1]


def test_uvar_count_formula():
    for (N, m, L, d) in [(4, 1, 3, 0), (10, 1, 6, 0), (6, 2, 4, 1), (5, 3, 3, 2)]:
        blocks, _, nv = P.build_layout(N, m, L, d)
        total = 0
        for b in blocks:
            G = len(b.cats)
            h = sum(1 for c in b.cats if c.mult >= 2)
            assert b.size == P.uvar_count_of(G, h) == 1 + 3 * G + G * (G - 1) + h
            assert sum(c.mult for c in b.cats) == N                 # Eq. multiplicity-molecule-sum
            assert sum(c.mult * sum(c.vec) for c in b.cats) == b.pattern.tier  # Eq. multiplicity-tier-sum
            total += b.size
        assert total == nv


def test_worked_example_21():
    # Sec. IV.A: [2,1] at N = 4 stands for 12 labels; Sec. V.A: 17 of 25
    # entries are distinct, and still 17 at N = 10 (121 entries).
    p = P.Pattern((), ((2,), (1,)))
    assert P.ordering_count(p, 4, 1) == 12
    for N in (4, 10):
        blocks, where, _ = P.build_layout(N, 1, 3, 0)
        b = where[p]
        assert [c.mult for c in b.cats] == [1, 1, N - 2]
        assert [c.vec for c in b.cats] == [(2,), (1,), (0,)]
        assert b.size == 17


def test_pattern_order_start():
    # Eq. global-R: empty, [1], [2], [1,1], ...
    pats = P.enumerate_patterns(5, 1, 3, 0)
    assert [p.pool for p in pats[:4]] == [(), ((1,),), ((2,),), ((1,), (1,))]


def _orbit_counts(N, m, L, d):
    """Brute force: canonical classes of conventional labels and classes of
    (label, row, column) entries under relabelings of molecules d..N-1."""
    labs = conventional.labels(N, m, L)
    perms = list(itertools.permutations(range(d, N)))
    lab_classes, entry_classes = set(), set()
    D = N + 1
    for n in labs:
        vecs = [tuple(n[i * m:(i + 1) * m]) for i in range(N)]
        images = []
        for pm in perms:
            full = list(range(d)) + list(pm)          # molecule i -> full[i]
            new = [None] * N
            for i in range(N):
                new[full[i]] = vecs[i]
            images.append((tuple(new), full))
        lab_classes.add(min(img for img, _ in images))
        for a in range(D):
            for b in range(D):
                best = None
                for img, full in images:
                    a2 = 0 if a == 0 else 1 + full[a - 1]
                    b2 = 0 if b == 0 else 1 + full[b - 1]
                    key = (img, a2, b2)
                    if best is None or key < best:
                        best = key
                entry_classes.add(best)
    return len(lab_classes), len(entry_classes)


@pytest.mark.parametrize("N,m,L,d", [(3, 1, 3, 0), (4, 1, 3, 0), (4, 2, 2, 0), (4, 1, 3, 1),
                                     (3, 2, 2, 1), (4, 1, 2, 2), (5, 1, 2, 0)])
def test_brute_force_orbits(N, m, L, d):
    ncan, nvar = counts(N, m, L, d)
    nlab, nent = _orbit_counts(N, m, L, d)
    assert ncan == nlab
    assert nvar == nent


def test_direct_ado_count():
    for (N, m, L) in [(2, 1, 3), (3, 2, 3), (4, 1, 4), (2, 3, 3)]:
        assert len(conventional.labels(N, m, L)) == math.comb(N * m + L, L)
