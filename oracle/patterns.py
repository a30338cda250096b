"""Canonical occupation patterns and unique-variable layout (oracle; test
infrastructure only).

Paper Sec. IV (first reduction) and Sec. V.A-B (second reduction), extended
to m exponentials per bath (each molecule carries a local vector
alpha_i in N^m that moves as a whole, Sec. III and the closing paragraph of
Sec. V.D) and to d distinguished molecules (Sec. VI.B, Eq. N-symmetric-pool).

Conventions fixed here (the paper leaves them open; each is a reading):

* Order of local vectors: v > w iff (|v|, v_0, ..., v_{m-1}) > (|w|, w_0, ...)
  lexicographically. For m = 1 this is the paper's descending order
  (Eq. pattern-one).
* A pattern is (dist, pool): the vectors of the d distinguished molecules in
  label order, and the nonzero vectors of the N-d pool molecules sorted
  descending (trailing zeros dropped, Eq. pattern-one).
* Pattern order in the global vector (Eq. global-R shows only its start):
  tier ascending; then the distinguished vectors compared in label order,
  smaller vector first; then the pool lists compared entry by entry, larger
  vector first. For m = 1, d = 0 this gives empty, [1], [2], [1,1], ...
* Categories (Sec. V.A): the d distinguished molecules (multiplicity 1
  each, in label order), then the distinct nonzero pool vectors in pattern
  order, then the zero pool vector if M_0 = N - d - r >= 1 (Eq. M0).
* Block layout ("a fixed order", Sec. V.C.1): the (G+1)x(G+1) category
  matrix row-major with index 0 = cavity (Z at (0,0), Y_q at (0,q),
  X_q at (q,0), P_q at (q,q), S_{q,r} at (q,r)), followed by T_q for every
  category with M_q >= 2, in category order. Block length (G+1)^2 + h
  (Eq. uvar-count).

Parity: pinned by tests/test_oracle_counts.py against the paper's printed
counts (Table I, Sec. VII), the worked examples of Sec. IV-V, closed-form
partition counts and brute-force orbit counts of conventional labels.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from functools import lru_cache
from typing import Dict, List, Optional, Sequence, Tuple

Vec = Tuple[int, ...]


def vkey(v: Vec) -> Tuple[int, ...]:
    return (sum(v),) + tuple(v)


def zero(m: int) -> Vec:
    return (0,) * m


def is_zero(v: Vec) -> bool:
    return not any(v)


@dataclasses.dataclass(frozen=True)
class Pattern:
    dist: Tuple[Vec, ...]
    pool: Tuple[Vec, ...]

    @property
    def tier(self) -> int:
        return sum(sum(v) for v in self.dist) + sum(sum(v) for v in self.pool)


def canonical(dist: Sequence[Vec], pool_vectors: Sequence[Vec]) -> Pattern:
    """The canonicalization C of Eq. canonical-target-*: sort the nonzero pool
    vectors descending and drop the zeros; distinguished vectors stay put."""
    pool = tuple(sorted((tuple(v) for v in pool_vectors if not is_zero(v)),
                        key=vkey, reverse=True))
    return Pattern(tuple(tuple(v) for v in dist), pool)


def order_key(p: Pattern):
    return (p.tier,
            tuple(vkey(v) for v in p.dist),
            tuple(tuple(-x for x in vkey(v)) for v in p.pool))


@lru_cache(maxsize=None)
def local_vectors(m: int, L: int) -> Tuple[Vec, ...]:
    """All v in N^m with 1 <= |v| <= L, descending."""
    out = [v for v in itertools.product(range(L + 1), repeat=m) if 0 < sum(v) <= L]
    out.sort(key=vkey, reverse=True)
    return tuple(out)


def _pools(vecs: Tuple[Vec, ...], start: int, budget: int, slots: int):
    """Non-increasing lists of vectors drawn from vecs[start:], total tier
    <= budget, length <= slots."""
    yield ()
    if slots == 0:
        return
    for j in range(start, len(vecs)):
        t = sum(vecs[j])
        if t > budget:
            continue
        for rest in _pools(vecs, j, budget - t, slots - 1):
            yield (vecs[j],) + rest


def enumerate_patterns(N: int, m: int, L: int, d: int) -> List[Pattern]:
    """Every canonical pattern with |Lambda| <= L and at most N-d nonzero pool
    vectors, in the order described in the module docstring."""
    if d > N:
        raise ValueError("d > N")
    vecs = local_vectors(m, L)
    all_vecs = vecs + (zero(m),)
    out = []
    for dist in itertools.product(all_vecs, repeat=d):
        t = sum(sum(v) for v in dist)
        if t > L:
            continue
        for pool in _pools(vecs, 0, L - t, N - d):
            out.append(Pattern(tuple(dist), pool))
    out.sort(key=order_key)
    return out


@dataclasses.dataclass(frozen=True)
class Category:
    vec: Vec
    mult: int                 # M_q (Eq. Mq, Eq. M0)
    dist_label: Optional[int]  # distinguished molecule index, or None for pool


def categories(p: Pattern, N: int, m: int) -> List[Category]:
    """Categories of pattern p (module docstring), with explicit m."""
    d = len(p.dist)
    cats = [Category(v, 1, j) for j, v in enumerate(p.dist)]
    seen: Dict[Vec, int] = {}
    for v in p.pool:
        seen[v] = seen.get(v, 0) + 1
    for v in sorted(seen, key=vkey, reverse=True):
        cats.append(Category(v, seen[v], None))
    M0 = N - d - len(p.pool)
    if M0 >= 1:
        cats.append(Category(zero(m), M0, None))
    return cats


@dataclasses.dataclass
class Block:
    """Unique-variable layout of one pattern."""
    pattern: Pattern
    cats: List[Category]
    offset: int
    t_index: Dict[int, int]    # category -> position of T_q in the block

    @property
    def G(self) -> int:
        return len(self.cats)

    @property
    def h(self) -> int:
        return len(self.t_index)

    @property
    def size(self) -> int:
        return (self.G + 1) ** 2 + self.h

    def mat(self, A: int, B: int) -> int:
        """Global index of category-matrix entry (A, B); 0 = cavity,
        category q has matrix index q + 1."""
        return self.offset + A * (self.G + 1) + B

    def T(self, q: int) -> int:
        return self.offset + self.t_index[q]


def build_layout(N: int, m: int, L: int, d: int):
    """Patterns in order, their blocks, and a pattern -> block map."""
    pats = enumerate_patterns(N, m, L, d)
    blocks, where = [], {}
    off = 0
    for p in pats:
        cats = categories(p, N, m)
        G = len(cats)
        t_index, pos = {}, (G + 1) ** 2
        for q, c in enumerate(cats):
            if c.mult >= 2:
                t_index[q] = pos
                pos += 1
        b = Block(p, cats, off, t_index)
        blocks.append(b)
        where[p] = b
        off += b.size
    return blocks, where, off


# ------------------------------------------------------------ closed forms
def uvar_count_of(G: int, h: int) -> int:
    """Eq. uvar-count: 1 + 3G + G(G-1) + h = (G+1)^2 + h."""
    return (G + 1) ** 2 + h


def partitions_at_most(n: int, k: int) -> int:
    """p_k(n): partitions of n into at most k parts (Eq. canonical-count-one);
    by conjugation, the partitions of n into parts no larger than k."""
    return _p_parts_le(n, k)


@lru_cache(maxsize=None)
def _p_parts_le(n: int, k: int) -> int:
    """Partitions of n into parts each <= k (conjugate of at most k parts)."""
    if n == 0:
        return 1
    if k == 0:
        return 0
    if k > n:
        return _p_parts_le(n, n)
    return _p_parts_le(n, k - 1) + _p_parts_le(n - k, k)


def canonical_count_m1(N: int, L: int) -> int:
    """Eq. canonical-count-one: sum over tiers of restricted partition numbers."""
    return sum(partitions_at_most(l, N) for l in range(L + 1))


def ordering_count(p: Pattern, N: int, m: int) -> int:
    """Eq. ordering-count (d = 0): N! / prod_q M_q!."""
    out = math.factorial(N)
    for c in categories(p, N, m):
        out //= math.factorial(c.mult)
    return out
