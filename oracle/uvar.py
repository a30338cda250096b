"""Unique-variable generator M_u of the symmetry-adapted HEOM (oracle; test
infrastructure only).

Each row of M_u is the time derivative of one unique variable
V = <a|R_Lambda|b> (Eq. generic-uvar), written from the paper's equations:

* system part: the matrix element of -i[H_S, R_Lambda] (Eq. HS), where the
  sum over intermediate basis states runs over the cavity and over all N
  molecules. Molecules of one category carry identical entries
  (Eq. within-representative), so the sum is taken category by category:
  the molecules a and b themselves are kept apart and the remaining members of
  a category are counted with their multiplicity -- the grouped sums of
  Eqs. grouped-row-sum and grouped-column-sum;
* damping -Gamma_Lambda V with Gamma_Lambda = sum over molecules and
  channels of n_ik nu_k (Eq. tier-damping);
* cavity loss -(kappa/2) <a|{|c><c|, R}|b> and the optional terminator
  -Delta sum_i <a|[Q_i,[Q_i,R]]|b> (the same terms as the conventional
  oracle);
* hierarchy: Eqs. uvar-up and uvar-down. Because of the Kronecker deltas of
  Eq. projector-commutator-element only the row molecule a (row term) and
  the column molecule b (column term) contribute. Each term reads one entry
  of an aligned target (Eq. aligned-accessor): the raw target label is
  n^Lambda with molecule i's local vector raised or lowered in channel k
  (Eqs. raw-target-*), its canonical pattern Lambda' = C(m) is a stored block,
  and the entry <x|R^[m]|y> of the aligned target is the entry of R_Lambda'
  whose row and column molecules carry, in Lambda', the local vectors that x
  and y carry in the raw label (Eqs. aligned-target, central-covariance).

Molecules are referenced symbolically as (category q, member j), so N may be
huge (only multiplicities enter). For small N, `expand` / `compress` map
between unique variables and the full conventional hierarchy; the tests pin
this generator by checking expand(M_u u) == A_conv expand(u) for random u,
and that expand(u) obeys Eq. central-covariance.

Parity: pinned by tests/test_oracle_uvar.py.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Tuple

import numpy as np
import scipy.sparse as sp

from .patterns import (Block, Pattern, build_layout, canonical, is_zero)

CAV = None  # the cavity basis state |c>
Mol = Tuple[int, int]  # (category, member)


class UVarSystem:
    """Layout plus generator rows for one problem."""

    def __init__(self, p):
        self.p = p
        self.N, self.m, self.L, self.d = p.N, p.m, p.L, p.d
        self.blocks, self.where, self.n_var = build_layout(p.N, p.m, p.L, p.d)
        self.a = [abs(complex(ck)) for ck in p.c]
        self._target_cache: Dict[tuple, Tuple[Block, tuple]] = {}

    # ----------------------------------------------------------- entries
    @staticmethod
    def entry(blk: Block, cx: Optional[int], cy: Optional[int], same: bool) -> int:
        """Index of the unique variable holding <x|R|y> when x lies in
        category cx and y in category cy (None = cavity); `same` says whether
        x and y are the same molecule."""
        if cx is None and cy is None:
            return blk.mat(0, 0)                      # Z
        if cy is None:
            return blk.mat(cx + 1, 0)                 # X_cx
        if cx is None:
            return blk.mat(0, cy + 1)                 # Y_cy
        if same:
            return blk.mat(cx + 1, cx + 1)            # P_cx
        if cx == cy:
            return blk.T(cx)                          # T_cx
        return blk.mat(cx + 1, cy + 1)                # S_cx,cy

    def variables(self, blk: Block):
        """(global index, row basis state a, column basis state b) for every
        unique variable of the block, with representative molecules."""
        out = []
        G = blk.G
        for A in range(G + 1):
            for B in range(G + 1):
                # member 0 of each category; A == B >= 1 is then the same
                # molecule (P), A != B two different molecules (S)
                a = CAV if A == 0 else (A - 1, 0)
                b = CAV if B == 0 else (B - 1, 0)
                out.append((blk.mat(A, B), a, b))
        for q in blk.t_index:
            out.append((blk.T(q), (q, 0), (q, 1)))
        return out

    @staticmethod
    def _cat(x: Optional[Mol]) -> Optional[int]:
        return None if x is None else x[0]

    def read(self, blk: Block, x, y) -> int:
        return self.entry(blk, self._cat(x), self._cat(y), x is not None and x == y)

    # ------------------------------------------------------ grouped sums
    def sum_molecules(self, blk: Block, specials, f) -> List[Tuple[float, int]]:
        """sum over all N molecules x of f(x), where f(x) is a variable index
        that depends only on x's category and on whether x coincides with one
        of `specials`. Returns (weight, index) pairs."""
        out = []
        for q, cat in enumerate(blk.cats):
            sp_members = sorted({s[1] for s in specials if s is not None and s[0] == q})
            for j in sp_members:
                out.append((1.0, f((q, j))))
            generic = cat.mult - len(sp_members)
            if generic > 0:
                j = 0
                while j in sp_members:
                    j += 1
                out.append((float(generic), f((q, j))))
        return out

    # ------------------------------------------------------ aligned target
    def target(self, blk: Block, q: int, k: int, sign: int):
        """Raw target of moving one molecule of category q by sign*e_k:
        returns (target block, category map) where the map takes a source
        molecule to its category in the target."""
        key = (blk.offset, q, k, sign)
        hit = self._target_cache.get(key)
        if hit is not None:
            return hit
        cat = blk.cats[q]
        new_vec = list(cat.vec)
        new_vec[k] += sign
        new_vec = tuple(new_vec)
        dist = list(blk.pattern.dist)
        pool = list(blk.pattern.pool)
        if cat.dist_label is not None:
            dist[cat.dist_label] = new_vec
        else:
            if not is_zero(cat.vec):
                pool.remove(cat.vec)
            pool.append(new_vec)
        tgt = self.where[canonical(dist, pool)]
        # category lookup in the target: distinguished by label, pool by vector
        by_label = {c.dist_label: t for t, c in enumerate(tgt.cats) if c.dist_label is not None}
        by_vec = {c.vec: t for t, c in enumerate(tgt.cats) if c.dist_label is None}
        res = (tgt, by_label, by_vec, new_vec)
        self._target_cache[key] = res
        return res

    def accessor(self, blk: Block, i: Mol, k: int, sign: int, x, y) -> int:
        """<x| R^[m] |y> for the raw target m = n^Lambda +- e_ik, returned as a
        unique-variable index of the canonical target."""
        tgt, by_label, by_vec, new_vec = self.target(blk, i[0], k, sign)

        def cat_of(z):
            if z is None:
                return None
            c = blk.cats[z[0]]
            if c.dist_label is not None:
                return by_label[c.dist_label]
            vec = new_vec if z == i else c.vec
            return by_vec[vec]

        return self.entry(tgt, cat_of(x), cat_of(y), x is not None and x == y)

    # ------------------------------------------------------------- rows
    def row(self, blk: Block, a, b) -> List[Tuple[complex, int]]:
        """Nonzero contributions (coefficient, source index) to d<a|R|b>/dt."""
        p = self.p
        out: List[Tuple[complex, int]] = []
        specials = [s for s in (a, b) if s is not None]

        # -i [H_S, R]_{ab} = -i (sum_x H_ax R_xb - sum_x R_ax H_xb)
        if a is None:
            out.append((-1j * p.omega_c, self.read(blk, CAV, b)))
            for w, j in self.sum_molecules(blk, specials, lambda x: self.read(blk, x, b)):
                out.append((-1j * p.g * w, j))
        else:
            out.append((-1j * p.eps, self.read(blk, a, b)))
            out.append((-1j * p.g, self.read(blk, CAV, b)))
        if b is None:
            out.append((1j * p.omega_c, self.read(blk, a, CAV)))
            for w, j in self.sum_molecules(blk, specials, lambda x: self.read(blk, a, x)):
                out.append((1j * p.g * w, j))
        else:
            out.append((1j * p.eps, self.read(blk, a, b)))
            out.append((1j * p.g, self.read(blk, a, CAV)))

        own = self.read(blk, a, b)
        # damping: sum over molecules and channels of n_ik nu_k
        counts = [sum(c.mult * c.vec[k] for c in blk.cats) for k in range(self.m)]
        gamma = 0.0
        for k in range(self.m):
            gamma += p.nu[k] * counts[k]
        out.append((-gamma + 0j, own))
        # cavity loss: -(kappa/2)(delta_ac R_cb + R_ac delta_bc)
        if a is None:
            out.append((-0.5 * p.kappa + 0j, self.read(blk, CAV, b)))
        if b is None:
            out.append((-0.5 * p.kappa + 0j, self.read(blk, a, CAV)))
        # terminator: [Q_i,[Q_i,R]]_ab = (delta_{a,e_i} - delta_{b,e_i})^2 R_ab
        if p.terminator != 0.0:
            w = 0
            if a is not None and b is not None:
                w = 0 if a == b else 2
            elif (a is None) != (b is None):
                w = 1
            if w:
                out.append((-p.terminator * w + 0j, own))

        chi = blk.pattern.tier < self.L
        for k in range(self.m):
            if self.a[k] == 0.0:
                continue
            ck, cck = complex(p.c[k]), complex(p.c_check[k])
            # row term: i = a
            if a is not None:
                n_ik = blk.cats[a[0]].vec[k]
                if chi:
                    s = math.sqrt((n_ik + 1) * self.a[k])
                    out.append((-1j * s, self.accessor(blk, a, k, +1, a, b)))
                if n_ik > 0:
                    w = math.sqrt(n_ik / self.a[k])
                    out.append((-1j * w * ck, self.accessor(blk, a, k, -1, a, b)))
            # column term: i = b
            if b is not None:
                n_ik = blk.cats[b[0]].vec[k]
                if chi:
                    s = math.sqrt((n_ik + 1) * self.a[k])
                    out.append((1j * s, self.accessor(blk, b, k, +1, a, b)))
                if n_ik > 0:
                    w = math.sqrt(n_ik / self.a[k])
                    out.append((1j * w * cck, self.accessor(blk, b, k, -1, a, b)))
        return out

    def generator(self) -> sp.csr_matrix:
        rows, cols, vals = [], [], []
        for blk in self.blocks:
            for idx, a, b in self.variables(blk):
                for coef, j in self.row(blk, a, b):
                    rows.append(idx)
                    cols.append(j)
                    vals.append(coef)
        A = sp.csr_matrix((np.asarray(vals, dtype=np.complex128),
                           (np.asarray(rows), np.asarray(cols))),
                          shape=(self.n_var, self.n_var))
        A.sum_duplicates()
        A.eliminate_zeros()
        return A

    def rows_at(self, indices) -> Dict[int, Dict[int, complex]]:
        """Generator rows for selected variable indices only (for sampled
        checks at sizes where the full matrix is too slow to assemble)."""
        want = sorted(set(int(i) for i in indices))
        starts = [b.offset for b in self.blocks]
        out = {}
        bi = 0
        for idx in want:
            while bi + 1 < len(self.blocks) and starts[bi + 1] <= idx:
                bi += 1
            blk = self.blocks[bi]
            for vidx, a, b in self.variables(blk):
                if vidx == idx:
                    acc: Dict[int, complex] = {}
                    for coef, j in self.row(blk, a, b):
                        acc[j] = acc.get(j, 0j) + coef
                    out[idx] = {j: v for j, v in acc.items() if v != 0}
        return out

    # -------------------------------------------- tier-0 initial state
    def tier0_block(self) -> Block:
        return self.blocks[0]

    def initial_state(self, amp=None, rho=None) -> np.ndarray:
        """Factorized initial condition (Eqs. factorized-initial-*): the
        tier-0 block holds rho_S(0), higher tiers are zero. rho_S(0) is given
        either as a pure state by its amplitude function amp(i) (i = 0 for
        the cavity, 1..N for the molecules) or entrywise by rho(i, j). Each
        tier-0 variable reads rho at its representative molecules."""
        blk = self.tier0_block()
        if rho is None:
            rho = lambda i, j: amp(i) * np.conj(amp(j))
        y = np.zeros(self.n_var, dtype=np.complex128)
        for idx, a, b in self.variables(blk):
            y[idx] = rho(self.molecule_index(blk, a), self.molecule_index(blk, b))
        return y

    def molecule_index(self, blk: Block, x) -> int:
        """Basis index of a symbolic molecule in the explicit representative
        label n^Lambda (Eq. n-pattern): distinguished molecules first (labels
        1..d), then pool molecules category by category; 0 = cavity."""
        if x is None:
            return 0
        q, j = x
        c = blk.cats[q]
        if c.dist_label is not None:
            return 1 + c.dist_label
        pos = self.d
        for t in range(q):
            if blk.cats[t].dist_label is None:
                pos += blk.cats[t].mult
        return 1 + pos + j

    # ----------------------------------------- conventional correspondence
    def _label_categories(self, n_flat: Tuple[int, ...]):
        """Canonical block of a conventional label and the category (in that
        block) of every molecule."""
        m, d, N = self.m, self.d, self.N
        vecs = [tuple(n_flat[i * m:(i + 1) * m]) for i in range(N)]
        blk = self.where[canonical(vecs[:d], vecs[d:])]
        by_label = {c.dist_label: t for t, c in enumerate(blk.cats) if c.dist_label is not None}
        by_vec = {c.vec: t for t, c in enumerate(blk.cats) if c.dist_label is None}
        cats = [by_label[i] if i < d else by_vec[vecs[i]] for i in range(N)]
        return blk, cats

    def expand(self, u: np.ndarray, conv_labels) -> np.ndarray:
        """Full conventional hierarchy represented by unique variables u
        (Eq. central-covariance applied to every label)."""
        N = self.N
        D = N + 1
        out = np.zeros(len(conv_labels) * D * D, dtype=np.complex128)
        for j, n in enumerate(conv_labels):
            blk, cats = self._label_categories(n)
            cat = [None] + cats
            base = j * D * D
            for x in range(D):
                for y in range(D):
                    out[base + x * D + y] = u[self.entry(blk, cat[x], cat[y], x != 0 and x == y)]
        return out

    def compress(self, rho: np.ndarray, conv_labels) -> np.ndarray:
        """Unique variables read from a conventional hierarchy at the
        representative labels n^Lambda."""
        N, m, d = self.N, self.m, self.d
        D = N + 1
        index = {n: j for j, n in enumerate(conv_labels)}
        u = np.zeros(self.n_var, dtype=np.complex128)
        for blk in self.blocks:
            n = [0] * (N * m)
            for q, c in enumerate(blk.cats):
                for j in range(c.mult):
                    i = self.molecule_index(blk, (q, j)) - 1
                    n[i * m:(i + 1) * m] = list(c.vec)
            base = index[tuple(n)] * D * D
            for idx, a, b in self.variables(blk):
                u[idx] = rho[base + self.molecule_index(blk, a) * D + self.molecule_index(blk, b)]
        return u
