"""Serialized canonical form of the oracle's tables, in the format of
heom_export_layout (include/heom.h), for bit-exact comparison."""
import numpy as np

from oracle import uvar


def serialize(S: uvar.UVarSystem) -> np.ndarray:
    v = [len(S.blocks), S.n_var, S.m, S.d]
    index = {id(b): i for i, b in enumerate(S.blocks)}
    for b in S.blocks:
        v += [b.offset, b.G, b.pattern.tier]
        for c in b.cats:
            v += [c.dist_label if c.dist_label is not None else -1, c.mult] + list(c.vec)
    for b in S.blocks:
        chi = b.pattern.tier < S.L
        for q, c in enumerate(b.cats):
            for k in range(S.m):
                for sign in (+1, -1):
                    if sign > 0 and not chi:
                        continue
                    if sign < 0 and c.vec[k] == 0:
                        continue
                    tgt, by_label, by_vec, new_vec = S.target(b, q, k, sign)
                    qn = by_label[c.dist_label] if c.dist_label is not None else by_vec[new_vec]
                    v += [index[id(tgt)], qn]
                    for r, cr in enumerate(b.cats):
                        if r == q and cr.mult == 1:
                            v.append(-1)            # no unmoved member remains
                        elif cr.dist_label is not None:
                            v.append(by_label[cr.dist_label])
                        else:
                            v.append(by_vec[cr.vec])
    return np.asarray(v, dtype=np.int64)
