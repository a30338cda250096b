// Host construction of the symmetry-adapted HEOM tables (the precomputation
// of Sec. V.C.4): local vectors, canonical patterns (Sec. IV), categories and
// multiplicities (Eqs. Mq, M0), unique-variable layout (Sec. V.A-B),
// connection records of every raise/lower move (Eqs. raw-target-*,
// canonical-target-*, aligned-target), workgroup tiles, coefficient look-up
// tables, and the packed device image.
//
// Compiled with -ffp-contract=off so that every floating-point table entry
// is the correctly ordered, unfused expression written here.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <functional>
#include <numeric>
#include <unordered_map>

#include "heom_internal.h"

namespace heom {
namespace {

// Order of local vectors: by (|v|, v_0, .., v_{m-1}).
struct VecKey {
    int m;
    bool greater(uint64_t a, uint64_t b) const {  // a > b
        uint32_t ta = 0, tb = 0;
        for (int k = 0; k < m; ++k) { ta += vcomp(a, k); tb += vcomp(b, k); }
        if (ta != tb) return ta > tb;
        for (int k = 0; k < m; ++k) {
            uint32_t x = vcomp(a, k), y = vcomp(b, k);
            if (x != y) return x > y;
        }
        return false;
    }
};

uint32_t vtier(uint64_t v, int m) {
    uint32_t t = 0;
    for (int k = 0; k < m; ++k) t += vcomp(v, k);
    return t;
}

void gen_vectors(int m, int L, int k, uint64_t cur, int budget, std::vector<uint64_t> &out) {
    if (k == m) {
        if (cur != 0) out.push_back(cur);
        return;
    }
    for (int x = 0; x <= budget; ++x)
        gen_vectors(m, L, k + 1, cur | ((uint64_t)x << (8 * k)), budget - x, out);
}

struct KeyHash {
    size_t operator()(const std::string &s) const { return std::hash<std::string>()(s); }
};

std::string key_of(const uint16_t *ids, size_t n) {
    return std::string(reinterpret_cast<const char *>(ids), n * sizeof(uint16_t));
}

}  // namespace

size_t tier0_size(const HostTables &t) { return t.hdr.empty() ? 0 : t.hdr[0].size; }

static int check_params(const heom_problem *p, std::string *err) {
    if (!p) { *err = "problem is NULL"; return HEOM_E_INVAL; }
    if (p->N < 1) { *err = "N must be >= 1"; return HEOM_E_INVAL; }
    if (p->m < 1 || p->m > HEOM_MAX_M) { *err = "m out of range 1..HEOM_MAX_M"; return HEOM_E_INVAL; }
    if (p->L < 0 || p->L > HEOM_MAX_L) { *err = "L out of range 0..HEOM_MAX_L"; return HEOM_E_INVAL; }
    if (p->d < 0 || (int64_t)p->d > p->N) { *err = "d out of range 0..N"; return HEOM_E_INVAL; }
    if (p->d >= HEOM_MAX_G) { *err = "d too large"; return HEOM_E_UNSUPPORTED; }
    if (p->reserved != 0) { *err = "reserved must be 0"; return HEOM_E_INVAL; }
    if (!p->c || !p->nu) { *err = "c and nu are required"; return HEOM_E_INVAL; }
    if (p->N > ((int64_t)1 << 52)) { *err = "N above 2^52 is not exactly representable"; return HEOM_E_UNSUPPORTED; }
    for (int k = 0; k < p->m; ++k) {
        if (!(p->nu[k] >= 0.0) || !std::isfinite(p->nu[k])) { *err = "nu_k must be finite and >= 0"; return HEOM_E_INVAL; }
        if (!std::isfinite(p->c[2 * k]) || !std::isfinite(p->c[2 * k + 1])) { *err = "c_k not finite"; return HEOM_E_INVAL; }
        if (p->c_check && (!std::isfinite(p->c_check[2 * k]) || !std::isfinite(p->c_check[2 * k + 1]))) {
            *err = "c_check_k not finite"; return HEOM_E_INVAL;
        }
    }
    const double s[5] = {p->eps, p->omega_c, p->g, p->kappa, p->terminator};
    for (double x : s)
        if (!std::isfinite(x)) { *err = "non-finite scalar parameter"; return HEOM_E_INVAL; }
    if (p->kappa < 0.0) { *err = "kappa must be >= 0"; return HEOM_E_INVAL; }
    return HEOM_OK;
}

static void copy_numeric(HostTables *t, const heom_problem *p) {
    t->prob = *p;
    t->prob.c = t->prob.c_check = t->prob.nu = nullptr;
    t->N = p->N;
    t->c.assign(p->c, p->c + 2 * p->m);
    t->nu.assign(p->nu, p->nu + p->m);
    t->cc.resize(2 * p->m);
    for (int k = 0; k < p->m; ++k) {
        if (p->c_check) {
            t->cc[2 * k] = p->c_check[2 * k];
            t->cc[2 * k + 1] = p->c_check[2 * k + 1];
        } else {
            t->cc[2 * k] = p->c[2 * k];
            t->cc[2 * k + 1] = -p->c[2 * k + 1];
        }
    }
    // coefficient look-up tables: up[k][n] = sqrt((n+1)|c_k|),
    // dn[k][n] = sqrt(n/|c_k|) (Eqs. scaled-HEOM, w-one-exp); a channel with
    // c_k = 0 is switched off.
    const int m = p->m, L = p->L;
    t->lut.assign(2 * m * (L + 1), 0.0);
    for (int k = 0; k < m; ++k) {
        double a = std::hypot(t->c[2 * k], t->c[2 * k + 1]);
        for (int n = 0; n <= L; ++n) {
            t->lut[k * (L + 1) + n] = (a == 0.0) ? 0.0 : std::sqrt((double)(n + 1) * a);
            t->lut[m * (L + 1) + k * (L + 1) + n] = (a == 0.0) ? 0.0 : std::sqrt((double)n / a);
        }
    }
}

int build(const heom_problem *p, HostTables *t, std::string *err) {
    int rc = check_params(p, err);
    if (rc) return rc;
    static std::atomic<uint64_t> next_id{1};
    t->id = next_id.fetch_add(1);
    const int m = p->m, L = p->L, d = p->d;
    const int64_t N = p->N;
    t->m = m; t->L = L; t->d = d;
    copy_numeric(t, p);

    // local vectors, descending; id = position, zero vector id = nv
    t->vecs.clear();
    gen_vectors(m, L, 0, 0, L, t->vecs);
    VecKey vk{m};
    std::sort(t->vecs.begin(), t->vecs.end(), [&](uint64_t a, uint64_t b) { return vk.greater(a, b); });
    const size_t nv = t->vecs.size();
    if (nv + 1 > 65535) { *err = "too many local vectors"; return HEOM_E_TOO_LARGE; }
    const uint16_t ZID = (uint16_t)nv;
    std::vector<uint32_t> vt(nv + 1);
    for (size_t i = 0; i < nv; ++i) vt[i] = vtier(t->vecs[i], m);
    vt[nv] = 0;
    std::unordered_map<uint64_t, uint16_t> vid;
    for (size_t i = 0; i < nv; ++i) vid[t->vecs[i]] = (uint16_t)i;
    vid[0] = ZID;

    // enumerate patterns: distinguished tuples x pool multisets
    std::vector<uint16_t> ids;
    std::vector<uint32_t> start;
    std::vector<uint8_t> tiers;
    const int64_t pool_slots64 = N - d;
    const int pool_slots = (int)std::min<int64_t>(pool_slots64, L);
    std::vector<uint16_t> dist(d), pool;
    const size_t max_patterns = (size_t)1 << 27;
    bool overflow = false;

    // recursive pool generator: non-decreasing ids (descending vectors)
    std::function<void(size_t, int, int, int)> rec_pool;
    rec_pool = [&](size_t from, int budget, int slots, int tier_so_far) {
        if (overflow) return;
        start.push_back((uint32_t)ids.size());
        ids.insert(ids.end(), dist.begin(), dist.end());
        ids.insert(ids.end(), pool.begin(), pool.end());
        tiers.push_back((uint8_t)tier_so_far);
        if (start.size() > max_patterns) { overflow = true; return; }
        if (slots == 0) return;
        for (size_t j = from; j < nv; ++j) {
            int tj = (int)vt[j];
            if (tj > budget) continue;
            pool.push_back((uint16_t)j);
            rec_pool(j, budget - tj, slots - 1, tier_so_far + tj);
            pool.pop_back();
        }
    };
    std::function<void(int, int)> rec_dist = [&](int j, int used) {
        if (overflow) return;
        if (j == d) {
            rec_pool(0, L - used, pool_slots, used);
            return;
        }
        for (size_t v = 0; v <= nv; ++v) {
            int tv = (int)vt[v];
            if (used + tv > L) continue;
            dist[j] = (uint16_t)v;
            rec_dist(j + 1, used + tv);
        }
    };
    rec_dist(0, 0);
    if (overflow) { *err = "more than 2^27 patterns"; return HEOM_E_TOO_LARGE; }
    start.push_back((uint32_t)ids.size());
    const size_t np = tiers.size();

    // canonical order: tier ascending; distinguished vectors smaller first
    // (larger id first); pool entries larger first (smaller id first)
    std::vector<uint32_t> order(np);
    std::iota(order.begin(), order.end(), 0u);
    std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        if (tiers[a] != tiers[b]) return tiers[a] < tiers[b];
        const uint16_t *pa = &ids[start[a]], *pb = &ids[start[b]];
        for (int j = 0; j < d; ++j)
            if (pa[j] != pb[j]) return pa[j] > pb[j];
        size_t na = start[a + 1] - start[a], nb = start[b + 1] - start[b];
        for (size_t j = d; j < std::min(na, nb); ++j)
            if (pa[j] != pb[j]) return pa[j] < pb[j];
        return na < nb;
    });
    t->pat_ids.clear();
    t->pat_start.clear();
    t->pat_ids.reserve(ids.size());
    for (uint32_t o : order) {
        t->pat_start.push_back((uint32_t)t->pat_ids.size());
        t->pat_ids.insert(t->pat_ids.end(), ids.begin() + start[o], ids.begin() + start[o + 1]);
    }
    t->pat_start.push_back((uint32_t)t->pat_ids.size());
    std::vector<uint8_t> tier_sorted(np);
    for (size_t i = 0; i < np; ++i) tier_sorted[i] = tiers[order[i]];
    { std::vector<uint16_t>().swap(ids); std::vector<uint32_t>().swap(start); }

    std::unordered_map<std::string, uint32_t, KeyHash> where;
    where.reserve(np * 2);
    for (size_t i = 0; i < np; ++i)
        where.emplace(key_of(&t->pat_ids[t->pat_start[i]], t->pat_start[i + 1] - t->pat_start[i]), (uint32_t)i);

    // categories, layout
    t->hdr.assign(np, PatHdr{});
    t->cat.clear();
    uint64_t off = 0;
    t->max_G = 0;
    for (size_t i = 0; i < np; ++i) {
        PatHdr &h = t->hdr[i];
        const uint16_t *pi = &t->pat_ids[t->pat_start[i]];
        size_t len = t->pat_start[i + 1] - t->pat_start[i];
        size_t r = len - d;
        h.cat_base = (uint32_t)t->cat.size();
        h.tier = tier_sorted[i];
        h.r = (uint32_t)r;
        uint64_t cnt = 0;
        int G = 0;
        uint16_t tmask = 0;
        for (int j = 0; j < d; ++j) {
            CatRec c{};
            c.vec = (pi[j] == ZID) ? 0 : t->vecs[pi[j]];
            c.mult = 1;
            c.flags = CAT_DIST;
            t->cat.push_back(c);
            ++G;
        }
        for (size_t j = d; j < len;) {
            size_t e = j;
            while (e < len && pi[e] == pi[j]) ++e;
            CatRec c{};
            c.vec = t->vecs[pi[j]];
            c.mult = (uint32_t)(e - j);
            if (c.mult >= 2) tmask |= (uint16_t)(1u << G);
            t->cat.push_back(c);
            ++G;
            j = e;
        }
        int64_t M0 = N - d - (int64_t)r;
        if (M0 >= 1) {
            CatRec c{};
            c.vec = 0;
            c.mult = 0;
            c.flags = CAT_ZERO;
            if (M0 >= 2) tmask |= (uint16_t)(1u << G);
            t->cat.push_back(c);
            ++G;
        }
        if (G > HEOM_MAX_G) { *err = "a pattern has more than HEOM_MAX_G categories"; return HEOM_E_UNSUPPORTED; }
        for (int q = 0; q < G; ++q) {
            const CatRec &c = t->cat[h.cat_base + q];
            uint64_t M = (c.flags & CAT_ZERO) ? 0 : c.mult;  // zero vector adds nothing
            for (int k = 0; k < m; ++k) cnt += ((uint64_t)(M * vcomp(c.vec, k))) << (8 * k);
        }
        h.G = (uint8_t)G;
        h.tmask = tmask;
        h.cnt = cnt;
        h.size = (uint32_t)((G + 1) * (G + 1) + __builtin_popcount(tmask));
        h.off = (uint32_t)off;
        off += h.size;
        if (off > 0xffffffffull) { *err = "more than 2^32-1 unique variables"; return HEOM_E_TOO_LARGE; }
        t->max_G = std::max(t->max_G, G);
    }
    t->n_var = (uint32_t)off;

    // connection records
    t->conn.clear();
    t->conn_target.clear();
    t->hier_gathers = 0;
    std::vector<uint16_t> tmp;
    for (size_t i = 0; i < np; ++i) {
        PatHdr &h = t->hdr[i];
        h.conn_base = (uint32_t)t->conn.size();
        const uint16_t *pi = &t->pat_ids[t->pat_start[i]];
        const size_t len = t->pat_start[i + 1] - t->pat_start[i];
        const bool chi = h.tier < L;
        const int G = h.G;
        int64_t M0 = N - d - (int64_t)h.r;
        for (int q = 0; q < G; ++q) {
            CatRec &c = t->cat[h.cat_base + q];
            c.conn_off = (uint16_t)(t->conn.size() - h.conn_base);
            for (int dir = 0; dir < 2; ++dir) {          // 0 = up, 1 = down
                if (dir == 0 && !chi) continue;
                for (int k = 0; k < m; ++k) {
                    uint32_t vk = vcomp(c.vec, k);
                    if (dir == 1 && vk == 0) continue;
                    uint64_t nvec = dir == 0 ? c.vec + ((uint64_t)1 << (8 * k)) : c.vec - ((uint64_t)1 << (8 * k));
                    uint16_t nid = vid.at(nvec);
                    tmp.assign(pi, pi + len);
                    bool vanish = false, isnew = false;
                    if (c.flags & CAT_DIST) {
                        tmp[q] = nid;                     // distinguished category q is label q
                    } else {
                        if (c.flags & CAT_ZERO) {
                            vanish = (M0 == 1);
                        } else {
                            auto it = std::find(tmp.begin() + d, tmp.end(), vid.at(c.vec));
                            tmp.erase(it);
                            vanish = (c.mult == 1);
                        }
                        if (nid != ZID) {
                            bool present = std::find(pi + d, pi + len, nid) != pi + len;
                            isnew = !present;
                            tmp.insert(std::upper_bound(tmp.begin() + d, tmp.end(), nid), nid);
                        } else {
                            isnew = (M0 < 1);
                        }
                    }
                    auto wt = where.find(key_of(tmp.data(), tmp.size()));
                    if (wt == where.end()) { *err = "internal: target pattern not found"; return HEOM_E_INVAL; }
                    const uint32_t tp = wt->second;
                    const PatHdr &th = t->hdr[tp];
                    // category of the moved molecule in the target
                    int qn;
                    if (c.flags & CAT_DIST) {
                        qn = q;
                    } else if (nid == ZID) {
                        qn = th.G - 1;                    // the zero category is last
                    } else {
                        qn = -1;
                        for (int u = d; u < th.G; ++u)
                            if (!(t->cat[th.cat_base + u].flags & CAT_ZERO) && t->cat[th.cat_base + u].vec == nvec) { qn = u; break; }
                    }
                    if (qn < 0) { *err = "internal: moved category not found"; return HEOM_E_INVAL; }
                    Conn cr;
                    cr.off = th.off;                      // block offsets are final here
                    cr.info = (uint32_t)th.G | ((uint32_t)qn << 5) | ((uint32_t)vanish << 9) |
                              ((uint32_t)isnew << 10) | ((uint32_t)th.tmask << 16);
                    // verify the remap rule against direct lookup (cheap; catches
                    // any inconsistency between the packed record and the target)
                    for (int rr = 0; rr < G; ++rr) {
                        const CatRec &sc = t->cat[h.cat_base + rr];
                        if (rr == q && vanish) continue;
                        int want;
                        if (sc.flags & CAT_DIST) want = rr;
                        else if (sc.flags & CAT_ZERO) want = th.G - 1;
                        else {
                            want = -1;
                            for (int u = d; u < th.G; ++u)
                                if (!(t->cat[th.cat_base + u].flags & CAT_ZERO) && t->cat[th.cat_base + u].vec == sc.vec) { want = u; break; }
                        }
                        if (conn_remap(cr.info, q, rr) != want) { *err = "internal: remap rule mismatch"; return HEOM_E_INVAL; }
                    }
                    t->conn.push_back(cr);
                    t->conn_target.push_back(tp);
                }
            }
        }
        // hierarchy reads of one RHS for this block (for reporting)
        int64_t g = 0;
        auto nrec = [&](int q) {
            const CatRec &c = t->cat[h.cat_base + q];
            int nz = 0;
            for (int k = 0; k < m; ++k) nz += vcomp(c.vec, k) > 0;
            return (int64_t)((chi ? m : 0) + nz);
        };
        auto ndown = [&](int q) {
            const CatRec &c = t->cat[h.cat_base + q];
            int nz = 0;
            for (int k = 0; k < m; ++k) nz += vcomp(c.vec, k) > 0;
            return (int64_t)nz;
        };
        for (int q = 0; q < G; ++q) {
            g += 2 * nrec(q);                       // X_q and Y_q
            g += ndown(q);                          // P_q
            if (h.tmask >> q & 1) g += 2 * nrec(q); // T_q
            for (int r = 0; r < G; ++r)
                if (r != q) g += nrec(q) + nrec(r); // S_qr
        }
        t->hier_gathers += g;
    }

    uint32_t maxblk = 0;
    for (auto &h : t->hdr) maxblk = std::max(maxblk, h.size);
    // default tile (measured on MI355X): 64 variables for states below 2^17
    // variables (more workgroups in flight for a latency-bound stage), 256
    // above; never below the largest block
    int tv = t->n_var <= (1u << 17) ? 64 : 256;
    while ((uint32_t)tv < maxblk) tv *= 2;
    if ((rc = make_tiles(t, tv, err))) return rc;
    t->uploaded = false;
    pack_image(t);
    return HEOM_OK;
}

// Index of the target variable <a'|R'|b'> of a connection record; a', b'
// are target categories (-1 = cavity), `same` = same molecule.
static uint32_t tgt_index(const Conn &cr, int a, int b, bool same) {
    const uint32_t G1 = conn_G(cr.info) + 1;
    if (a < 0 && b < 0) return cr.off;
    if (b < 0) return cr.off + (uint32_t)(a + 1) * G1;
    if (a < 0) return cr.off + (uint32_t)(b + 1);
    if (same) return cr.off + (uint32_t)(a + 1) * (G1 + 1);
    if (a == b) return cr.off + G1 * G1 + (uint32_t)__builtin_popcount(conn_tmask(cr.info) & ((1u << a) - 1u));
    return cr.off + (uint32_t)(a + 1) * G1 + (uint32_t)(b + 1);
}

// Append, for every unique variable of pattern p in layout order, the target
// indices of its live hierarchy gathers in slot order (see live_slots). The
// target of a move of one molecule of category q by +-e_k is read through
// the connection record of (q, k, direction): the moved molecule lies in q'
// of the target, an unmoved molecule of category r in conn_remap(q, r).
// With transposed copies (t.trcol) a column move names its target's position
// in the transposed copy, which is the row-major position of the mirrored
// entry (row and column categories exchanged; a T_q stays in place).
void expand_gathers(const HostTables &t, uint32_t p, std::vector<uint32_t> *out) {
    const PatHdr &H = t.hdr[p];
    const int G = H.G, G1 = G + 1, M = t.m;
    const bool chi = H.tier < t.L;
    const CatRec *cats = t.cat.data() + H.cat_base;
    const Conn *cons = t.conn.data() + H.conn_base;   // may be one past the end: a pattern with no moves
    auto rup = [&](const CatRec &c, int k) { return cons[c.conn_off + k]; };
    auto rdn = [&](const CatRec &c, int k) {
        uint32_t r = c.conn_off + (chi ? M : 0);
        for (int j = 0; j < k; ++j) r += vcomp(c.vec, j) != 0;
        return cons[r];
    };
    for (uint32_t loc = 0; loc < H.size; ++loc) {
        int A, B;
        bool isT = false;
        if (loc < (uint32_t)(G1 * G1)) {
            A = (int)loc / G1;
            B = (int)loc - A * G1;
        } else {
            uint32_t mask = H.tmask;
            for (int s = (int)loc - G1 * G1; s > 0; --s) mask &= mask - 1u;
            A = B = __builtin_ffs(mask);
            isT = true;
        }
        if (t.compact && A > B) continue;    // lower triangle: the conjugate of its mirror
        const int kind = (A == 0 && B == 0) ? KIND_Z : (B == 0 ? KIND_X : (A == 0 ? KIND_Y : ((A == B && !isT) ? KIND_P : KIND_S)));
        const int q = A - 1, r = B - 1;
        const CatRec cq = A > 0 ? cats[q] : CatRec{}, cr = B > 0 ? cats[r] : CatRec{};
        const uint32_t live = live_slots(kind, chi, cq.vec, cr.vec, M);
        for (int j = 0; j < 4 * M; ++j) {
            if (!((live >> j) & 1u)) continue;
            const int k = j % M, grp = j / M;
            uint32_t idx;
            if (grp == 0) {          // row molecule raised
                const Conn c = rup(cq, k);
                idx = tgt_index(c, (int)conn_q(c.info), kind == KIND_X ? -1 : conn_remap(c.info, q, r), false);
            } else if (grp == 1) {   // row molecule lowered
                const Conn c = rdn(cq, k);
                const int qn = (int)conn_q(c.info);
                idx = kind == KIND_P ? tgt_index(c, qn, qn, true)
                                     : tgt_index(c, qn, kind == KIND_X ? -1 : conn_remap(c.info, q, r), false);
            } else {                 // column molecule raised (grp 2) or lowered (grp 3)
                const Conn c = grp == 2 ? rup(cr, k) : rdn(cr, k);
                const int ra = kind == KIND_Y ? -1 : conn_remap(c.info, r, q), cb = (int)conn_q(c.info);
                idx = t.trcol ? tgt_index(c, cb, ra, false) : tgt_index(c, ra, cb, false);
            }
            out->push_back(idx);
        }
    }
}

// Decode records of the variables of one tile, in variable order (VarRec);
// for compact tiles only the entries with row <= column and the T_q, each
// with its tile-relative variable in *loc_out.
static int var_records(const HostTables &t, const TileRec &r, std::vector<VarRec> *out,
                       std::vector<uint16_t> *loc_out) {
    const int M = t.m;
    uint32_t goff = 0;
    for (uint32_t pi = 0; pi < r.np; ++pi) {
        const PatHdr &H = t.hdr[r.p0 + pi];
        const int G = H.G, G1 = G + 1;
        const bool chi = H.tier < t.L;
        const CatRec *cats = t.cat.data() + H.cat_base;
        for (uint32_t loc = 0; loc < H.size; ++loc) {
            int A, B;
            bool isT = false;
            if (loc < (uint32_t)(G1 * G1)) {
                A = (int)loc / G1;
                B = (int)loc - A * G1;
            } else {
                uint32_t mask = H.tmask;
                for (int s = (int)loc - G1 * G1; s > 0; --s) mask &= mask - 1u;
                A = B = __builtin_ffs(mask);
                isT = true;
            }
            if (t.compact && A > B) continue;
            const int kind = (A == 0 && B == 0) ? KIND_Z : (B == 0 ? KIND_X : (A == 0 ? KIND_Y : ((A == B && !isT) ? KIND_P : KIND_S)));
            const CatRec cq = A > 0 ? cats[A - 1] : CatRec{}, cr = B > 0 ? cats[B - 1] : CatRec{};
            const uint32_t live = live_slots(kind, chi, cq.vec, cr.vec, M);
            if (goff > VREC_MAX_GOFF) return HEOM_E_UNSUPPORTED;
            out->push_back(vrec_pack(pi, (uint32_t)A, (uint32_t)B, isT, goff, live));
            if (t.compact) loc_out->push_back((uint16_t)(H.off - r.v0 + loc));
            goff += (uint32_t)__builtin_popcount(live);
        }
    }
    return goff == r.ng ? HEOM_OK : HEOM_E_INVAL;
}

int make_tiles(HostTables *t, int tile_vars, std::string *err) {
    uint32_t maxblk = 0;
    for (auto &h : t->hdr) maxblk = std::max(maxblk, h.size);
    if (tile_vars != 64 && tile_vars != 128 && tile_vars != 256 && tile_vars != 512) {
        *err = "tile_vars must be 64, 128, 256 or 512";
        return HEOM_E_INVAL;
    }
    if ((uint32_t)tile_vars < maxblk) {
        *err = "tile_vars is smaller than the largest pattern block";
        return HEOM_E_INVAL;
    }
    t->tile_vars = tile_vars;
    t->layout_gen += 1;
    t->compact = t->tune.compact != 0;
    t->trcol = t->compact || (t->tune.transposed < 0 ? t->n_var >= TRANSPOSED_MIN_VARS : t->tune.transposed != 0);
    t->tiles.clear();
    const size_t np = t->hdr.size();
    size_t i = 0;
    t->max_np = t->max_nc = t->max_ng = 0;
    t->val_len = t->compact ? 0u : (uint32_t)tile_vars;
    t->gidx.clear();
    t->vrec.clear();
    t->vloc.clear();
    t->vrec.reserve(t->n_var);
    // entries a compact tile covers in a block: row <= column, and the T_q
    auto covered = [](const PatHdr &h) { return (uint32_t)(h.G + 1) * (uint32_t)(h.G + 2) / 2u + (h.size - (uint32_t)(h.G + 1) * (uint32_t)(h.G + 1)); };
    while (i < np) {
        TileRec r{};
        r.p0 = (uint32_t)i;
        r.v0 = t->hdr[i].off;
        uint32_t acc = 0, work = 0;
        if (t->compact) {
            // up to tile_vars covered entries and 2 tile_vars variables (the LDS values)
            while (i < np && work + covered(t->hdr[i]) <= (uint32_t)tile_vars &&
                   acc + t->hdr[i].size <= 2u * (uint32_t)tile_vars && i - r.p0 < VREC_MAX_NP) {
                acc += t->hdr[i].size;
                work += covered(t->hdr[i++]);
            }
        } else {
            while (i < np && acc + t->hdr[i].size <= (uint32_t)tile_vars) acc += t->hdr[i++].size;
            work = acc;
        }
        r.np = (uint32_t)i - r.p0;
        r.nv = work;
        if (t->compact) t->val_len = std::max(t->val_len, acc);
        r.c0 = t->hdr[r.p0].cat_base;
        r.nc = (i < np ? t->hdr[i].cat_base : (uint32_t)t->cat.size()) - r.c0;
        r.g0 = (uint32_t)t->gidx.size();
        for (uint32_t p = r.p0; p < r.p0 + r.np; ++p) expand_gathers(*t, p, &t->gidx);
        if (t->gidx.size() > 0xffffffffull) { *err = "more than 2^32-1 hierarchy gathers"; return HEOM_E_TOO_LARGE; }
        r.ng = (uint32_t)t->gidx.size() - r.g0;
        if (r.np > VREC_MAX_NP || r.ng > VREC_MAX_GOFF + 1u) {
            *err = "a tile has more patterns or hierarchy gathers than its records can address";
            return HEOM_E_UNSUPPORTED;
        }
        // compact tables keep one record slot per variable (v0 + thread)
        if (t->compact) {
            t->vrec.resize(r.v0);
            t->vloc.resize(r.v0);
        }
        if (int rc = var_records(*t, r, &t->vrec, &t->vloc)) { *err = "variable records do not match the gather lists"; return rc; }
        // each tile's list starts on a 16-byte boundary (staged as 16-byte words)
        while (t->gidx.size() % 4) t->gidx.push_back(0u);
        t->max_np = std::max(t->max_np, r.np);
        t->max_nc = std::max(t->max_nc, r.nc);
        t->max_ng = std::max(t->max_ng, r.ng);
        t->tiles.push_back(r);
    }
    if (t->compact) {
        t->vrec.resize(t->n_var);
        t->vloc.resize(t->n_var);
    }
    t->top_tile = (uint32_t)t->tiles.size();
    for (size_t k = 0; k < t->tiles.size(); ++k)
        if (t->hdr[t->tiles[k].p0].tier == t->L) { t->top_tile = (uint32_t)k; break; }
    // LDS per workgroup: values, pattern headers, categories, coefficient
    // tables, category multiplicities (FP64, padded to 16 bytes), then the
    // gather indices and the grouped sums. A workgroup that stages its tile
    // for one stage keeps the sums in the gather list's place (the list is
    // dead by then), so it needs the larger of the two; a launch over tiles
    // with shorter lists can allocate less (the top tier's lists, which have
    // no up moves, are about a third as long). The persistent kernel keeps
    // the lists for every stage: the sums follow the longest list.
    const uint32_t lds_fixed = 16u * t->val_len + 32u * t->max_np + 16u * t->max_nc +
                               16u * (uint32_t)t->m * (uint32_t)(t->L + 1) + 8u * ((t->max_nc + 1u) & ~1u);
    const uint32_t sums = 16u * t->val_len;
    uint32_t ng_low = 0, ng_top = 0;
    for (size_t k = 0; k < t->tiles.size(); ++k) {
        uint32_t &ng = k < t->top_tile ? ng_low : ng_top;
        ng = std::max(ng, t->tiles[k].ng);
    }
    auto list_bytes = [](uint32_t ng) { return 4u * ((ng + 3u) & ~3u); };
    t->lds_bytes = lds_fixed + std::max(list_bytes(t->max_ng), sums);
    t->lds_low = lds_fixed + std::max(list_bytes(ng_low), sums);
    t->lds_top = lds_fixed + std::max(list_bytes(ng_top), sums);
    t->lds_persist = lds_fixed + list_bytes(t->max_ng) + sums;
    // element-level reads of one right-hand side: own values and the
    // distinct gather targets (a transposed copy's positions counted as the
    // vector's); with compact tiles the own values are the covered entries
    {
        std::vector<unsigned char> seen(t->n_var, 0);
        uint32_t own = 0, rd = 0;
        for (const TileRec &r : t->tiles) {
            own += r.nv;
            for (uint32_t th = 0; th < r.nv; ++th) {
                const uint32_t v = r.v0 + (t->compact ? t->vloc[r.v0 + th] : th);
                rd += seen[v] ? 0u : 1u;
                seen[v] = 1;
            }
            for (uint32_t g = 0; g < r.ng; ++g) {
                const uint32_t v = t->gidx[r.g0 + g];
                rd += seen[v] ? 0u : 1u;
                seen[v] = 1;
            }
        }
        t->own_entries = own;
        t->read_entries = rd;
    }
    if (t->lds_persist > 64u * 1024u) {
        *err = "tile needs more than 64 KiB of LDS";
        return HEOM_E_UNSUPPORTED;
    }
    t->uploaded = false;
    pack_image(t);
    return HEOM_OK;
}

int set_params(HostTables *t, const heom_problem *p, std::string *err) {
    int rc = check_params(p, err);
    if (rc) return rc;
    auto key = [](int64_t N, int m, int L, int d) {
        return std::vector<int64_t>{std::min<int64_t>(N, (int64_t)L + d + 2), m, L, d};
    };
    if (key(p->N, p->m, p->L, p->d) != key(t->N, t->m, t->L, t->d)) {
        *err = "structure key (min(N, L+d+2), m, L, d) changed; build new tables";
        return HEOM_E_INVAL;
    }
    copy_numeric(t, p);
    t->uploaded = false;
    pack_image(t);
    return HEOM_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Scalars, bath coefficients and section offsets of the device image.
// `num` supplies the numeric parameters, `st` the structure.
static InstParams make_params(const HostTables &num, const HostTables &st) {
    InstParams ip{};
    const heom_problem &p = num.prob;
    ip.g = p.g;
    ip.delta = p.eps - p.omega_c;
    ip.kappa = p.kappa;
    ip.term = p.terminator;
    ip.npool = (double)(num.N - st.d);
    ip.Nd = (double)num.N;
    ip.inv_sqrtN = 1.0 / std::sqrt((double)num.N);
    double th = 0.5 * std::atan2(2.0 * p.g * std::sqrt((double)num.N), p.omega_c - p.eps);
    ip.cos_th = std::cos(th);
    ip.sin_th = std::sin(th);
    for (int k = 0; k < st.m; ++k) {
        ip.nu[k] = num.nu[k];
        ip.cr[k] = num.c[2 * k];
        ip.ci[k] = num.c[2 * k + 1];
        ip.ccr[k] = num.cc[2 * k];
        ip.cci[k] = num.cc[2 * k + 1];
    }
    ip.m = st.m;
    ip.L = st.L;
    ip.d = st.d;
    ip.n_pat = (int32_t)st.hdr.size();
    ip.n_var = st.n_var;
    ip.n_tiles = (uint32_t)st.tiles.size();
    ip.tile_vars = (uint32_t)st.tile_vars;
    ip.max_np = st.max_np;
    ip.max_nc = st.max_nc;
    ip.max_ng = st.max_ng;
    ip.lds_bytes = st.lds_bytes;
    ip.val_len = st.val_len;
    ip.compact = st.compact ? 1u : 0u;
    ip.tcol = st.trcol ? 1u : 0u;
    size_t o = align256(sizeof(InstParams));
    ip.off_lut = o;   o = align256(o + st.lut.size() * sizeof(double));
    ip.off_hdr = o;   o = align256(o + st.hdr.size() * sizeof(PatHdr));
    ip.off_cat = o;   o = align256(o + st.cat.size() * sizeof(CatRec));
    ip.off_gidx = o;  o = align256(o + st.gidx.size() * sizeof(uint32_t));
    ip.off_tile = o;  o = align256(o + st.tiles.size() * sizeof(TileRec));
    ip.off_vrec = o;  o = align256(o + st.vrec.size() * sizeof(VarRec));
    ip.off_end = o;
    return ip;
}

size_t image_bytes(const HostTables &t) {
    return make_params(t, t).off_end;
}

// Copy a section into the image (an empty section copies nothing: memcpy
// from the null data() of an empty vector would be undefined).
template <class V>
static void put_section(std::vector<unsigned char> *img, uint64_t off, const std::vector<V> &v) {
    if (!v.empty()) std::memcpy(img->data() + off, v.data(), v.size() * sizeof(V));
}

int pack_params(const HostTables &t, const heom_problem *p, std::vector<unsigned char> *out, std::string *err) {
    int rc = check_params(p, err);
    if (rc) return rc;
    auto key = [](int64_t N, int m, int L, int d) {
        return std::vector<int64_t>{std::min<int64_t>(N, (int64_t)L + d + 2), m, L, d};
    };
    if (key(p->N, p->m, p->L, p->d) != key(t.N, t.m, t.L, t.d)) {
        *err = "structure key (min(N, L+d+2), m, L, d) differs from the tables";
        return HEOM_E_INVAL;
    }
    HostTables num;
    num.m = t.m;
    num.L = t.L;
    num.d = t.d;
    copy_numeric(&num, p);
    const InstParams ip = make_params(num, t);
    out->assign(ip.off_hdr, 0);
    std::memcpy(out->data(), &ip, sizeof ip);
    put_section(out, ip.off_lut, num.lut);
    return HEOM_OK;
}

void pack_image(HostTables *t) {
    const InstParams ip = make_params(*t, *t);
    const size_t o = image_bytes(*t);
    t->image.assign(o, 0);
    std::memcpy(t->image.data(), &ip, sizeof ip);
    put_section(&t->image, ip.off_lut, t->lut);
    put_section(&t->image, ip.off_hdr, t->hdr);
    put_section(&t->image, ip.off_cat, t->cat);
    put_section(&t->image, ip.off_gidx, t->gidx);
    put_section(&t->image, ip.off_tile, t->tiles);
    put_section(&t->image, ip.off_vrec, t->vrec);
}

}  // namespace heom
