// Host-side check of the workgroup tiles built by the table builder, for
// plain, transposed-target and compact tiles: every tile's ranges, decode
// records and gather indices stay in bounds; with compact tiles every
// variable of a tile is either a covered entry (row <= column, or a T_q) or
// the mirror of exactly one covered entry, found from its decode record and
// its block's header alone; with transposed targets a column
// move names the mirrored position of the entry a plain table names; every
// tile's metadata fits the LDS its launch allocates.
// Prints "ok" and exits 0, or names the first failure and exits 1.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>
#include "heom_internal.h"
using namespace heom;

static int fail(const char *what, long long a = 0, long long b = 0) {
    std::printf("FAIL %s %lld %lld\n", what, a, b);
    return 1;
}

static bool build_tables(HostTables *t, int64_t N, int m, int L, int d, int tv, int transposed, int compact) {
    heom_problem p{};
    static double c[16], nu[8];
    for (int k = 0; k < 8; ++k) { c[2 * k] = 0.01 * (k + 1); c[2 * k + 1] = -0.02; nu[k] = 0.1 * (k + 1); }
    p.N = N; p.m = m; p.L = L; p.d = d; p.c = c; p.nu = nu; p.g = 0.1;
    std::string err;
    if (build(&p, t, &err)) return false;
    t->tune.transposed = transposed;
    t->tune.compact = compact;
    return make_tiles(t, tv, &err) == HEOM_OK;
}

// (pattern, A, B, isT) of every variable, from the headers (layout of Sec. V.C.1 as the tables use it)
struct Entry { uint32_t p, A, B; bool T; };
static std::vector<Entry> entries(const HostTables &t) {
    std::vector<Entry> e(t.n_var);
    for (uint32_t q = 0; q < t.hdr.size(); ++q) {
        const PatHdr &H = t.hdr[q];
        const uint32_t G1 = H.G + 1u;
        uint32_t mask = H.tmask;
        for (uint32_t loc = 0; loc < H.size; ++loc) {
            if (loc < G1 * G1) e[H.off + loc] = {q, loc / G1, loc % G1, false};
            else { const uint32_t c = (uint32_t)__builtin_ctz(mask) + 1u; mask &= mask - 1u; e[H.off + loc] = {q, c, c, true}; }
        }
    }
    return e;
}

static int check(int64_t N, int m, int L, int d, int tv) {
    HostTables plain, trans, comp;
    if (!build_tables(&plain, N, m, L, d, tv, 0, 0)) return 0;   // tile too small for this structure
    if (!build_tables(&trans, N, m, L, d, tv, 1, 0) || !build_tables(&comp, N, m, L, d, tv, 0, 1))
        return fail("build", N, tv);
    const std::vector<Entry> E = entries(plain);
    auto mirror = [&](uint32_t v) -> uint32_t {
        const Entry &e = E[v];
        if (e.T) return v;
        const PatHdr &H = plain.hdr[e.p];
        return H.off + e.B * (H.G + 1u) + e.A;
    };
    // transposed targets: same lists, column moves (slots 2M..4M-1) at the mirrored position
    if (plain.gidx.size() != trans.gidx.size()) return fail("transposed list length");
    for (const TileRec &R : plain.tiles)
        for (uint32_t th = 0; th < R.nv; ++th) {
            const VarRec vr = plain.vrec[R.v0 + th];
            uint32_t live = vr.y, j2 = 0;
            for (int j = 0; live; ++j, live >>= 1) {
                if (!(live & 1u)) continue;
                const uint32_t g = R.g0 + (vr.x >> 18) + j2++;
                const uint32_t want = j >= 2 * m ? mirror(plain.gidx[g]) : plain.gidx[g];
                if (trans.gidx[g] != want) return fail("transposed target", R.v0 + th, j);
                if (plain.gidx[g] >= plain.n_var) return fail("gather index", g, plain.gidx[g]);
            }
        }
    // LDS: values, headers, categories, coefficient tables and multiplicities,
    // then the gather list, whose place the grouped sums (16 bytes per value)
    // take once the list has been read; a tile's list and the sums must fit
    // what its launch allocates (lower tiers / top tier), and the persistent
    // kernel, which keeps the lists, holds both
    for (const HostTables *T : {&plain, &trans, &comp}) {
        const uint32_t fixed = 16u * T->val_len + 32u * T->max_np + 16u * T->max_nc +
                               16u * (uint32_t)T->m * (uint32_t)(T->L + 1) + 8u * ((T->max_nc + 1u) & ~1u);
        const uint32_t sums = 16u * T->val_len;
        auto list = [](uint32_t ng) { return 4u * ((ng + 3u) & ~3u); };
        if (T->lds_low > T->lds_bytes || T->lds_top > T->lds_bytes) return fail("launch LDS", T->lds_low, T->lds_top);
        if (T->lds_persist != fixed + list(T->max_ng) + sums) return fail("persistent LDS", T->lds_persist, T->max_ng);
        for (size_t k = 0; k < T->tiles.size(); ++k) {
            const TileRec &R = T->tiles[k];
            const uint32_t alloc = k < T->top_tile ? T->lds_low : T->lds_top;
            if (R.np > T->max_np || R.nc > T->max_nc || fixed + std::max(list(R.ng), sums) > alloc ||
                fixed + std::max(list(R.ng), sums) > T->lds_bytes)
                return fail("tile LDS", (long long)k, R.ng);
        }
    }
    // compact tiles: coverage, bounds
    std::vector<int> cover(comp.n_var, 0);
    for (const TileRec &R : comp.tiles) {
        if (R.nv > (uint32_t)tv || R.np == 0 || R.np > VREC_MAX_NP) return fail("compact tile size", R.nv, R.np);
        uint32_t full = 0;
        for (uint32_t q = R.p0; q < R.p0 + R.np; ++q) full += comp.hdr[q].size;
        if (full > comp.val_len || comp.val_len > 2u * (uint32_t)tv) return fail("compact LDS values", full, comp.val_len);
        for (uint32_t th = 0; th < R.nv; ++th) {
            const VarRec vr = comp.vrec[R.v0 + th];
            const uint32_t pi = vr.x & 127u, A = (vr.x >> 7) & 31u, B = (vr.x >> 12) & 31u;
            const bool isT = (vr.x >> 17) & 1u;
            if (pi >= R.np) return fail("pattern index", R.v0 + th, pi);
            const uint32_t v = R.v0 + comp.vloc[R.v0 + th];
            const Entry &e = E[v];
            if (e.p != R.p0 + pi || e.A != A || e.B != B || e.T != isT) return fail("decode record", v, th);
            if (A > B) return fail("lower-triangle thread", v, th);
            // the kernels find the entry from the record and the block header alone
            const PatHdr &H = comp.hdr[R.p0 + pi];
            const uint32_t G1 = H.G + 1u;
            const uint32_t derived = H.off + (isT ? G1 * G1 + (uint32_t)__builtin_popcount(H.tmask & ((1u << (A - 1u)) - 1u))
                                                  : A * G1 + B);
            if (derived != v) return fail("entry from record and header", v, derived);
            cover[v]++;
            if (A != B && !isT) cover[mirror(v)]++;
            const uint32_t goff = vr.x >> 18, nl = (uint32_t)__builtin_popcount(vr.y);
            if (goff + nl > R.ng) return fail("gather list range", v, goff + nl);
            for (uint32_t j = 0; j < nl; ++j)
                if (comp.gidx[R.g0 + goff + j] >= comp.n_var) return fail("compact gather index", v, j);
        }
    }
    for (uint32_t v = 0; v < comp.n_var; ++v)
        if (cover[v] != 1) return fail("coverage", v, cover[v]);
    return 0;
}

int main(int argc, char **argv) {
    const int cases[][4] = {{5, 2, 3, 1}, {7, 3, 3, 0}, {4, 1, 2, 2}, {64, 2, 6, 1}, {6, 5, 2, 0}, {3, 2, 4, 1},
                            {2, 1, 3, 0}, {12, 4, 3, 0}, {40, 3, 4, 1}, {100, 3, 6, 0}, {9, 8, 2, 0}};
    for (auto &c : cases)
        for (int tv : {64, 128, 256, 512})
            if (check(c[0], c[1], c[2], c[3], tv)) return 1;
    // seeded sweep over small structures: argv[1] = seed, argv[2] = count
    if (argc > 2) {
        uint64_t x = std::strtoull(argv[1], nullptr, 10) * 0x9E3779B97F4A7C15ull + 1;
        auto next = [&](int lo, int hi) {   // xorshift64*, uniform in [lo, hi]
            x ^= x >> 12; x ^= x << 25; x ^= x >> 27;
            return lo + (int)(((x * 0x2545F4914F6CDD1Dull) >> 33) % (uint64_t)(hi - lo + 1));
        };
        const int n = std::atoi(argv[2]);
        for (int i = 0; i < n; ++i) {
            const int N = next(1, 30), m = next(1, 4), L = next(0, m >= 3 ? 5 : 7), d = next(0, N < 3 ? N : 3);
            const int tv = 64 << next(0, 3);
            if (check(N, m, L, d, tv)) {
                std::printf("case N=%d m=%d L=%d d=%d tile=%d\n", N, m, L, d, tv);
                return 1;
            }
        }
    }
    std::printf("ok\n");
    return 0;
}
