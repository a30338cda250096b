// gfx950 kernels and the C ABI of libheom (include/heom.h).
//
// The right-hand side is evaluated in pull form, one thread per unique
// variable (Sec. V.C): a workgroup owns a tile of whole pattern blocks,
// stages the tile's input values in LDS (the grouped multiplicity sums of
// Eqs. grouped-row-sum / grouped-column-sum and the Hamiltonian terms read
// only the variable's own block), and gathers hierarchy neighbours from
// tiers |Lambda| +- 1 through the connection records (Eqs. uvar-up,
// uvar-down). Each launch also applies one fused RK4 combination, so a time
// step is four launches. No atomics: every output element has one writer.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>

#include "heom_internal.h"

using namespace heom;

struct heom_tables {
    HostTables t;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return fail(HEOM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------ device view
struct Dev {
    const InstParams *ip;
    const double *lut;
    const PatHdr *hdr;
    const CatRec *cat;
    const Conn *conn;
    const uint32_t *tiles;
};

Dev dev_view(const HostTables &t) {
    const unsigned char *b = static_cast<const unsigned char *>(t.dev);
    const InstParams *ip = reinterpret_cast<const InstParams *>(t.image.data());
    Dev D;
    D.ip = reinterpret_cast<const InstParams *>(b);
    D.lut = reinterpret_cast<const double *>(b + ip->off_lut);
    D.hdr = reinterpret_cast<const PatHdr *>(b + ip->off_hdr);
    D.cat = reinterpret_cast<const CatRec *>(b + ip->off_cat);
    D.conn = reinterpret_cast<const Conn *>(b + ip->off_conn);
    D.tiles = reinterpret_cast<const uint32_t *>(b + ip->off_tile);
    return D;
}

// ------------------------------------------------------------ complex ops
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// acc += w * v
__device__ __forceinline__ void cfma(double2 &acc, double2 w, double2 v) {
    acc.x += w.x * v.x - w.y * v.y;
    acc.y += w.x * v.y + w.y * v.x;
}

// ------------------------------------------------------------ input views
struct InF64 {
    const double2 *a;
    __device__ __forceinline__ double2 load(uint32_t j) const { return a[j]; }
};
struct InF32 {
    const float2 *b;
    __device__ __forceinline__ double2 load(uint32_t j) const {
        float2 v = b[j];
        return make_double2((double)v.x, (double)v.y);
    }
};
struct InSum {  // y + u with y complex FP64 and u complex FP32
    const double2 *a;
    const float2 *b;
    __device__ __forceinline__ double2 load(uint32_t j) const {
        double2 y = a[j];
        float2 u = b[j];
        return make_double2(y.x + (double)u.x, y.y + (double)u.y);
    }
};

__device__ __forceinline__ void store(double2 *p, double2 v) { *p = v; }
__device__ __forceinline__ void store(float2 *p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }

// blockIdx -> tile such that each of the 8 XCDs (workgroups are dealt to
// XCDs round robin) processes one contiguous run of tiles.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n) {
    const uint32_t X = 8;
    uint32_t q = n / X, rem = n % X, x = b % X, idx = b / X;
    return x < rem ? x * (q + 1) + idx : rem * (q + 1) + (x - rem) * q + idx;
}

// Index of the target variable <a'|R'|b'> for a connection record; a', b'
// are target categories (-1 = cavity), `same` = same molecule.
__device__ __forceinline__ uint32_t tgt_index(Conn cr, int a, int b, bool same) {
    const uint32_t G1 = conn_G(cr.info) + 1;
    if (a < 0 && b < 0) return cr.off;
    if (b < 0) return cr.off + (uint32_t)(a + 1) * G1;
    if (a < 0) return cr.off + (uint32_t)(b + 1);
    if (same) return cr.off + (uint32_t)(a + 1) * (G1 + 1);
    if (a == b) return cr.off + G1 * G1 + __popc(conn_tmask(cr.info) & ((1u << a) - 1u));
    return cr.off + (uint32_t)(a + 1) * G1 + (uint32_t)(b + 1);
}

__device__ __forceinline__ uint32_t vbyte(uint64_t v, int k) { return (uint32_t)(v >> (8 * k)) & 0xffu; }

// first record of category c for a move in channel k (up or down)
__device__ __forceinline__ uint32_t rec_up(const PatHdr &H, const CatRec &c, int k) {
    return H.conn_base + c.conn_off + k;
}
__device__ __forceinline__ uint32_t rec_dn(const PatHdr &H, const CatRec &c, int k, bool chi, int m) {
    uint32_t r = H.conn_base + c.conn_off + (chi ? m : 0);
    for (int j = 0; j < k; ++j) r += vbyte(c.vec, j) != 0;
    return r;
}

// Observables of the tier-0 block v (Sec. V.D, any d).
__device__ void tier0_observables(const InstParams &P, const PatHdr &H, const CatRec *cats,
                                  const double2 *v, double *out) {
    const int G = H.G, G1 = G + 1;
    auto M = [&](int q) {
        const CatRec c = cats[H.cat_base + q];
        return (c.flags & CAT_ZERO) ? (P.npool - (double)H.r) : (double)c.mult;
    };
    const double2 Z = v[0];
    double2 pexc = make_double2(0, 0), tot, bc = make_double2(0, 0), cb = make_double2(0, 0);
    for (int q = 0; q < G; ++q) {
        const double Mq = M(q);
        pexc = cadd(pexc, cscale(Mq, v[(q + 1) * G1 + q + 1]));
        bc = cadd(bc, cscale(Mq, v[(q + 1) * G1]));
        cb = cadd(cb, cscale(Mq, v[q + 1]));
    }
    tot = pexc;
    for (int q = 0; q < G; ++q) {
        const double Mq = M(q);
        if ((H.tmask >> q) & 1u)
            tot = cadd(tot, cscale(Mq * (Mq - 1.0), v[G1 * G1 + __popc(H.tmask & ((1u << q) - 1u))]));
        for (int r = 0; r < G; ++r)
            if (r != q) tot = cadd(tot, cscale(Mq * M(r), v[(q + 1) * G1 + r + 1]));
    }
    const double pb = tot.x / P.Nd;
    const double x = (bc.x + cb.x) * P.inv_sqrtN;
    const double s = P.sin_th, c = P.cos_th;
    // molecule 1: distinguished category 0 if d >= 1, else the zero category
    const double site1 = v[1 * G1 + 1].x;  // category 0 in both cases (d = 0: only category)
    out[0] = Z.x + pexc.x;
    out[1] = Z.x;
    out[2] = pexc.x;
    out[3] = pb;
    out[4] = pexc.x - pb;
    out[5] = Z.x * c * c + pb * s * s + s * c * x;
    out[6] = Z.x * s * s + pb * c * c - s * c * x;
    out[7] = site1;
    out[8] = pexc.x - site1;
    out[9] = Z.y + pexc.y;
}

constexpr int MAX_TILE = 512;

// One fused stage: out[i] = base(i) + alpha * ((M in)[i] + extra_scale * extra[i])
// over the variables of one tile per workgroup.
template <class IN, class OutT, bool BASE_Y, bool BASE_IS_IN, bool EXTRA>
__global__ __launch_bounds__(MAX_TILE) void stage_kernel(Dev D, IN in, const double2 *ybase,
                                                       const float2 *extra, double extra_scale,
                                                       OutT *out, double alpha, double *obs, int xcd) {
    __shared__ double2 sval[MAX_TILE];
    __shared__ uint32_t soff[MAX_TILE];
    const InstParams &P = *D.ip;
    const uint32_t tile = xcd ? xcd_tile(blockIdx.x, P.n_tiles) : blockIdx.x;
    const uint32_t p0 = D.tiles[tile], p1 = D.tiles[tile + 1];
    const uint32_t v0 = D.hdr[p0].off;
    const uint32_t v1 = (p1 < (uint32_t)P.n_pat) ? D.hdr[p1].off : P.n_var;
    const uint32_t nloc = v1 - v0, npl = p1 - p0;
    for (uint32_t i = threadIdx.x; i < nloc; i += blockDim.x) sval[i] = in.load(v0 + i);
    for (uint32_t j = threadIdx.x; j < npl; j += blockDim.x) soff[j] = D.hdr[p0 + j].off - v0;
    __syncthreads();

    const uint32_t t = threadIdx.x;
    double2 res = make_double2(0.0, 0.0);
    if (t < nloc) {
        uint32_t lo = 0, hi = npl;  // soff[lo] <= t < start of block hi
        while (hi - lo > 1) {
            uint32_t mid = (lo + hi) >> 1;
            if (soff[mid] <= t) lo = mid; else hi = mid;
        }
        const PatHdr H = D.hdr[p0 + lo];
        const uint32_t base = soff[lo];
        const uint32_t loc = t - base;
        const int G = H.G, G1 = G + 1, nm = G1 * G1;
        int A, B;
        bool isT;
        if (loc < (uint32_t)nm) {
            A = (int)loc / G1;
            B = (int)loc - A * G1;
            isT = false;
        } else {
            uint32_t mask = H.tmask;
            for (int s = (int)loc - nm; s > 0; --s) mask &= mask - 1u;
            A = B = __ffs(mask);  // category index + 1
            isT = true;
        }
        const int m = P.m, L = P.L;
        const double *up = D.lut;
        const double *dn = D.lut + m * (L + 1);
        const CatRec *cats = D.cat + H.cat_base;
        const bool chi = H.tier < L;
        auto mult = [&](int q) -> double {
            const CatRec c = cats[q];
            return (c.flags & CAT_ZERO) ? (P.npool - (double)H.r) : (double)c.mult;
        };
        auto sv = [&](int a, int b) { return sval[base + a * G1 + b]; };
        auto svT = [&](int q) { return sval[base + nm + __popc(H.tmask & ((1u << q) - 1u))]; };

        double gam = 0.0;
        for (int k = 0; k < m; ++k) gam += P.nu[k] * (double)vbyte(H.cnt, k);
        const double g = P.g;
        const double2 own = sval[t];
        double2 acc = make_double2(0.0, 0.0);
        double2 hsum;  // Hamiltonian bracket, multiplied by -i g below

        if (A == 0 && B == 0) {
            // Z: -i g sum_q M_q (X_q - Y_q) - (Gamma + kappa) Z   (Eq. HZ)
            hsum = make_double2(0, 0);
            for (int q = 0; q < G; ++q) hsum = cadd(hsum, cscale(mult(q), csub(sv(q + 1, 0), sv(0, q + 1))));
            acc = cscale(-(gam + P.kappa), own);
        } else if (B == 0) {
            // X_q: -i(delta)X - i g (Z - R_q) - (Gamma + kappa/2 + Delta) X   (Eq. HX)
            const int q = A - 1;
            double2 R = sv(A, A);
            if ((H.tmask >> q) & 1u) R = cadd(R, cscale(mult(q) - 1.0, svT(q)));
            for (int r = 0; r < G; ++r)
                if (r != q) R = cadd(R, cscale(mult(r), sv(A, r + 1)));
            hsum = csub(sv(0, 0), R);
            const double re = -(gam + 0.5 * P.kappa + P.term);
            acc = make_double2(re * own.x + P.delta * own.y, re * own.y - P.delta * own.x);
            const CatRec c = cats[q];
            for (int k = 0; k < m; ++k) {
                const uint32_t n = vbyte(c.vec, k);
                if (chi) {
                    const Conn cr = D.conn[rec_up(H, c, k)];
                    const double w = up[k * (L + 1) + n];
                    cfma(acc, make_double2(0.0, -w), in.load(tgt_index(cr, (int)conn_q(cr.info), -1, false)));
                }
                if (n) {
                    const Conn cr = D.conn[rec_dn(H, c, k, chi, m)];
                    const double w = dn[k * (L + 1) + n];
                    // -i w c_k
                    cfma(acc, make_double2(w * P.ci[k], -w * P.cr[k]), in.load(tgt_index(cr, (int)conn_q(cr.info), -1, false)));
                }
            }
        } else if (A == 0) {
            // Y_q: +i(delta)Y - i g (C_q - Z) - (Gamma + kappa/2 + Delta) Y
            const int q = B - 1;
            double2 C = sv(B, B);
            if ((H.tmask >> q) & 1u) C = cadd(C, cscale(mult(q) - 1.0, svT(q)));
            for (int r = 0; r < G; ++r)
                if (r != q) C = cadd(C, cscale(mult(r), sv(r + 1, B)));
            hsum = csub(C, sv(0, 0));
            const double re = -(gam + 0.5 * P.kappa + P.term);
            acc = make_double2(re * own.x - P.delta * own.y, re * own.y + P.delta * own.x);
            const CatRec c = cats[q];
            for (int k = 0; k < m; ++k) {
                const uint32_t n = vbyte(c.vec, k);
                if (chi) {
                    const Conn cr = D.conn[rec_up(H, c, k)];
                    const double w = up[k * (L + 1) + n];
                    cfma(acc, make_double2(0.0, w), in.load(tgt_index(cr, -1, (int)conn_q(cr.info), false)));
                }
                if (n) {
                    const Conn cr = D.conn[rec_dn(H, c, k, chi, m)];
                    const double w = dn[k * (L + 1) + n];
                    // +i w cc_k
                    cfma(acc, make_double2(-w * P.cci[k], w * P.ccr[k]), in.load(tgt_index(cr, -1, (int)conn_q(cr.info), false)));
                }
            }
        } else if (A == B && !isT) {
            // P_q: -i g (Y_q - X_q) - Gamma P; down only, coefficient -i w (c_k - cc_k)
            const int q = A - 1;
            hsum = csub(sv(0, A), sv(A, 0));
            acc = cscale(-gam, own);
            const CatRec c = cats[q];
            for (int k = 0; k < m; ++k) {
                const uint32_t n = vbyte(c.vec, k);
                if (!n) continue;
                const Conn cr = D.conn[rec_dn(H, c, k, chi, m)];
                const double w = dn[k * (L + 1) + n];
                const double dr = P.cr[k] - P.ccr[k], di = P.ci[k] - P.cci[k];
                const int qn = (int)conn_q(cr.info);
                cfma(acc, make_double2(w * di, -w * dr), in.load(tgt_index(cr, qn, qn, true)));
            }
        } else {
            // S_{q,r} (q = A-1, r = B-1) or T_q (q = r): -i g (Y_r - X_q) - (Gamma + 2 Delta) V
            const int q = A - 1, r = B - 1;
            hsum = csub(sv(0, B), sv(A, 0));
            acc = cscale(-(gam + 2.0 * P.term), own);
            // row term: the row molecule (category q) moves
            {
                const CatRec c = cats[q];
                for (int k = 0; k < m; ++k) {
                    const uint32_t n = vbyte(c.vec, k);
                    if (chi) {
                        const Conn cr = D.conn[rec_up(H, c, k)];
                        const double w = up[k * (L + 1) + n];
                        const int a2 = (int)conn_q(cr.info), b2 = conn_remap(cr.info, q, r);
                        cfma(acc, make_double2(0.0, -w), in.load(tgt_index(cr, a2, b2, false)));
                    }
                    if (n) {
                        const Conn cr = D.conn[rec_dn(H, c, k, chi, m)];
                        const double w = dn[k * (L + 1) + n];
                        const int a2 = (int)conn_q(cr.info), b2 = conn_remap(cr.info, q, r);
                        cfma(acc, make_double2(w * P.ci[k], -w * P.cr[k]), in.load(tgt_index(cr, a2, b2, false)));
                    }
                }
            }
            // column term: the column molecule (category r) moves
            {
                const CatRec c = cats[r];
                for (int k = 0; k < m; ++k) {
                    const uint32_t n = vbyte(c.vec, k);
                    if (chi) {
                        const Conn cr = D.conn[rec_up(H, c, k)];
                        const double w = up[k * (L + 1) + n];
                        const int b2 = (int)conn_q(cr.info), a2 = conn_remap(cr.info, r, q);
                        cfma(acc, make_double2(0.0, w), in.load(tgt_index(cr, a2, b2, false)));
                    }
                    if (n) {
                        const Conn cr = D.conn[rec_dn(H, c, k, chi, m)];
                        const double w = dn[k * (L + 1) + n];
                        const int b2 = (int)conn_q(cr.info), a2 = conn_remap(cr.info, r, q);
                        cfma(acc, make_double2(-w * P.cci[k], w * P.ccr[k]), in.load(tgt_index(cr, a2, b2, false)));
                    }
                }
            }
        }
        // -i g * hsum
        acc.x += g * hsum.y;
        acc.y -= g * hsum.x;
        if (EXTRA) {
            const float2 e = extra[v0 + t];
            acc.x += extra_scale * (double)e.x;
            acc.y += extra_scale * (double)e.y;
        }
        res = cscale(alpha, acc);
        if (BASE_Y) res = cadd(res, BASE_IS_IN ? own : ybase[v0 + t]);
        store(out + v0 + t, res);
    }
    if (obs != nullptr && tile == 0) {
        // the empty pattern is the first block of tile 0: evaluate the
        // observables of the freshly written tier-0 block
        __syncthreads();
        const uint32_t n0 = D.hdr[0].size;
        if (t < n0) sval[t] = res;
        __syncthreads();
        if (t == 0) tier0_observables(P, D.hdr[0], D.cat, sval, obs);
    }
}

__global__ void observables_kernel(Dev D, const double2 *y, double *obs) {
    __shared__ double2 v[MAX_TILE];
    const uint32_t n0 = D.hdr[0].size;
    for (uint32_t i = threadIdx.x; i < n0; i += blockDim.x) v[i] = y[i];
    __syncthreads();
    if (threadIdx.x == 0) tier0_observables(*D.ip, D.hdr[0], D.cat, v, obs);
}

__global__ void zero_kernel(double2 *y, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        y[i] = make_double2(0.0, 0.0);
}

__global__ void copy_kernel(const double2 *src, double2 *dst, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        dst[i] = src[i];
}

int g_xcd_map = 1;

template <class IN, class OutT, bool BASE_Y, bool BASE_IS_IN, bool EXTRA>
int launch_stage(const HostTables &t, hipStream_t s, IN in, const double2 *ybase, const float2 *extra,
                 double extra_scale, OutT *out, double alpha, double *obs) {
    const uint32_t ntiles = (uint32_t)(t.tiles.size() - 1);
    hipLaunchKernelGGL((stage_kernel<IN, OutT, BASE_Y, BASE_IS_IN, EXTRA>), dim3(ntiles), dim3(t.tile_vars), 0, s,
                       dev_view(t), in, ybase, extra, extra_scale, out, alpha, obs, g_xcd_map);
    HIP_TRY(hipGetLastError());
    return HEOM_OK;
}

int check_ready(const heom_tables *h) {
    if (!h) return fail(HEOM_E_INVAL, "tables handle is NULL");
    if (!h->t.uploaded) return fail(HEOM_E_STATE, "tables not uploaded (call heom_upload)");
    return HEOM_OK;
}

int check_dev(const void *p, const char *name) {
    if (!p) return fail(HEOM_E_INVAL, std::string(name) + " is NULL");
    if (reinterpret_cast<uintptr_t>(p) % 16) return fail(HEOM_E_INVAL, std::string(name) + " is not 16-byte aligned");
    return HEOM_OK;
}

}  // namespace

extern "C" {

int heom_build_tables(const heom_problem *prob, heom_tables **out) {
    if (!out) return fail(HEOM_E_INVAL, "out is NULL");
    *out = nullptr;
    heom_tables *h = new (std::nothrow) heom_tables;
    if (!h) return fail(HEOM_E_NOMEM, "host allocation failed");
    std::string err;
    int rc;
    try {
        rc = build(prob, &h->t, &err);
    } catch (const std::bad_alloc &) {
        rc = HEOM_E_NOMEM;
        err = "host allocation failed";
    } catch (const std::exception &e) {
        rc = HEOM_E_INVAL;
        err = e.what();
    }
    if (rc) {
        delete h;
        return fail(rc, err);
    }
    *out = h;
    g_err.clear();
    return HEOM_OK;
}

int heom_set_params(heom_tables *h, const heom_problem *prob) {
    if (!h) return fail(HEOM_E_INVAL, "tables handle is NULL");
    std::string err;
    int rc;
    try {
        rc = set_params(&h->t, prob, &err);
    } catch (const std::exception &e) {
        rc = HEOM_E_NOMEM;
        err = e.what();
    }
    return rc ? fail(rc, err) : HEOM_OK;
}

int heom_table_info(const heom_tables *h, heom_sizes *out) {
    if (!h || !out) return fail(HEOM_E_INVAL, "NULL argument");
    const HostTables &t = h->t;
    out->n_patterns = (int64_t)t.hdr.size();
    out->n_var = t.n_var;
    out->n_conn = (int64_t)t.conn.size();
    out->n_tiles = (int64_t)t.tiles.size() - 1;
    out->n_categories = (int64_t)t.cat.size();
    out->table_bytes = (int64_t)t.image.size();
    out->work_bytes_fp64 = (int64_t)t.n_var * 32;
    out->work_bytes_fp32 = (int64_t)t.n_var * 32;
    out->tier0_size = (int64_t)tier0_size(t);
    out->max_G = t.max_G;
    out->tile_vars = t.tile_vars;
    out->hier_gathers = t.hier_gathers;
    return HEOM_OK;
}

int heom_upload(heom_tables *h, void *dev, size_t bytes, void *stream) {
    if (!h) return fail(HEOM_E_INVAL, "tables handle is NULL");
    if (!dev) return fail(HEOM_E_INVAL, "device pointer is NULL");
    if (reinterpret_cast<uintptr_t>(dev) % 256) return fail(HEOM_E_INVAL, "device image must be 256-byte aligned");
    if (bytes < h->t.image.size()) return fail(HEOM_E_TOO_LARGE, "device buffer smaller than table_bytes");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(dev, h->t.image.data(), h->t.image.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    h->t.dev = dev;
    h->t.dev_bytes = bytes;
    h->t.uploaded = true;
    return HEOM_OK;
}

int heom_tier0_pure(const heom_tables *h, const double a_c[2], const double *a_dist, const double a_pool[2],
                    double *out) {
    if (!h || !a_c || !a_pool || !out) return fail(HEOM_E_INVAL, "NULL argument");
    const HostTables &t = h->t;
    if (t.d > 0 && !a_dist) return fail(HEOM_E_INVAL, "a_dist is required when d > 0");
    const PatHdr &H = t.hdr[0];
    const int G = H.G, G1 = G + 1;
    auto amp = [&](int idx, double *re, double *im) {  // idx 0 = cavity, q+1 = category q
        if (idx == 0) { *re = a_c[0]; *im = a_c[1]; return; }
        const CatRec &c = t.cat[H.cat_base + idx - 1];
        if (c.flags & CAT_DIST) {
            int j = idx - 1;
            *re = a_dist[2 * j]; *im = a_dist[2 * j + 1];
        } else {
            *re = a_pool[0]; *im = a_pool[1];
        }
    };
    auto put = [&](size_t pos, int A, int B) {
        double ar, ai, br, bi;
        amp(A, &ar, &ai);
        amp(B, &br, &bi);
        out[2 * pos] = ar * br + ai * bi;       // a * conj(b)
        out[2 * pos + 1] = ai * br - ar * bi;
    };
    for (int A = 0; A < G1; ++A)
        for (int B = 0; B < G1; ++B) put((size_t)A * G1 + B, A, B);
    size_t pos = (size_t)G1 * G1;
    for (int q = 0; q < G; ++q)
        if ((H.tmask >> q) & 1u) put(pos++, q + 1, q + 1);
    return HEOM_OK;
}

int heom_init_state(const heom_tables *h, const double *tier0, void *y_dev, void *stream) {
    if (int rc = check_ready(h)) return rc;
    if (!tier0) return fail(HEOM_E_INVAL, "tier0 is NULL");
    if (int rc = check_dev(y_dev, "y_dev")) return rc;
    const HostTables &t = h->t;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(zero_kernel, dim3(1024), dim3(256), 0, s, static_cast<double2 *>(y_dev), t.n_var);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(y_dev, tier0, tier0_size(t) * 16, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return HEOM_OK;
}

int heom_rhs(const heom_tables *h, const void *y_dev, void *dy_dev, void *stream) {
    if (int rc = check_ready(h)) return rc;
    if (int rc = check_dev(y_dev, "y_dev")) return rc;
    if (int rc = check_dev(dy_dev, "dy_dev")) return rc;
    if (y_dev == dy_dev) return fail(HEOM_E_INVAL, "y_dev and dy_dev must differ");
    hipStream_t s = static_cast<hipStream_t>(stream);
    return launch_stage<InF64, double2, false, false, false>(h->t, s, InF64{static_cast<const double2 *>(y_dev)},
                                                             nullptr, nullptr, 0.0, static_cast<double2 *>(dy_dev),
                                                             1.0, nullptr);
}

int heom_observables(const heom_tables *h, const void *y_dev, double *obs_dev, void *stream) {
    if (int rc = check_ready(h)) return rc;
    if (int rc = check_dev(y_dev, "y_dev")) return rc;
    if (!obs_dev) return fail(HEOM_E_INVAL, "obs_dev is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(observables_kernel, dim3(1), dim3(64), 0, s, dev_view(h->t),
                       static_cast<const double2 *>(y_dev), obs_dev);
    HIP_TRY(hipGetLastError());
    return HEOM_OK;
}

int heom_propagate(const heom_tables *h, void *y_dev, void *work_dev, size_t work_bytes, double dt, int64_t nsteps,
                   int64_t obs_every, double *obs_dev, int precision, void *stream) {
    if (int rc = check_ready(h)) return rc;
    if (int rc = check_dev(y_dev, "y_dev")) return rc;
    if (int rc = check_dev(work_dev, "work_dev")) return rc;
    if (!(std::isfinite(dt)) || nsteps < 0 || obs_every < 0) return fail(HEOM_E_INVAL, "bad dt, nsteps or obs_every");
    if (obs_every > 0 && !obs_dev) return fail(HEOM_E_INVAL, "obs_dev is NULL");
    if (precision != HEOM_FP64 && precision != HEOM_FP32) return fail(HEOM_E_INVAL, "unknown precision");
    const HostTables &t = h->t;
    const size_t n = t.n_var;
    if (work_bytes < n * 32) return fail(HEOM_E_TOO_LARGE, "work buffer smaller than work_bytes");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double2 *y = static_cast<double2 *>(y_dev);
    if (obs_every > 0) {
        hipLaunchKernelGGL(observables_kernel, dim3(1), dim3(64), 0, s, dev_view(t), y, obs_dev);
        HIP_TRY(hipGetLastError());
    }
    const double h1 = dt / 4.0, h2 = dt / 3.0, h3 = dt / 2.0, h4 = dt;
    int rc;
    if (precision == HEOM_FP64) {
        double2 *wa = static_cast<double2 *>(work_dev);
        double2 *wb = wa + n;
        for (int64_t st = 1; st <= nsteps; ++st) {
            double *ob = (obs_every > 0 && st % obs_every == 0) ? obs_dev + (st / obs_every) * HEOM_NOBS : nullptr;
            if ((rc = launch_stage<InF64, double2, true, true, false>(t, s, InF64{y}, y, nullptr, 0.0, wa, h1, nullptr))) return rc;
            if ((rc = launch_stage<InF64, double2, true, false, false>(t, s, InF64{wa}, y, nullptr, 0.0, wb, h2, nullptr))) return rc;
            if ((rc = launch_stage<InF64, double2, true, false, false>(t, s, InF64{wb}, y, nullptr, 0.0, wa, h3, nullptr))) return rc;
            if ((rc = launch_stage<InF64, double2, true, false, false>(t, s, InF64{wa}, y, nullptr, 0.0, y, h4, ob))) return rc;
        }
    } else {
        double2 *y2 = static_cast<double2 *>(work_dev);
        float2 *u1 = reinterpret_cast<float2 *>(y2 + n);
        float2 *u2 = u1 + n;
        double2 *cur = y, *nxt = y2;
        const double inv_h1 = 1.0 / h1;
        for (int64_t st = 1; st <= nsteps; ++st) {
            double *ob = (obs_every > 0 && st % obs_every == 0) ? obs_dev + (st / obs_every) * HEOM_NOBS : nullptr;
            if ((rc = launch_stage<InF64, float2, false, false, false>(t, s, InF64{cur}, nullptr, nullptr, 0.0, u1, h1, nullptr))) return rc;
            if ((rc = launch_stage<InF32, float2, false, false, true>(t, s, InF32{u1}, nullptr, u1, inv_h1, u2, h2, nullptr))) return rc;
            if ((rc = launch_stage<InF32, float2, false, false, true>(t, s, InF32{u2}, nullptr, u1, inv_h1, u1, h3, nullptr))) return rc;
            if ((rc = launch_stage<InSum, double2, true, false, false>(t, s, InSum{cur, u1}, cur, nullptr, 0.0, nxt, h4, ob))) return rc;
            std::swap(cur, nxt);
        }
        if (cur != y) {
            hipLaunchKernelGGL(copy_kernel, dim3(1024), dim3(256), 0, s, cur, y, t.n_var);
            HIP_TRY(hipGetLastError());
        }
    }
    return HEOM_OK;
}

int heom_export_layout(const heom_tables *h, int64_t *out, size_t cap, size_t *needed) {
    if (!h || !needed) return fail(HEOM_E_INVAL, "NULL argument");
    const HostTables &t = h->t;
    std::vector<int64_t> v;
    v.push_back((int64_t)t.hdr.size());
    v.push_back(t.n_var);
    v.push_back(t.m);
    v.push_back(t.d);
    for (const PatHdr &H : t.hdr) {
        v.push_back(H.off);
        v.push_back(H.G);
        v.push_back(H.tier);
        for (int q = 0; q < H.G; ++q) {
            const CatRec &c = t.cat[H.cat_base + q];
            v.push_back((c.flags & CAT_DIST) ? q : -1);
            v.push_back((c.flags & CAT_ZERO) ? (t.N - t.d - (int64_t)H.r) : (int64_t)c.mult);
            for (int k = 0; k < t.m; ++k) v.push_back(vcomp(c.vec, k));
        }
    }
    for (const PatHdr &H : t.hdr) {
        const bool chi = H.tier < t.L;
        for (int q = 0; q < H.G; ++q) {
            const CatRec &c = t.cat[H.cat_base + q];
            for (int k = 0; k < t.m; ++k) {
                for (int dir = 0; dir < 2; ++dir) {
                    uint32_t idx;
                    if (dir == 0) {
                        if (!chi) continue;
                        idx = H.conn_base + c.conn_off + k;
                    } else {
                        if (vcomp(c.vec, k) == 0) continue;
                        idx = H.conn_base + c.conn_off + (chi ? t.m : 0);
                        for (int j = 0; j < k; ++j) idx += vcomp(c.vec, j) != 0;
                    }
                    const Conn &cr = t.conn[idx];
                    v.push_back(t.conn_target[idx]);
                    v.push_back(conn_q(cr.info));
                    for (int r = 0; r < H.G; ++r)
                        v.push_back((r == q && (conn_vanish(cr.info) || (c.flags & CAT_DIST)))
                                        ? -1 : conn_remap(cr.info, q, r));
                }
            }
        }
    }
    *needed = v.size();
    if (out) {
        if (cap < v.size()) return fail(HEOM_E_TOO_LARGE, "output capacity too small");
        std::copy(v.begin(), v.end(), out);
    }
    return HEOM_OK;
}

int heom_export_coefficients(const heom_tables *h, double *out, size_t cap, size_t *needed) {
    if (!h || !needed) return fail(HEOM_E_INVAL, "NULL argument");
    *needed = h->t.lut.size();
    if (out) {
        if (cap < h->t.lut.size()) return fail(HEOM_E_TOO_LARGE, "output capacity too small");
        std::copy(h->t.lut.begin(), h->t.lut.end(), out);
    }
    return HEOM_OK;
}

void heom_free_tables(heom_tables *h) { delete h; }

const char *heom_last_error(void) { return g_err.c_str(); }

const char *heom_version(void) { return "heom-mi355x 0.1 (gfx950)"; }

}  // extern "C"
