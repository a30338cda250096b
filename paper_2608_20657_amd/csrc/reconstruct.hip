// Dense rho_S(t) by linear reconstruction (Sec. VI.C, Table II) on gfx950.
//
// The reduced map is linear in rho_S(0) and covariant under relabelings of
// the molecules (Eqs. Gt-linearity, Gt-covariance). An arbitrary
// single-excitation rho_S(0) splits into five operator types (Eq.
// arbitrary-initial-expansion): |c><c|, |e_k><c|, |c><e_k|, |e_k><e_k| and
// |e_k><e_l| (k != l), and every operator of a type is a relabeling of one
// representative. Given the representatives' responses at one time as slot
// matrices (cavity, distinguished molecules, two pool molecules) the dense
// output is the sum over types of the relabeled responses weighted by
// rho_S(0)'s entries of that type. Summed over the relabelings the weights
// enter only through their totals and, for |e_k><e_l|, the row and column
// sums of rho_S(0)'s molecule block, so each output entry is a short closed
// form; the cost is one pass over the (N+1)^2 entries.
//
// Three launches per call: row and column sums of the molecule block (one
// workgroup per row for the row sums, one thread per column for the column
// sums), the totals (one workgroup), and the entries (one thread each).

#include <hip/hip_runtime.h>

#include <string>

#include "heom_internal.h"

namespace {

typedef double2 cplx;

__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Slot matrices of the five representatives at one time, by value.
struct Slots {
    cplx cc[3][3];    // |c><c|, d = 0: cavity, two pool molecules
    cplx ec[4][4];    // |e_1><c|, d = 1: cavity, e_1, two pool molecules
    cplx ce[4][4];    // |c><e_1|
    cplx ee[4][4];    // |e_1><e_1|
    cplx e12[5][5];   // |e_1><e_2|, d = 2: cavity, e_1, e_2, two pool molecules
    uint32_t mask;    // representatives present (bit order as above)
};

// work: r[N], s[N] (row and column sums of the molecule block without its
// diagonal), then the totals W_ec, W_ce, W_ee, W_m.
constexpr int RB = 256;

__global__ __launch_bounds__(RB) void row_sums_kernel(const cplx *rho0, uint32_t N, cplx *r) {
    // workgroup i: row i+1 of rho0 over molecule columns j != i+1
    __shared__ cplx part[RB];
    const uint32_t i = blockIdx.x, D = N + 1u;
    const cplx *row = rho0 + (size_t)(i + 1u) * D;
    cplx acc = make_double2(0.0, 0.0);
    for (uint32_t j = threadIdx.x; j < N; j += RB)
        if (j != i) acc = cadd(acc, row[j + 1u]);
    part[threadIdx.x] = acc;
    __syncthreads();
    for (uint32_t w = RB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] = cadd(part[threadIdx.x], part[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) r[i] = part[0];
}

__global__ __launch_bounds__(RB) void col_sums_kernel(const cplx *rho0, uint32_t N, cplx *s) {
    // thread j: column j+1 of rho0 over molecule rows i != j+1 (adjacent
    // threads read adjacent entries of each row)
    const uint32_t j = blockIdx.x * RB + threadIdx.x, D = N + 1u;
    if (j >= N) return;
    cplx acc = make_double2(0.0, 0.0);
    for (uint32_t i = 0; i < N; ++i)
        if (i != j) acc = cadd(acc, rho0[(size_t)(i + 1u) * D + j + 1u]);
    s[j] = acc;
}

__global__ __launch_bounds__(RB) void totals_kernel(const cplx *rho0, uint32_t N, const cplx *r, cplx *tot) {
    // one workgroup: W_ec = sum_k rho0[k][c], W_ce = sum_k rho0[c][k],
    // W_ee = sum_k rho0[k][k], W_m = sum_k r_k
    __shared__ cplx part[4][RB];
    const uint32_t D = N + 1u;
    cplx a = make_double2(0.0, 0.0), b = a, c = a, m = a;
    for (uint32_t k = threadIdx.x; k < N; k += RB) {
        a = cadd(a, rho0[(size_t)(k + 1u) * D]);
        b = cadd(b, rho0[k + 1u]);
        c = cadd(c, rho0[(size_t)(k + 1u) * D + k + 1u]);
        m = cadd(m, r[k]);
    }
    part[0][threadIdx.x] = a;
    part[1][threadIdx.x] = b;
    part[2][threadIdx.x] = c;
    part[3][threadIdx.x] = m;
    __syncthreads();
    for (uint32_t w = RB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int q = 0; q < 4; ++q) part[q][threadIdx.x] = cadd(part[q][threadIdx.x], part[q][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x < 4) tot[threadIdx.x] = part[threadIdx.x][0];
}

// sum_k w_k U_k G U_k^+ at entry (a, b) for a d = 1 response R (slots c, e_1,
// p, q; molecule k takes e_1's place, the others are pool molecules); 0 is
// the cavity, molecules are 1..N.
__device__ cplx d1_entry(const cplx (*R)[4], uint32_t a, uint32_t b, cplx wa, cplx wb, cplx W) {
    if (a == 0 && b == 0) return cmul(W, R[0][0]);
    if (a == 0) return cadd(cmul(wb, R[0][1]), cmul(csub(W, wb), R[0][2]));
    if (b == 0) return cadd(cmul(wa, R[1][0]), cmul(csub(W, wa), R[2][0]));
    if (a == b) return cadd(cmul(wa, R[1][1]), cmul(csub(W, wa), R[2][2]));
    return cadd(cadd(cmul(wa, R[1][2]), cmul(wb, R[2][1])), cmul(csub(csub(W, wa), wb), R[2][3]));
}

__global__ __launch_bounds__(RB) void dense_kernel(const cplx *rho0, uint32_t N, const cplx *work, Slots S,
                                                   cplx *out) {
    const uint32_t D = N + 1u;
    const size_t e = (size_t)blockIdx.x * RB + threadIdx.x;
    if (e >= (size_t)D * D) return;
    const uint32_t a = (uint32_t)(e / D), b = (uint32_t)(e % D);
    const cplx *r = work, *s = work + N, *tot = work + 2u * (size_t)N;
    cplx acc = make_double2(0.0, 0.0);
    if (S.mask & 1u) {   // rho0[c][c] |c><c|: every relabeling leaves it as it is
        // slots: cavity, a pool molecule, a second pool molecule
        const uint32_t sa = a == 0 ? 0u : 1u, sb = b == 0 ? 0u : ((a == 0 || a == b) ? 1u : 2u);
        acc = cadd(acc, cmul(rho0[0], S.cc[sa][sb]));
    }
    // |e_k><c| weighted by rho0[k][c], |c><e_k| by rho0[c][k], |e_k><e_k| by rho0[k][k]
    if (S.mask & 2u) {
        const cplx wa = a ? rho0[(size_t)a * D] : make_double2(0.0, 0.0), wb = b ? rho0[(size_t)b * D] : wa;
        acc = cadd(acc, d1_entry(S.ec, a, b, wa, wb, tot[0]));
    }
    if (S.mask & 4u) {
        const cplx wa = a ? rho0[a] : make_double2(0.0, 0.0), wb = b ? rho0[b] : wa;
        acc = cadd(acc, d1_entry(S.ce, a, b, wa, wb, tot[1]));
    }
    if (S.mask & 8u) {
        const cplx wa = a ? rho0[(size_t)a * D + a] : make_double2(0.0, 0.0), wb = b ? rho0[(size_t)b * D + b] : wa;
        acc = cadd(acc, d1_entry(S.ee, a, b, wa, wb, tot[2]));
    }
    if (S.mask & 16u) {
        // |e_k><e_l| (k != l) weighted by rho0[k][l]: molecule k takes e_1's
        // place and l e_2's; r_k, s_k = sums of row and column k without the
        // diagonal, W = their total
        const cplx W = tot[3];
        cplx v;
        if (a == 0 && b == 0) {
            v = cmul(W, S.e12[0][0]);
        } else if (a == 0 || b == 0) {
            const uint32_t k = (a ? a : b) - 1u;
            const cplx rest = csub(csub(W, r[k]), s[k]);
            v = a == 0 ? cadd(cadd(cmul(r[k], S.e12[0][1]), cmul(s[k], S.e12[0][2])), cmul(rest, S.e12[0][3]))
                       : cadd(cadd(cmul(r[k], S.e12[1][0]), cmul(s[k], S.e12[2][0])), cmul(rest, S.e12[3][0]));
        } else if (a == b) {
            const uint32_t k = a - 1u;
            const cplx rest = csub(csub(W, r[k]), s[k]);
            v = cadd(cadd(cmul(r[k], S.e12[1][1]), cmul(s[k], S.e12[2][2])), cmul(rest, S.e12[3][3]));
        } else {
            const uint32_t i = a - 1u, j = b - 1u;
            const cplx wij = rho0[(size_t)a * D + b], wji = rho0[(size_t)b * D + a];
            // molecules a, b are: e_1 and e_2 (weight w_ab), e_2 and e_1 (w_ba),
            // e_1 and a pool molecule (r_a - w_ab), e_2 and pool (s_a - w_ba),
            // pool and e_1 (r_b - w_ba), pool and e_2 (s_b - w_ab), or both in
            // the pool (the rest)
            const cplx rest = cadd(cadd(csub(csub(csub(csub(W, r[i]), s[i]), r[j]), s[j]), wij), wji);
            v = cmul(wij, S.e12[1][2]);
            v = cadd(v, cmul(wji, S.e12[2][1]));
            v = cadd(v, cmul(csub(r[i], wij), S.e12[1][3]));
            v = cadd(v, cmul(csub(s[i], wji), S.e12[2][3]));
            v = cadd(v, cmul(csub(r[j], wji), S.e12[3][1]));
            v = cadd(v, cmul(csub(s[j], wij), S.e12[3][2]));
            v = cadd(v, cmul(rest, S.e12[3][4]));
        }
        acc = cadd(acc, v);
    }
    out[e] = acc;
}

void load(cplx *dst, const double *src, int n) {
    for (int i = 0; i < n; ++i) dst[i] = make_double2(src[2 * i], src[2 * i + 1]);
}

}  // namespace

extern "C" {

size_t heom_reconstruct_work_bytes(int64_t N) {
    if (N < 1 || N > HEOM_RECON_MAX_N) return 0;
    return sizeof(cplx) * (2 * (size_t)N + 4);
}

int heom_reconstruct_dense(int64_t N, const void *rho0_dev, const double *R, uint32_t mask, void *work_dev,
                           size_t work_bytes, void *out_dev, void *stream) {
    if (N < 1 || N > HEOM_RECON_MAX_N) return heom::set_error(HEOM_E_INVAL, "N out of range for the dense output");
    if (!rho0_dev || !R || !work_dev || !out_dev) return heom::set_error(HEOM_E_INVAL, "NULL pointer");
    if ((reinterpret_cast<uintptr_t>(rho0_dev) | reinterpret_cast<uintptr_t>(work_dev) |
         reinterpret_cast<uintptr_t>(out_dev)) % 16)
        return heom::set_error(HEOM_E_INVAL, "device buffers must be 16-byte aligned");
    if (mask & ~(0x1fu | HEOM_RECON_CE_ADJOINT)) return heom::set_error(HEOM_E_INVAL, "unknown mask bits");
    if ((mask & HEOM_RECON_CE_ADJOINT) && (mask & 4u) == 0)
        return heom::set_error(HEOM_E_INVAL, "the adjoint form is for the |c><e_1| type");
    if (work_bytes < heom_reconstruct_work_bytes(N)) return heom::set_error(HEOM_E_TOO_LARGE, "work buffer too small");
    Slots S;
    load(&S.cc[0][0], R, 9);
    load(&S.ec[0][0], R + 18, 16);
    load(&S.ce[0][0], R + 50, 16);
    load(&S.ee[0][0], R + 82, 16);
    load(&S.e12[0][0], R + 114, 25);
    if (mask & HEOM_RECON_CE_ADJOINT) {
        // the response to |c><e_1| is the adjoint of the response to |e_1><c|
        // (Eq. adjoint-preservation)
        for (int x = 0; x < 4; ++x)
            for (int y = 0; y < 4; ++y) S.ce[x][y] = make_double2(S.ec[y][x].x, -S.ec[y][x].y);
    }
    S.mask = mask & 0x1fu;
    const uint32_t n = (uint32_t)N;
    const cplx *rho0 = static_cast<const cplx *>(rho0_dev);
    cplx *work = static_cast<cplx *>(work_dev);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(row_sums_kernel, dim3(n), dim3(RB), 0, s, rho0, n, work);
    hipLaunchKernelGGL(col_sums_kernel, dim3((n + RB - 1) / RB), dim3(RB), 0, s, rho0, n, work + n);
    hipLaunchKernelGGL(totals_kernel, dim3(1), dim3(RB), 0, s, rho0, n, work, work + 2 * (size_t)n);
    const size_t entries = (size_t)(n + 1) * (n + 1);
    hipLaunchKernelGGL(dense_kernel, dim3((unsigned)((entries + RB - 1) / RB)), dim3(RB), 0, s, rho0, n,
                       static_cast<const cplx *>(work), S, static_cast<cplx *>(out_dev));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return heom::set_error(HEOM_E_HIP, std::string("reconstruction launch: ") + hipGetErrorString(e));
    return HEOM_OK;
}

}  // extern "C"
