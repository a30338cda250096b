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
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>

#include "heom_internal.h"

using namespace heom;

struct heom_tables {
    HostTables t;
};

struct BatchSlotHost {
    bool used = false;
    const heom_tables *tables = nullptr;
    const void *params = nullptr;   // caller's parameter block, or null: the one in the tables' image
    bool adjoint = false;           // c_check = conj(c) for this slot's parameters (resolved at commit)
    void *y = nullptr, *work = nullptr;
    size_t work_bytes = 0;
    double dt = 0.0;
    double *obs = nullptr;
    int64_t obs_every = 0, obs_cap = 0, steps = 0;
};

// One slot of a batch: an uploaded structure image, a params block (the
// head of an image: InstParams + coefficient tables) and the slot's own
// state, work and observable buffers.
struct SlotRec {
    const unsigned char *img;
    const unsigned char *params;
    // table sections of img and the coefficient tables of params, resolved on
    // the host so that a workgroup's first loads do not wait for each other
    const PatHdr *hdr;
    const CatRec *cat;
    const uint32_t *gidx;
    const TileRec *tiles;
    const VarRec *vrec;
    const double *lut;
    double2 *y, *w0, *w1;     // FP64 stage vectors
    float2 *u1, *u2, *u3;     // FP32 increments
    double2 *yT, *w0T, *w1T;  // transposed copies (null without them)
    float2 *u1T, *u2T, *u3T;
    double *obs;
    int64_t obs_every, obs_cap, step0;
    double dt;
};
struct BatchTile {
    uint32_t slot, tile;   // tile | BTILE_TOP for a tile of the top tier
};
constexpr uint32_t BTILE_TOP = 0x80000000u;

struct heom_batch {
    std::vector<BatchSlotHost> slots;
    bool committed = false;
    void *dev = nullptr;
    size_t dev_bytes = 0;
    int64_t steps_since_commit = 0;
    // One launch per group: tiles of one m, one tile size and one tier class
    // (top-tier tiles have no up moves and run a lighter kernel variant).
    struct Group {
        int m;       // 0: the small groups' tiles in one launch (batch_stage_merged)
        bool top;
        uint32_t block, lds, first, count;
        int32_t slot;     // >= 0: tiles tile0.. of this slot alone (batch_stage_single)
        uint32_t tile0;
        bool shared = false;   // tiles of structures shared by several slots (batch_stage_shared)
        bool compact = false;  // every slot of the group has compact tiles (kernels specialised for them)
    };
    std::vector<SlotRec> recs;        // host copy of the committed slot records
    std::vector<Group> groups;
    // Steps replayed from a captured HIP graph (0 = launch every kernel).
    int32_t graph_steps = 0;
    // The smallest groups with m <= 4, up to this many tiles in all, run each
    // stage as one launch instead of one per group.
    int32_t merge_tiles = 16384;
    // Slots that share one structure image: 2 = computed in pairs, side by
    // side in one workgroup per tile (batch_stage_pair), 1 = every slot has
    // its own workgroups.
    int32_t share_slots = 1;
    // Slots that share one structure image, in the groups with one
    // workgroup per slot and tile: 0 = slot by slot, c > 0 = chunks of c
    // consecutive tiles taken from each such slot in turn.
    int32_t interleave = 32;
    size_t list_off = 0;                // slot lists of the shared groups in the batch buffer
    hipGraphExec_t gexec = nullptr;
    int gprec = -1;
    size_t ctr_off = 0;                 // device step counter in the batch buffer
    ~heom_batch() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
    }
};

// Work memory of heom_propagate_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends. In host code `scratch` names a
// host-side stand-in, never the device memory: its device address is looked
// up once per device (hipGetSymbolAddress, with that device current, in
// scratch_address below) and only that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[HEOM_NOALLOC_WORK_BYTES];

namespace {

thread_local std::string g_err;

// Parameter blocks written by heom_upload_params, by device address: the
// tables handle and image layout they were written for, and whether their
// bath maps Hermitian ADOs to Hermitian ADOs. A batch commit checks a slot's
// block against its tables here, so a block left over from before a
// re-tuning (other LDS layout, section offsets or tile kind) is refused
// instead of read.
struct ParamsStamp {
    uint64_t tables_id, layout_gen;
    bool adjoint;
};
std::mutex g_params_mu;
std::unordered_map<uintptr_t, ParamsStamp> g_params;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

}  // namespace

int heom::set_error(int code, const std::string &msg) { return fail(code, msg); }

namespace {

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
    const uint32_t *gidx;
    const TileRec *tiles;
    const VarRec *vrec;
};

Dev dev_view(const HostTables &t) {
    const unsigned char *b = static_cast<const unsigned char *>(t.dev);
    const InstParams *ip = reinterpret_cast<const InstParams *>(t.image.data());
    Dev D;
    D.ip = reinterpret_cast<const InstParams *>(b);
    D.lut = reinterpret_cast<const double *>(b + ip->off_lut);
    D.hdr = reinterpret_cast<const PatHdr *>(b + ip->off_hdr);
    D.cat = reinterpret_cast<const CatRec *>(b + ip->off_cat);
    D.gidx = reinterpret_cast<const uint32_t *>(b + ip->off_gidx);
    D.tiles = reinterpret_cast<const TileRec *>(b + ip->off_tile);
    D.vrec = reinterpret_cast<const VarRec *>(b + ip->off_vrec);
    return D;
}

// ------------------------------------------------------------ complex ops
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// acc += w * v, as explicit fused multiply-adds: their rounding is fixed,
// so kernel variants that order or contract the surrounding code differently
// (the top-tier variant, batch kernels) still sum a variable's terms alike
__device__ __forceinline__ void cfma(double2 &acc, double2 w, double2 v) {
    acc.x = fma(-w.y, v.y, fma(w.x, v.x, acc.x));
    acc.y = fma(w.y, v.x, fma(w.x, v.y, acc.y));
}

// blockIdx -> tile such that each of the 8 XCDs (workgroups are dealt to
// XCDs round robin) processes one contiguous run of tiles.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n) {
    const uint32_t X = 8;
    uint32_t q = n / X, rem = n % X, x = b % X, idx = b / X;
    return x < rem ? x * (q + 1) + idx : rem * (q + 1) + (x - rem) * q + idx;
}

__device__ __forceinline__ uint32_t vbyte(uint64_t v, int k) { return (uint32_t)(v >> (8 * k)) & 0xffu; }

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

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double2 ld_stream(const double2 *p) {
    const dvec2 v = __builtin_nontemporal_load(reinterpret_cast<const dvec2 *>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st_stream(double2 *p, double2 v) {
    dvec2 w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<dvec2 *>(p));
}
__device__ __forceinline__ void st_stream(float2 *p, double2 v) {
    fvec2 w = {(float)v.x, (float)v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<fvec2 *>(p));
}

// Vectors one stage reads and writes:
//   out[i] = base(i) + alpha * ((M_u in)[i] + extra_scale * extra[i])
// with in = in64 (+ in32), base = in (BASE 1) or ybase (BASE 2) or 0.
// With transposed copies, inT64 / inT32 hold `in` with every block's
// category matrix transposed (column moves gather there) and outT64 /
// outT32, if set, receive `out` in the same form; a null inT means `in`.
struct StageArgs {
    const double2 *in64;
    const float2 *in32;
    const double2 *inT64;
    const float2 *inT32;
    double2 *outT64;
    float2 *outT32;
    const double2 *ybase;
    const float2 *extra;
    double extra_scale;
    double2 *out64;
    float2 *out32;
    double alpha;
    double *obs;          // observables of the tier-0 block after this stage
    uint32_t policy;      // bit 0: non-temporal own-value loads, 1: y loads, 2: stores;
                          // bit 3: mirrored column gathers (see load_col)
    uint32_t tile0;       // first tile of this launch
};

enum { BASE_NONE = 0, BASE_IN = 1, BASE_Y = 2 };

// LDS carve-up of one workgroup: tile values, pattern headers, categories,
// coefficient tables, category multiplicities, gather indices, grouped sums.
// The gather indices are read only before the workgroup's first barrier and
// the grouped sums written only after it, so a workgroup that stages its
// tile's metadata for one stage (`overlay`) keeps the sums in the gather
// list's place: its LDS is the larger of the two, not their sum (the
// lower-tier tiles of the probe: 25.1 -> 18.0 KB). The persistent kernel
// keeps a tile's metadata for every stage, and so the sums after the list.
struct Smem {
    double2 *val;
    double2 *rc;      // grouped sums of the tile's blocks (see process_tile)
    PatHdr *hdr;
    CatRec *cat;
    uint32_t *gix;
    double *lut;
    double *md;       // M_q of the tile's categories as doubles (M_0 resolved per instance)
    uint32_t rco;     // rc - val, in values
};

__device__ __forceinline__ Smem carve(unsigned char *smem, const InstParams &P, bool overlay) {
    Smem S;
    S.val = reinterpret_cast<double2 *>(smem);
    S.hdr = reinterpret_cast<PatHdr *>(smem + 16u * P.val_len);
    S.cat = reinterpret_cast<CatRec *>(S.hdr + P.max_np);
    S.lut = reinterpret_cast<double *>(S.cat + P.max_nc);
    S.md = S.lut + 2u * (uint32_t)P.m * (uint32_t)(P.L + 1);
    S.gix = reinterpret_cast<uint32_t *>(S.md + ((P.max_nc + 1u) & ~1u));
    S.rc = reinterpret_cast<double2 *>(S.gix + (overlay ? 0u : (P.max_ng + 3u) & ~3u));
    S.rco = (uint32_t)(S.rc - S.val);
    return S;
}

// LDS of a workgroup holding two problems of one structure: the shared
// metadata (headers, categories, gather indices for max_ng), then per half
// the tile values and grouped sums, coefficient tables and multiplicities.
__host__ __device__ __forceinline__ uint32_t pair_shared_bytes(const InstParams &P) {
    return 32u * P.max_np + 16u * P.max_nc + 4u * ((P.max_ng + 3u) & ~3u);
}
__host__ __device__ __forceinline__ uint32_t pair_half_bytes(const InstParams &P) {
    return 32u * P.val_len + 16u * (uint32_t)P.m * (uint32_t)(P.L + 1) + 8u * ((P.max_nc + 1u) & ~1u);
}
__device__ __forceinline__ Smem carve_pair(unsigned char *smem, const InstParams &P, uint32_t half) {
    Smem S;
    S.hdr = reinterpret_cast<PatHdr *>(smem);
    S.cat = reinterpret_cast<CatRec *>(S.hdr + P.max_np);
    S.gix = reinterpret_cast<uint32_t *>(S.cat + P.max_nc);
    unsigned char *h = smem + pair_shared_bytes(P) + half * pair_half_bytes(P);
    S.val = reinterpret_cast<double2 *>(h);
    S.rc = S.val + P.val_len;
    S.rco = P.val_len;
    S.lut = reinterpret_cast<double *>(h + 32u * P.val_len);
    S.md = S.lut + 2u * (uint32_t)P.m * (uint32_t)(P.L + 1);
    return S;
}

// Copy a tile's metadata (pattern headers, categories, gather indices) and,
// if lut_words > 0, the coefficient tables into LDS, as 16-byte words. The
// four sources are one index range, and each thread issues its loads (two
// words per round) before it writes any of them, so the copy costs about
// one memory latency instead of one per array and round. Every section
// starts 16-byte aligned in the image and in LDS (a tile's gather list is
// padded to a multiple of four indices).
__device__ __forceinline__ void stage_tile(const Dev &D, const TileRec &TR, const Smem &S, uint32_t lut_words) {
    const uint32_t e1 = 2u * TR.np, e2 = e1 + TR.nc, e3 = e2 + ((TR.ng + 3u) >> 2), e4 = e3 + lut_words;
    const uint4 *sh = reinterpret_cast<const uint4 *>(D.hdr + TR.p0);
    const uint4 *sc = reinterpret_cast<const uint4 *>(D.cat + TR.c0);
    const uint4 *sg = reinterpret_cast<const uint4 *>(D.gidx + TR.g0);
    const uint4 *sl = reinterpret_cast<const uint4 *>(D.lut);
    uint4 *dh = reinterpret_cast<uint4 *>(S.hdr), *dc = reinterpret_cast<uint4 *>(S.cat);
    uint4 *dg = reinterpret_cast<uint4 *>(S.gix), *dl = reinterpret_cast<uint4 *>(S.lut);
    const uint32_t bd = blockDim.x;
    for (uint32_t b = threadIdx.x; b < e4; b += 2u * bd) {
        uint4 r0 = make_uint4(0u, 0u, 0u, 0u), r1 = r0;
        const uint32_t i0 = b, i1 = b + bd;
        auto src = [&](uint32_t i) {
            return i < e1 ? sh + i : (i < e2 ? sc + (i - e1) : (i < e3 ? sg + (i - e2) : sl + (i - e3)));
        };
        auto dst = [&](uint32_t i) {
            return i < e1 ? dh + i : (i < e2 ? dc + (i - e1) : (i < e3 ? dg + (i - e2) : dl + (i - e3)));
        };
        if (i0 < e4) r0 = *src(i0);
        if (i1 < e4) r1 = *src(i1);
        if (i0 < e4) *dst(i0) = r0;
        if (i1 < e4) *dst(i1) = r1;
    }
}

// 16-byte words of the coefficient tables (2 m (L+1) doubles).
__device__ __forceinline__ uint32_t lut_words(const InstParams &P) { return (uint32_t)P.m * (uint32_t)(P.L + 1); }

__device__ __forceinline__ void stage_lut(const Dev &D, const InstParams &P, double *lut) {
    const uint32_t n = 2u * lut_words(P);
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) lut[i] = D.lut[i];
}

template <bool HAS64, bool HAS32>
__device__ __forceinline__ double2 load_in(const StageArgs &a, uint32_t j) {
    double2 v = make_double2(0.0, 0.0);
    if (HAS64) v = a.in64[j];
    if (HAS32) {
        const float2 u = a.in32[j];
        v.x += (double)u.x;
        v.y += (double)u.y;
    }
    return v;
}

template <bool HAS64, bool HAS32>
__device__ __forceinline__ double2 load_own(const StageArgs &a, uint32_t j) {
    if (!(a.policy & 1u)) return load_in<HAS64, HAS32>(a, j);
    double2 v = make_double2(0.0, 0.0);
    if (HAS64) v = ld_stream(a.in64 + j);
    if (HAS32) {
        const fvec2 u = __builtin_nontemporal_load(reinterpret_cast<const fvec2 *>(a.in32 + j));
        v.x += (double)u.x;
        v.y += (double)u.y;
    }
    return v;
}

// One fused stage over one tile, one thread per unique variable.
//
// 1. The thread's own loads (its decode record, input value, base and extra
//    terms) go out first and stay in flight while the tile's metadata and
//    coefficient tables are staged into LDS (stage_tile; skipped when
//    `stage` is false and they are there already). Barriers wait for LDS
//    traffic only.
// 2. Every variable has up to 4M hierarchy gathers ("slots"): for each
//    channel k, the row molecule raised (k), lowered (M+k), the column
//    molecule raised (2M+k), lowered (3M+k) (Eqs. uvar-up, uvar-down). The
//    record names the live slots and where their target indices sit in the
//    tile's list; the gathers go out in one batch (two, up moves then down
//    moves, where m >= 3 and the tier has up moves) and their weighted sum
//    is formed before the barrier that publishes the tile's values.
// 3. Grouped sums (Eqs. grouped-row-sum, grouped-column-sum, HZ): in each
//    block, the thread at position l < 2G+1 forms one of them -- l = 0 the
//    Z bracket sum_q M_q (X_q - Y_q), l = 1..G the row sum R_{l-1}, l =
//    G+1..2G the column sum C_{l-1-G} -- into LDS, so the loops over the
//    block's categories run on a few lanes instead of on every lane. Each
//    sum walks one strided run of the block (column 0, row c+1 or column
//    c+1) with the multiplicities the threads l = 1..G wrote to LDS as
//    doubles during the gathers; the excluded diagonal term gets weight 0,
//    so the loop body has no branches.
// 4. Every thread reads its Hamiltonian bracket from LDS, adds damping,
//    loss, the terminator and the extra term, and writes the combination.
// Compact tiles (Hermitian ADOs) cover only the entries with row <= column
// and the T_q: a thread also fills its mirrored entry (the conjugate) into
// LDS, the grouped sums are the Z bracket and the row sums (the column sums
// are their conjugates), and the results go through LDS so that the tile's
// variables are stored as one contiguous run.
// What a call of process_tile stages into LDS before computing: nothing (the
// tile's metadata and coefficient tables are there already), everything, or
// only the coefficient tables (the metadata of the same tile is there, for
// another problem with its own parameters).
// STAGE_PAIR: two problems of the same structure side by side in one
// workgroup (each half of the threads computes one of them): the tile's
// metadata is staged once by all threads, each half stages its problem's
// coefficient tables into its own LDS region.
enum { STAGE_NONE = 0, STAGE_ALL = 1, STAGE_LUT = 2, STAGE_PAIR = 3 };

__device__ __forceinline__ void stage_lut_words(const Dev &D, const Smem &S, uint32_t words) {
    const uint4 *src = reinterpret_cast<const uint4 *>(D.lut);
    uint4 *dst = reinterpret_cast<uint4 *>(S.lut);
    for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
}

// tbase, tcount: the threads that compute this problem (all of the block,
// or one half of it for STAGE_PAIR).
template <int M, bool HAS64, bool HAS32, int BASE, bool EXTRA, bool OUT64, bool TOP, int CM>
__device__ __forceinline__ void process_tile(const InstParams &P, const Dev &D, const TileRec &TR, const Smem &S,
                                             const StageArgs &a, bool first_tile, int stage, uint32_t lut_w,
                                             uint32_t tbase = 0u, uint32_t tcount = 0u) {
    const uint32_t t = threadIdx.x - tbase;
    const uint32_t tn = tcount ? tcount : blockDim.x;
    const bool active = t < TR.nv;
    // compact tiles: this thread's entry is variable vt of the tile (row <=
    // column or a T_q); it also owns the mirrored entry, the conjugate.
    // CM: 0 plain tiles, 1 compact tiles, 2 as the parameter block says
    // (batches, whose slots may differ)
    const bool cmp = CM == 2 ? P.compact != 0 : CM == 1;
    uint32_t vt = t;
    double2 own = make_double2(0.0, 0.0), ybv = make_double2(0.0, 0.0);
    float2 ex = make_float2(0.0f, 0.0f);
    VarRec vr{0u, 0u};
    if (active) {
        vr = D.vrec[TR.v0 + t];
        if (!cmp) {
            own = load_own<HAS64, HAS32>(a, TR.v0 + vt);
            if (BASE == BASE_Y) ybv = (a.policy & 2u) ? ld_stream(a.ybase + TR.v0 + vt) : a.ybase[TR.v0 + vt];
            if (EXTRA) ex = a.extra[TR.v0 + vt];
        }
    }
    if (stage == STAGE_ALL) stage_tile(D, TR, S, lut_w);
    else if (stage == STAGE_LUT) stage_lut_words(D, S, lut_w);
    else if (stage == STAGE_PAIR) {
        stage_tile(D, TR, S, 0u);            // the shared metadata, by every thread of the block
        const uint4 *src = reinterpret_cast<const uint4 *>(D.lut);
        uint4 *dst = reinterpret_cast<uint4 *>(S.lut);
        for (uint32_t i = t; i < lut_w; i += tn) dst[i] = src[i];
    }
    __syncthreads();

    const uint32_t p = vr.x & 127u, A = (vr.x >> 7) & 31u, B = (vr.x >> 12) & 31u;
    const bool isT = (vr.x >> 17) & 1u;
    const uint32_t goff = vr.x >> 18, live = vr.y;
    const PatHdr H = S.hdr[p];
    const uint32_t base = H.off - TR.v0;
    const int G = H.G, G1 = G + 1, nm = G1 * G1;
    if (cmp) {
        // compact tiles: the thread's entry follows from its record and the
        // block's header (category matrix row-major, then the T_q in category
        // order); its own value is loaded now and arrives with the first
        // gathers, the base and extra terms after the gathers
        vt = base + (isT ? (uint32_t)nm + (uint32_t)__popc(H.tmask & ((1u << (A - 1u)) - 1u))
                         : A * (uint32_t)G1 + B);
        if (active) own = load_own<HAS64, HAS32>(a, TR.v0 + vt);
    }
    const uint32_t loc = vt - base;
    // position of the mirrored entry (row and column exchanged) in the tile,
    // for compact tiles' off-diagonal entries
    const bool has_mirror = cmp && A != B && !isT;
    const uint32_t vmir = base + B * (uint32_t)G1 + A;
    const int kind = (A == 0 && B == 0) ? KIND_Z : (B == 0 ? KIND_X : (A == 0 ? KIND_Y : ((A == B && !isT) ? KIND_P : KIND_S)));
    const CatRec *cats = S.cat + (H.cat_base - TR.c0);
    double2 hier = make_double2(0.0, 0.0);
    if (active) {
        const CatRec cq = A > 0 ? cats[A - 1] : CatRec{}, cr2 = B > 0 ? cats[B - 1] : CatRec{};
        // Column-move gathers (slots 2M..4M-1) read the transposed copy when
        // there is one. With policy bit 3 the ADOs are Hermitian
        // (rho_n^dagger = rho_n): the entry with row and column exchanged,
        // read from `in` itself at the position the transposed copy would
        // have, is the complex conjugate of the one needed; it is conjugated
        // where it is used. Nothing is done to a value between its load and
        // its use, so the loads of a phase go out as one batch.
        const bool mirror = (a.policy & 8u) != 0;
        const double2 *c64 = (mirror || !a.inT64) ? a.in64 : a.inT64;
        const float2 *c32 = (mirror || !a.inT32) ? a.in32 : a.inT32;
        // +0.0f that the compiler cannot see as a constant (policy < 2^16):
        // with a constant for the dead slots it moves each widening into the
        // load's branch, which then waits for that load alone
        const float fz = __int_as_float((int)(a.policy >> 16));
        // row moves -i sqrt((n+1)|c|), -i sqrt(n/|c|) c_k (P: c_k - cc_k);
        // column moves +i sqrt((n+1)|c|), +i sqrt(n/|c|) cc_k
        const int L1 = P.L + 1;
        const double *up = S.lut;
        const double *dn = S.lut + M * L1;
        // mirrored column gathers are conjugated: sign bit of the imaginary part
        const uint32_t csign = (a.policy & 8u) ? 0x80000000u : 0u;
        auto conj_if = [&](double2 w) {
            const uint64_t b = (uint64_t)__double_as_longlong(w.y) ^ ((uint64_t)csign << 32);
            return make_double2(w.x, __longlong_as_double((long long)b));
        };
        // The terms are summed in one fixed order of positions: row up moves
        // (slot k), column up moves (2M+k), row down moves (M+k), column down
        // moves (3M+k). With m >= 3 and up moves present the gathers go out
        // in two phases, the up moves and then the down moves: all 4M slots
        // in flight at once held 104-109 VGPRs at m = 4 (4 waves per SIMD).
        // The top tier has no up moves and skips their positions.
        constexpr int P0 = TOP ? 2 * M : 0;
        constexpr int NPH = (!TOP && M >= 3) ? 2 : 1;
        constexpr int SPP = (4 * M - P0) / NPH;
        auto slot_at = [](int q) { return q < M ? q : (q < 2 * M ? q + M : (q < 3 * M ? q - M : q)); };
        uint32_t gph = goff;
#pragma unroll
        for (int ph = 0; ph < NPH; ++ph) {
            uint32_t idx[SPP];
            double2 v[SPP];   // FP64 gathers
            float2 f[SPP];    // FP32 gathers, widened where they are used
#pragma unroll
            for (int i = 0; i < SPP; ++i) {
                const int j = slot_at(P0 + ph * SPP + i);
                idx[i] = ((live >> j) & 1u) ? S.gix[gph + __popc(live & ((1u << j) - 1u))] : 0u;
            }
#pragma unroll
            for (int i = 0; i < SPP; ++i) {
                const int j = slot_at(P0 + ph * SPP + i);
                const bool colmv = j >= 2 * M;
                v[i] = make_double2(0.0, 0.0);
                f[i] = make_float2(fz, fz);
                if ((live >> j) & 1u) {
                    if (HAS64) v[i] = (colmv ? c64 : a.in64)[idx[i]];
                    if (HAS32) f[i] = (colmv ? c32 : a.in32)[idx[i]];
                }
            }
            if (ph == 0) {
                S.val[vt] = own;
                if (has_mirror) S.val[vmir] = make_double2(own.x, -own.y);
            }
#pragma unroll
            for (int i = 0; i < SPP; ++i) {
                const int j = slot_at(P0 + ph * SPP + i);
                const int k = j % M, grp = j / M;   // 0 row up, 1 row down, 2 column up, 3 column down
                double2 z = v[i];
                if (HAS32) {
                    z.x += (double)f[i].x;
                    z.y += (double)f[i].y;
                }
                double2 w;
                if (grp == 0) {
                    w = make_double2(0.0, -up[k * L1 + vbyte(cq.vec, k)]);
                } else if (grp == 1) {
                    const double dq = dn[k * L1 + vbyte(cq.vec, k)];
                    const double cre = kind == KIND_P ? P.cr[k] - P.ccr[k] : P.cr[k];
                    const double cim = kind == KIND_P ? P.ci[k] - P.cci[k] : P.ci[k];
                    w = make_double2(dq * cim, -dq * cre);
                } else if (grp == 2) {
                    w = make_double2(0.0, up[k * L1 + vbyte(cr2.vec, k)]);
                    z = conj_if(z);
                } else {
                    const double dr = dn[k * L1 + vbyte(cr2.vec, k)];
                    w = make_double2(-dr * P.cci[k], dr * P.ccr[k]);
                    z = conj_if(z);
                }
                cfma(hier, w, z);
            }
            // the down moves' index reads (and so their loads) depend on the
            // up moves' sum: the compiler would otherwise hoist them and hold
            // all slots at once
            if (ph + 1 < NPH) asm("" : "+v"(gph) : "v"(hier.x), "v"(hier.y));
        }
    }
    if (cmp && active) {
        // used last: loaded after the gathers, they arrive during the grouped sums
        if (BASE == BASE_Y) ybv = (a.policy & 2u) ? ld_stream(a.ybase + TR.v0 + vt) : a.ybase[TR.v0 + vt];
        if (EXTRA) ex = a.extra[TR.v0 + vt];
    }
    double *md = S.md + (H.cat_base - TR.c0);
    if (active && loc - 1u < (uint32_t)G) {   // one thread per category of the block
        const CatRec cc = cats[loc - 1u];
        md[loc - 1u] = (cc.flags & CAT_ZERO) ? (P.npool - (double)H.r) : (double)cc.mult;
    }
    __syncthreads();

    // compact tiles: only the row sums R_c (lanes 1..G, the entries (0, c+1));
    // the column sums of a Hermitian block are their conjugates
    if (active && loc < (uint32_t)(cmp ? G + 1 : 2 * G + 1)) {
        const bool isZ = loc == 0, isRow = loc <= (uint32_t)G;
        const int c = isZ ? -1 : (isRow ? (int)loc - 1 : (int)loc - 1 - G);
        // Z: entries (x+1, 0) minus (0, x+1); R_c: (c+1, x+1); C_c: (x+1, c+1)
        const uint32_t i0 = base + (isZ ? (uint32_t)G1 : (isRow ? (uint32_t)((c + 1) * G1 + 1) : (uint32_t)(G1 + c + 1)));
        const uint32_t st = (isRow && !isZ) ? 1u : (uint32_t)G1;
        double2 sum = make_double2(0.0, 0.0);
        if (!isZ) {
            sum = S.val[base + (c + 1) * G1 + c + 1];
            if ((H.tmask >> c) & 1u)
                sum = cadd(sum, cscale(md[c] - 1.0, S.val[base + nm + __popc(H.tmask & ((1u << c) - 1u))]));
        }
        // branch-free body: the Y_x term is read by every lane and weighted
        // by zf (1 for the Z bracket, else 0); the diagonal's weight is
        // masked to +0 with integer ops, so no load is predicated
        const double zf = isZ ? 1.0 : 0.0;
#pragma unroll 2
        for (int x = 0; x < G; ++x) {
            const double2 w1 = S.val[i0 + (uint32_t)x * st], w2 = S.val[base + 1u + (uint32_t)x];
            const unsigned long long keep = x == c ? 0ull : ~0ull;
            const double mx = __longlong_as_double((long long)((unsigned long long)__double_as_longlong(md[x]) & keep));
            const double2 w = make_double2(w1.x - zf * w2.x, w1.y - zf * w2.y);
            sum = cadd(sum, cscale(mx, w));
        }
        S.rc[base + loc] = sum;
    }
    __syncthreads();

    double2 res = make_double2(0.0, 0.0);
    if (active) {
        // Hamiltonian bracket (multiplied by -i g below):
        //   Z: sum_q M_q (X_q - Y_q)   X_q: Z - R_q   Y_r: C_r - Z
        //   P_q: Y_q - X_q             S_qr, T_q: Y_r - X_q
        // (compact tiles: C_r = conj(R_r))
        const double2 *VR = S.val;   // index rco + i is rc[i]
        const uint32_t vl = S.rco;
        uint32_t i1, i2;
        if (kind == KIND_Z) { i1 = vl + base; i2 = base; }
        else if (kind == KIND_X) { i1 = base; i2 = vl + base + A; }
        else if (kind == KIND_Y) { i1 = vl + base + (cmp ? 0u : (uint32_t)G) + B; i2 = base; }
        else { i1 = base + B; i2 = base + A * G1; }
        double2 h1 = VR[i1];
        const double2 h2 = kind == KIND_Z ? make_double2(0.0, 0.0) : VR[i2];
        if (cmp && kind == KIND_Y) h1.y = -h1.y;
        const double2 hsum = csub(h1, h2);
        double gam = 0.0;
#pragma unroll
        for (int k = 0; k < M; ++k) gam += P.nu[k] * (double)vbyte(H.cnt, k);
        // diagonal: Z -(Gamma + kappa); X, Y -(Gamma + kappa/2 + Delta) -/+ i delta;
        // P -Gamma; S, T -(Gamma + 2 Delta)
        const double re = kind == KIND_Z ? -(gam + P.kappa)
                          : (kind == KIND_X || kind == KIND_Y) ? -(gam + 0.5 * P.kappa + P.term)
                          : (kind == KIND_P ? -gam : -(gam + 2.0 * P.term));
        const double dl = kind == KIND_X ? P.delta : (kind == KIND_Y ? -P.delta : 0.0);
        double2 acc = make_double2(re * own.x + dl * own.y, re * own.y - dl * own.x);
        acc = cadd(acc, hier);
        acc.x += P.g * hsum.y;
        acc.y -= P.g * hsum.x;
        if (EXTRA) {
            acc.x += a.extra_scale * (double)ex.x;
            acc.y += a.extra_scale * (double)ex.y;
        }
        res = cscale(a.alpha, acc);
        if (BASE == BASE_IN) res = cadd(res, own);
        if (BASE == BASE_Y) res = cadd(res, ybv);
        if (!cmp) {
            if (a.policy & 4u) {
                if (OUT64) st_stream(a.out64 + TR.v0 + vt, res);
                else st_stream(a.out32 + TR.v0 + vt, res);
            } else {
                if (OUT64) a.out64[TR.v0 + vt] = res;
                else a.out32[TR.v0 + vt] = make_float2((float)res.x, (float)res.y);
            }
        }
        if (OUT64 ? a.outT64 != nullptr : a.outT32 != nullptr) {
            // position of this entry in the transposed copy (T_q in place)
            const uint32_t tp = TR.v0 + (isT ? vt : vmir);
            if (a.policy & 4u) {
                if (OUT64) st_stream(a.outT64 + tp, res);
                else st_stream(a.outT32 + tp, res);
            } else {
                if (OUT64) a.outT64[tp] = res;
                else a.outT32[tp] = make_float2((float)res.x, (float)res.y);
            }
        }
    }
    __syncthreads();
    if (cmp) {
        // compact tiles: the results and their mirrors are gathered in LDS
        // first, so that the tile's variables are stored as one contiguous
        // run of whole lines (scattered mirror stores leave partial lines)
        if (active) {
            S.val[vt] = res;
            if (has_mirror) S.val[vmir] = make_double2(res.x, -res.y);
        }
        __syncthreads();
        const PatHdr HL = S.hdr[TR.np - 1];
        const uint32_t nfull = HL.off + HL.size - TR.v0;
        for (uint32_t i = t; i < nfull; i += tn) {
            const double2 r = S.val[i];
            if (a.policy & 4u) {
                if (OUT64) st_stream(a.out64 + TR.v0 + i, r);
                else st_stream(a.out32 + TR.v0 + i, r);
            } else {
                if (OUT64) a.out64[TR.v0 + i] = r;
                else a.out32[TR.v0 + i] = make_float2((float)r.x, (float)r.y);
            }
        }
    }
    // the empty pattern is the first block of tile 0: evaluate the
    // observables of the freshly computed tier-0 block (compact tiles hold it
    // in LDS already). With two problems in the block, both halves take the
    // barriers whether or not their problem samples observables now.
    const bool obs_here = a.obs != nullptr && first_tile;
    if (stage == STAGE_PAIR ? first_tile : obs_here) {
        const uint32_t n0 = S.hdr[0].size;
        if (obs_here && !cmp && active && vt < n0) S.val[vt] = res;
        __syncthreads();
        if (obs_here && t == 0) tier0_observables(P, S.hdr[0], S.cat, S.val, a.obs);
        __syncthreads();
    }
}

// One launch = one stage over all tiles (used by heom_rhs and as the
// non-persistent path).
template <int M, bool HAS64, bool HAS32, int BASE, bool EXTRA, bool OUT64, bool TOP, int CM>
__global__ __launch_bounds__(MAX_TILE) void stage_kernel(Dev D, StageArgs a, int xcd) {
    extern __shared__ __align__(16) unsigned char smem[];
    const InstParams &P = *D.ip;
    const Smem S = carve(smem, P, true);
    const uint32_t tile = a.tile0 + (xcd ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x);
    const TileRec TR = D.tiles[tile];
    process_tile<M, HAS64, HAS32, BASE, EXTRA, OUT64, TOP, CM>(P, D, TR, S, a, tile == 0, true, lut_words(P));
}

// Grid-wide barrier for the persistent kernel. Workgroup w publishes its
// arrival by a release store of `epoch` into its own flag slot (flags are 64
// bytes apart); every workgroup then polls all slots, one per thread, until
// each holds at least `epoch`. No read-modify-write is shared between
// workgroups. A bounded wait: after `limit` polling rounds the workgroup sets
// the timeout word and returns false, and every workgroup then leaves the
// kernel.
__device__ __forceinline__ bool grid_barrier(uint32_t *flags, uint32_t *timeout, uint32_t epoch, uint32_t limit) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    const uint32_t W = gridDim.x;
    if (threadIdx.x == 0)
        __hip_atomic_store(flags + 16u * blockIdx.x, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t polls = 0;  // counted by thread 0 only
    bool ok = true;
    while (true) {
        int mine = 1;
        for (uint32_t i = threadIdx.x; i < W; i += blockDim.x)
            mine &= __hip_atomic_load(flags + 16u * i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= epoch;
        int stop = 0;
        if (threadIdx.x == 0)
            stop = (__hip_atomic_load(timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) || (++polls > limit);
        // every thread reaches both workgroup reductions in every round
        const int all = __syncthreads_and(mine);
        const int any_stop = __syncthreads_or(stop);
        if (all) break;
        if (any_stop) {
            if (threadIdx.x == 0) __hip_atomic_store(timeout, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = false;
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok;
}

// The same grid barrier with arrival counters: every workgroup adds one to
// the counter of its group (G = min(8, workgroups) groups, workgroup w in group
// w % G; counters 64 bytes apart), the last arrival of a group adds one to the
// top counter, and one thread per workgroup polls the top counter until every
// group has arrived (epoch x G). Counters only grow within a launch (they are
// cleared before it), so epoch e is complete when the top counter reaches e G.
// Bounded like grid_barrier: a poller that gives up sets the timeout word.
__device__ __forceinline__ bool grid_barrier_ctr(uint32_t *ctrs, uint32_t *timeout, uint32_t epoch, uint32_t limit) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    const uint32_t W = gridDim.x, G = W < 8u ? W : 8u, g = blockIdx.x % G;
    const uint32_t gsize = W / G + (g < W % G ? 1u : 0u);
    int ok = 1;
    if (threadIdx.x == 0) {
        uint32_t *top = ctrs + 16u * 8u;
        const uint32_t old = __hip_atomic_fetch_add(ctrs + 16u * g, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1u == epoch * gsize) __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t polls = 0;
        while (__hip_atomic_load(top, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch * G) {
            if (__hip_atomic_load(timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || ++polls > limit) {
                __hip_atomic_store(timeout, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    ok = __syncthreads_and(ok);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok != 0;
}

struct PersistArgs {
    double2 *y;         // state (FP64), updated in place
    double2 *w0, *w1;   // FP64 stage vectors
    float2 *u1, *u2, *u3;  // FP32 increments
    double dt;
    int64_t step0;      // index of the first step of this launch (for observables)
    int64_t nsteps;
    int64_t obs_every;
    double *obs;
    uint32_t *flags;    // one 64-byte slot per workgroup
    uint32_t *timeout;  // set when a barrier gives up
    uint32_t limit;
    uint32_t policy;    // cache hints, as StageArgs::policy
};

// All RK4 steps of heom_propagate in one cooperative launch: every workgroup
// owns a fixed set of tiles (a contiguous run per XCD), processes its tiles
// for each of the four stages, and meets the grid at a barrier after each
// stage. A workgroup that owns a single tile keeps its metadata in LDS for the
// whole launch.
template <int M, int PREC, int BAR>
__global__ __launch_bounds__(MAX_TILE) void persistent_kernel(Dev D, PersistArgs pa) {
    extern __shared__ __align__(16) unsigned char smem[];
    const InstParams &P = *D.ip;
    const Smem S = carve(smem, P, false);
    const uint32_t T = P.n_tiles, W = gridDim.x, w = blockIdx.x;
    // tiles of this workgroup: XCD x = w % 8 owns tiles [x*T/8, (x+1)*T/8)
    const uint32_t X = W < 8 ? W : 8;
    const uint32_t x = w % X, j = w / X;
    const uint32_t wx = W / X + (x < W % X ? 1u : 0u);
    const uint32_t t_lo = (uint32_t)((uint64_t)x * T / X), t_hi = (uint32_t)((uint64_t)(x + 1) * T / X);
    const bool single = (t_hi - t_lo) <= wx;
    stage_lut(D, P, S.lut);
    TileRec TR0 = {};
    if (single && t_lo + j < t_hi) {
        TR0 = D.tiles[t_lo + j];
        stage_tile(D, TR0, S, 0u);
    }
    __syncthreads();
    const double h = pa.dt;
    const double al[4] = {h / 4.0, h / 3.0, h / 2.0, h};
    uint32_t epoch = 0;
    for (int64_t st = 1; st <= pa.nsteps; ++st) {
        const int64_t gst = pa.step0 + st;
        double *ob = (pa.obs != nullptr && pa.obs_every > 0 && gst % pa.obs_every == 0)
                         ? pa.obs + (gst / pa.obs_every) * HEOM_NOBS : nullptr;
        for (int s = 0; s < 4; ++s) {
            StageArgs a{};
            a.alpha = al[s];
            if (PREC == HEOM_FP64) {
                a.in64 = s == 0 ? pa.y : (s == 2 ? pa.w1 : pa.w0);
                a.ybase = pa.y;
                a.out64 = s == 3 ? pa.y : (s == 1 ? pa.w1 : pa.w0);
            } else {
                a.in64 = s == 0 ? pa.y : nullptr;
                a.in32 = s == 1 ? pa.u1 : (s == 2 ? pa.u2 : (s == 3 ? pa.u3 : nullptr));
                a.extra = pa.u1;
                a.extra_scale = 4.0 / h;
                a.ybase = pa.y;
                a.out32 = s == 0 ? pa.u1 : (s == 1 ? pa.u2 : pa.u3);
                a.out64 = pa.y;
            }
            a.obs = s == 3 ? ob : nullptr;
            a.policy = pa.policy;
            for (uint32_t tl = t_lo + j; tl < t_hi; tl += wx) {
                const TileRec TR = single ? TR0 : D.tiles[tl];
                const bool sd = !single;   // one tile per workgroup: staged once above
                if (PREC == HEOM_FP64) {
                    if (s == 0) process_tile<M, true, false, BASE_IN, false, true, false, 0>(P, D, TR, S, a, tl == 0, sd, 0u);
                    else process_tile<M, true, false, BASE_Y, false, true, false, 0>(P, D, TR, S, a, tl == 0, sd, 0u);
                } else {
                    if (s == 0) process_tile<M, true, false, BASE_NONE, false, false, false, 0>(P, D, TR, S, a, false, sd, 0u);
                    else if (s < 3) process_tile<M, false, true, BASE_NONE, true, false, false, 0>(P, D, TR, S, a, false, sd, 0u);
                    else process_tile<M, false, true, BASE_Y, true, true, false, 0>(P, D, TR, S, a, tl == 0, sd, 0u);
                }
            }
            epoch += 1;
            if (!(BAR ? grid_barrier_ctr(pa.flags, pa.timeout, epoch, pa.limit)
                      : grid_barrier(pa.flags, pa.timeout, epoch, pa.limit)))
                return;
        }
    }
}

// ---------------------------------------------------------------- batches

// A pointer read from memory has no known address space, so accesses
// through it would be flat instructions (which also hold up every LDS wait)
// and its uniform loads could not go through the scalar unit. Slot records
// only ever hold global-memory addresses: say so.
template <class T>
__device__ __forceinline__ T *as_global(T *p) {
    return (T *)(reinterpret_cast<__attribute__((address_space(1))) T *>(reinterpret_cast<uintptr_t>(p)));
}

// One RK4 stage of every tile of every slot in a tile list (all of one m).
// Each variable is computed by the same arithmetic as in stage_kernel, so a
// problem's trajectory does not depend on the other problems in the batch.
// SV selects the stage's vector pattern at compile time (FP64: 0 = first
// stage, 1 = the others; FP32: 0 = first, 1 = second and third, 2 = last),
// so each instance holds only the registers of its own pattern.
// Everything a workgroup of a batch launch needs about its tile's slot.
struct BatchCtx {
    SlotRec R;
    Dev D;
    TileRec TR;
    StageArgs a;
    bool first;
};

template <int PREC>
__device__ __forceinline__ BatchCtx batch_ctx(const SlotRec &rec, uint32_t tile, int s, int64_t *ctr,
                                              uint32_t policy) {
    BatchCtx c;
    SlotRec &R = c.R;
    R = rec;
    R.img = as_global(R.img);
    R.params = as_global(R.params);
    R.hdr = as_global(R.hdr);
    R.cat = as_global(R.cat);
    R.gidx = as_global(R.gidx);
    R.tiles = as_global(R.tiles);
    R.vrec = as_global(R.vrec);
    R.lut = as_global(R.lut);
    R.y = as_global(R.y);
    R.w0 = as_global(R.w0);
    R.w1 = as_global(R.w1);
    R.u1 = as_global(R.u1);
    R.u2 = as_global(R.u2);
    R.u3 = as_global(R.u3);
    R.yT = as_global(R.yT);
    R.w0T = as_global(R.w0T);
    R.w1T = as_global(R.w1T);
    R.u1T = as_global(R.u1T);
    R.u2T = as_global(R.u2T);
    R.u3T = as_global(R.u3T);
    R.obs = as_global(R.obs);
    const InstParams &P = *reinterpret_cast<const InstParams *>(R.params);
    Dev &D = c.D;
    D.ip = &P;
    D.lut = R.lut;
    D.hdr = R.hdr;
    D.cat = R.cat;
    D.gidx = R.gidx;
    D.tiles = R.tiles;
    D.vrec = R.vrec;
    c.TR = D.tiles[tile];
    const double h = R.dt;
    // Steps of this slot so far, this one included, for the observable row
    // of the last stage. The counter (steps of the batch since the last
    // commit, this one included) is advanced on the device by the first
    // launch of each step's first stage, so a captured graph of steps
    // replays with the right rows; only the last stage reads it.
    const int64_t gst = s == 3 ? R.step0 + *as_global(ctr) : 0;
    StageArgs &a = c.a;
    a = StageArgs{};
    // mirrored column gathers need transposed column targets; with them the
    // slot neither reads nor writes copies
    const bool mirror = (policy & 8u) && P.tcol != 0;
    a.policy = mirror ? policy : (policy & ~8u);
    if (mirror) R.yT = R.w0T = R.w1T = nullptr, R.u1T = R.u2T = R.u3T = nullptr;
    a.alpha = s == 0 ? h / 4.0 : (s == 1 ? h / 3.0 : (s == 2 ? h / 2.0 : h));
    a.obs = (s == 3 && R.obs != nullptr && R.obs_every > 0 && gst % R.obs_every == 0 && gst / R.obs_every < R.obs_cap)
                ? R.obs + (gst / R.obs_every) * HEOM_NOBS : nullptr;
    c.first = tile == 0;
    if (PREC == HEOM_FP64) {
        a.in64 = s == 0 ? R.y : (s == 2 ? R.w1 : R.w0);
        a.inT64 = s == 0 ? R.yT : (s == 2 ? R.w1T : R.w0T);
        a.ybase = R.y;
        a.out64 = s == 3 ? R.y : (s == 1 ? R.w1 : R.w0);
        a.outT64 = s == 3 ? R.yT : (s == 1 ? R.w1T : R.w0T);
    } else {
        a.in64 = R.y;
        a.inT64 = R.yT;
        a.in32 = s == 1 ? R.u1 : (s == 2 ? R.u2 : R.u3);
        a.inT32 = s == 1 ? R.u1T : (s == 2 ? R.u2T : R.u3T);
        a.extra = R.u1;
        a.extra_scale = 4.0 / h;
        a.ybase = R.y;
        a.out32 = s == 0 ? R.u1 : (s == 1 ? R.u2 : R.u3);
        a.outT32 = s == 0 ? R.u1T : (s == 1 ? R.u2T : R.u3T);
        a.out64 = R.y;
        a.outT64 = R.yT;
    }
    return c;
}

// The stage pattern SV of one tile (FP64: 0 = first stage, 1 = the others;
// FP32: 0 = first, 1 = second and third, 2 = last).
// CM: 2 = the tile kind read from each slot's parameter block, 1 = every
// slot of the launch has compact tiles (the registers of the compact-only
// code, as in stage_kernel).
template <int M, int PREC, bool TOP, int SV, int CM = 2>
__device__ __forceinline__ void batch_tile(const BatchCtx &c, unsigned char *smem, int stage = STAGE_ALL) {
    const InstParams &P = *c.D.ip;
    const Smem S = carve(smem, P, true);
    const uint32_t lw = lut_words(P);
    if (PREC == HEOM_FP64) {
        if (SV == 0) process_tile<M, true, false, BASE_IN, false, true, TOP, CM>(P, c.D, c.TR, S, c.a, c.first, stage, lw);
        else process_tile<M, true, false, BASE_Y, false, true, TOP, CM>(P, c.D, c.TR, S, c.a, c.first, stage, lw);
    } else {
        if (SV == 0) process_tile<M, true, false, BASE_NONE, false, false, TOP, CM>(P, c.D, c.TR, S, c.a, false, stage, lw);
        else if (SV == 1) process_tile<M, false, true, BASE_NONE, true, false, TOP, CM>(P, c.D, c.TR, S, c.a, false, stage, lw);
        else process_tile<M, false, true, BASE_Y, true, true, TOP, CM>(P, c.D, c.TR, S, c.a, c.first, stage, lw);
    }
}

// The first launch of a step's first stage advances the batch's step counter
// (one thread, last thing in the kernel: a store ahead of the record loads
// would keep the compiler from proving them unclobbered and moving them to
// the scalar unit).
__device__ __forceinline__ void advance_counter(int64_t *ctr, uint32_t advance) {
    if (advance && blockIdx.x == 0 && threadIdx.x == 0) *as_global(ctr) += 1;
}

// One RK4 stage of every tile of every slot in a tile list (all of one m,
// one tile size and one tier class). Each variable is computed by the same
// arithmetic as in stage_kernel, so a problem's trajectory does not depend
// on the other problems in the batch. SV is a template parameter, so each
// instance holds only the registers of its own stage pattern.
template <int M, int PREC, bool TOP, int SV, int CM>
__global__ __launch_bounds__(MAX_TILE) void batch_stage_kernel(const SlotRec *slots, const BatchTile *btiles, int s,
                                                             int64_t *ctr, uint32_t policy, uint32_t advance) {
    extern __shared__ __align__(16) unsigned char smem[];
    const BatchTile B = btiles[blockIdx.x];
    const BatchCtx c = batch_ctx<PREC>(slots[B.slot], B.tile & ~BTILE_TOP, s, ctr, policy);
    batch_tile<M, PREC, TOP, SV, CM>(c, smem);
    advance_counter(ctr, advance);
}

// The tiles tile0.. of one slot, whose record comes in the kernel arguments
// (as a state's tables do for stage_kernel): no list or record lookups
// before the first loads. For slots large enough to fill launches alone.
template <int M, int PREC, bool TOP, int SV, int CM>
__global__ __launch_bounds__(MAX_TILE) void batch_stage_single(SlotRec R, uint32_t tile0, int s, int64_t *ctr,
                                                             uint32_t policy, uint32_t advance) {
    extern __shared__ __align__(16) unsigned char smem[];
    const BatchCtx c = batch_ctx<PREC>(R, tile0 + blockIdx.x, s, ctr, policy);
    batch_tile<M, PREC, TOP, SV, CM>(c, smem);
    advance_counter(ctr, advance);
}

// One tile of one structure for two problems that share that structure
// (their slots use the same uploaded image, each with its own parameter
// block), side by side: the block has twice the tile's threads, each half
// computes the tile for one problem, and the tile's metadata is staged into
// LDS once for both (N-independence of the tables beyond saturation, Sec.
// V.C.4). lists[B.slot] = 2, followed by the two slot indices. Every thread
// runs the same code as in a one-problem workgroup (same registers); every
// variable is computed as in stage_kernel.
template <int M, int PREC, bool TOP, int SV>
__global__ __launch_bounds__(MAX_TILE) void batch_stage_pair(const SlotRec *slots, const BatchTile *btiles,
                                                           const uint32_t *lists, int s, int64_t *ctr,
                                                           uint32_t policy, uint32_t advance) {
    extern __shared__ __align__(16) unsigned char smem[];
    const BatchTile B = btiles[blockIdx.x];
    const uint32_t tv = blockDim.x / 2u;
    // each wave lies in one half (tv is a multiple of the wave size)
    const uint32_t half = __builtin_amdgcn_readfirstlane(threadIdx.x / tv);
    const uint32_t slot = __builtin_amdgcn_readfirstlane(lists[B.slot + 1u + half]);
    const BatchCtx c = batch_ctx<PREC>(slots[slot], B.tile & ~BTILE_TOP, s, ctr, policy);
    const InstParams &P = *c.D.ip;
    const Smem S = carve_pair(smem, P, half);
    const uint32_t lw = lut_words(P), tb = half * tv;
    if (PREC == HEOM_FP64) {
        if (SV == 0) process_tile<M, true, false, BASE_IN, false, true, TOP, 2>(P, c.D, c.TR, S, c.a, c.first, STAGE_PAIR, lw, tb, tv);
        else process_tile<M, true, false, BASE_Y, false, true, TOP, 2>(P, c.D, c.TR, S, c.a, c.first, STAGE_PAIR, lw, tb, tv);
    } else {
        if (SV == 0) process_tile<M, true, false, BASE_NONE, false, false, TOP, 2>(P, c.D, c.TR, S, c.a, false, STAGE_PAIR, lw, tb, tv);
        else if (SV == 1) process_tile<M, false, true, BASE_NONE, true, false, TOP, 2>(P, c.D, c.TR, S, c.a, false, STAGE_PAIR, lw, tb, tv);
        else process_tile<M, false, true, BASE_Y, true, true, TOP, 2>(P, c.D, c.TR, S, c.a, c.first, STAGE_PAIR, lw, tb, tv);
    }
    advance_counter(ctr, advance);
}

// The same for a whole batch in one launch per stage, for batches of small
// problems whose stages are bound by launch latency: each workgroup takes the
// kernel variant of its slot's m (at most MERGE_MAX_M) and tier class. The
// block has the largest tile size of the batch (threads past a tile's last
// variable only help stage its metadata).
constexpr int MERGE_MAX_M = 4;
template <int PREC, int SV>
__global__ __launch_bounds__(MAX_TILE) void batch_stage_merged(const SlotRec *slots, const BatchTile *btiles, int s,
                                                             int64_t *ctr, uint32_t policy, uint32_t advance) {
    extern __shared__ __align__(16) unsigned char smem[];
    const BatchTile B = btiles[blockIdx.x];
    const bool top = (B.tile & BTILE_TOP) != 0;
    const BatchCtx c = batch_ctx<PREC>(slots[B.slot], B.tile & ~BTILE_TOP, s, ctr, policy);
    switch (c.D.ip->m * 2 + (top ? 1 : 0)) {
        case 2: batch_tile<1, PREC, false, SV>(c, smem); break;
        case 3: batch_tile<1, PREC, true, SV>(c, smem); break;
        case 4: batch_tile<2, PREC, false, SV>(c, smem); break;
        case 5: batch_tile<2, PREC, true, SV>(c, smem); break;
        case 6: batch_tile<3, PREC, false, SV>(c, smem); break;
        case 7: batch_tile<3, PREC, true, SV>(c, smem); break;
        case 8: batch_tile<4, PREC, false, SV>(c, smem); break;
        case 9: batch_tile<4, PREC, true, SV>(c, smem); break;
        default: break;   // excluded when the batch is committed
    }
    advance_counter(ctr, advance);
}

__global__ void observables_kernel(Dev D, const double2 *y, double *obs) {
    __shared__ double2 v[MAX_TILE];
    const uint32_t n0 = D.hdr[0].size;
    for (uint32_t i = threadIdx.x; i < n0; i += blockDim.x) v[i] = y[i];
    __syncthreads();
    if (threadIdx.x == 0) tier0_observables(*D.ip, D.hdr[0], D.cat, v, obs);
}

// Non-finite check at the end of a propagation: the tier-0 block of y (the
// observables' input) and the observable rows the call wrote. Any thread that
// sees a NaN or an infinity makes thread 0 set *flag.
__global__ void finite_check_kernel(const double *y0, uint32_t n_y0, const double *obs, uint32_t n_obs,
                                    uint32_t *flag) {
    int bad = 0;
    for (uint32_t i = threadIdx.x; i < n_y0; i += blockDim.x) bad |= !__builtin_isfinite(y0[i]);
    for (uint32_t i = threadIdx.x; i < n_obs; i += blockDim.x) bad |= !__builtin_isfinite(obs[i]);
    if (__syncthreads_or(bad) && threadIdx.x == 0) *flag = 1u;
}

// The same for every occupied slot of a batch (one workgroup per slot): the
// tier-0 block of the slot's state; flags[slot] is set if it is not finite.
__global__ void batch_finite_kernel(const SlotRec *slots, uint32_t *flags) {
    const SlotRec R = slots[blockIdx.x];
    if (R.y == nullptr) return;            // an empty slot: the whole workgroup leaves
    const uint32_t n = 2u * as_global(R.hdr)[0].size;
    const double *y0 = reinterpret_cast<const double *>(as_global(R.y));
    int bad = 0;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) bad |= !__builtin_isfinite(y0[i]);
    if (__syncthreads_or(bad) && threadIdx.x == 0) flags[blockIdx.x] = 1u;
}

// Advance a batch's device step counter by n (steps taken without the
// batch kernels, which otherwise advance it themselves).
__global__ void counter_add_kernel(int64_t *ctr, int64_t n) {
    if (threadIdx.x == 0) *ctr += n;
}

__global__ void zero_kernel(double2 *y, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        y[i] = make_double2(0.0, 0.0);
}

// yT = y with every block's category matrix transposed (T_q in place); one
// workgroup per tile, one thread per variable (complex FP64 or FP32 values).
template <class V>
__global__ void transpose_kernel(const TileRec *tiles, const VarRec *vrec, const PatHdr *hdr, const V *y, V *yT) {
    const TileRec TR = tiles[blockIdx.x];
    const uint32_t t = threadIdx.x;
    if (t >= TR.nv) return;
    const VarRec vr = vrec[TR.v0 + t];
    const uint32_t p = vr.x & 127u, A = (vr.x >> 7) & 31u, B = (vr.x >> 12) & 31u;
    const bool isT = (vr.x >> 17) & 1u;
    const PatHdr H = hdr[TR.p0 + p];
    const uint32_t base = H.off - TR.v0, G1 = (uint32_t)H.G + 1u;
    yT[TR.v0 + (isT ? t : base + B * G1 + A)] = y[TR.v0 + t];
}

// States of at least this many tiles run their top tier as a second launch
// with the kernel variant that has no up moves (fewer registers, more waves);
// for smaller ones the extra launch costs more than it saves.
constexpr uint32_t TOP_SPLIT_TILES = 2048;

template <int M, bool HAS64, bool HAS32, int BASE, bool EXTRA, bool OUT64>
void launch_m(const HostTables &t, const Dev &D, hipStream_t s, StageArgs a) {
    a.policy = (uint32_t)t.tune.cache_policy | (a.policy & 8u);
    const uint32_t T = (uint32_t)t.tiles.size();
    // Large states: the top tier (no up moves) runs in its own launch with a
    // kernel that has no up-move slots, fewer registers and more waves.
    const uint32_t split = (T >= TOP_SPLIT_TILES && t.top_tile > 0 && t.top_tile < T) ? t.top_tile : T;
    a.tile0 = 0;
    // compact tiles (Hermitian ADOs) have kernels of their own
    if (t.compact) {
        hipLaunchKernelGGL((stage_kernel<M, HAS64, HAS32, BASE, EXTRA, OUT64, false, 1>), dim3(split),
                           dim3(t.tile_vars), split < T ? t.lds_low : t.lds_bytes, s, D, a,
                           t.tune.xcd_map);
        if (split < T) {
            a.tile0 = split;
            hipLaunchKernelGGL((stage_kernel<M, HAS64, HAS32, BASE, EXTRA, OUT64, true, 1>), dim3(T - split),
                               dim3(t.tile_vars), t.lds_top, s, D, a, t.tune.xcd_map);
        }
        return;
    }
    hipLaunchKernelGGL((stage_kernel<M, HAS64, HAS32, BASE, EXTRA, OUT64, false, 0>), dim3(split),
                       dim3(t.tile_vars), split < T ? t.lds_low : t.lds_bytes, s, D, a, t.tune.xcd_map);
    if (split < T) {
        a.tile0 = split;
        hipLaunchKernelGGL((stage_kernel<M, HAS64, HAS32, BASE, EXTRA, OUT64, true, 0>), dim3(T - split),
                           dim3(t.tile_vars), t.lds_top, s, D, a, t.tune.xcd_map);
    }
}

// One RK4 stage of one state; D = the tables' device view, or one whose
// parameter block is another problem's of the same structure (a batch slot).
template <bool HAS64, bool HAS32, int BASE, bool EXTRA, bool OUT64>
int launch_stage(const HostTables &t, hipStream_t s, const StageArgs &a, const Dev *D = nullptr) {
    const Dev Dv = D ? *D : dev_view(t);
#define HEOM_CASE(MM) \
    case MM: launch_m<MM, HAS64, HAS32, BASE, EXTRA, OUT64>(t, Dv, s, a); break;
    switch (t.m) {
        HEOM_CASE(1) HEOM_CASE(2) HEOM_CASE(3) HEOM_CASE(4)
        HEOM_CASE(5) HEOM_CASE(6) HEOM_CASE(7) HEOM_CASE(8)
        default: return fail(HEOM_E_UNSUPPORTED, "m out of range");
    }
#undef HEOM_CASE
    HIP_TRY(hipGetLastError());
    return HEOM_OK;
}

__global__ void zero_u32_kernel(uint32_t *p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// Control area of the work buffer, after the state-sized vectors:
//   byte 4: barrier timeout word; byte 8: non-finite flag of the last
//   propagation; bytes 256..: one 64-byte flag slot per persistent workgroup.
constexpr uint32_t MAX_PERSIST_WG = 2048;
constexpr size_t CTRL_BYTES = 256 + 64 * (size_t)MAX_PERSIST_WG;

// Work buffer: the stage vectors (32 bytes per variable; 80 with transposed
// copies), then the control area.
//   FP64: w0 [0, 16n), w1 [16n, 32n); copies yT [32n, 48n), w0T [48n, 64n),
//         w1T [64n, 80n)
//   FP32: u3 [0, 8n), u1 [16n, 24n), u2 [24n, 32n); copies yT [32n, 48n),
//         u1T [48n, 56n), u2T [56n, 64n), u3T [64n, 72n)
struct WorkView {
    double2 *w0, *w1, *yT, *w0T, *w1T;
    float2 *u1, *u2, *u3, *u1T, *u2T, *u3T;
    unsigned char *ctrl;
};
// transposed copies exist for tables with transposed column targets that are
// not compact (compact tables serve Hermitian ADOs only, which need none)
bool has_copies(const HostTables &t) { return t.trcol && !t.compact; }
size_t vec_bytes(const HostTables &t) { return (size_t)t.n_var * (has_copies(t) ? 80 : 32); }
WorkView work_view(const HostTables &t, void *work) {
    const size_t n = t.n_var;
    unsigned char *wb = static_cast<unsigned char *>(work);
    WorkView w{};
    w.w0 = reinterpret_cast<double2 *>(wb);
    w.w1 = w.w0 + n;
    w.u3 = reinterpret_cast<float2 *>(wb);
    w.u1 = reinterpret_cast<float2 *>(wb + 16 * n);
    w.u2 = w.u1 + n;
    if (has_copies(t)) {
        w.yT = reinterpret_cast<double2 *>(wb + 32 * n);
        w.w0T = w.yT + n;
        w.w1T = w.w0T + n;
        w.u1T = reinterpret_cast<float2 *>(wb + 48 * n);
        w.u2T = w.u1T + n;
        w.u3T = w.u2T + n;
    }
    w.ctrl = wb + vec_bytes(t);
    return w;
}

template <class V>
int launch_transpose(const HostTables &t, hipStream_t s, const V *y, V *yT) {
    const Dev D = dev_view(t);
    hipLaunchKernelGGL(transpose_kernel<V>, dim3((uint32_t)t.tiles.size()), dim3(t.tile_vars), 0, s, D.tiles, D.vrec,
                       D.hdr, y, yT);
    HIP_TRY(hipGetLastError());
    return HEOM_OK;
}

template <int M, int PREC>
int launch_persistent_m(const HostTables &t, hipStream_t s, PersistArgs pa, bool *used) {
    auto kern = t.tune.persistent == 3 ? persistent_kernel<M, PREC, 1> : persistent_kernel<M, PREC, 0>;
    int dev = 0, ncu = 0, per_cu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, t.tile_vars, t.lds_persist));
    if (per_cu < 1) { *used = false; return HEOM_OK; }
    uint64_t nwg = std::min<uint64_t>((uint64_t)per_cu * (uint64_t)ncu, t.tiles.size());
    nwg = std::min<uint64_t>(nwg, MAX_PERSIST_WG);
    if (t.tune.max_workgroups > 0) nwg = std::min<uint64_t>(nwg, (uint64_t)t.tune.max_workgroups);
    // barrier epochs (4 per step) and the arrival counters (epoch x group
    // size, at most 256) must not wrap within one launch
    const int64_t chunk = (int64_t)1 << 22;
    const int64_t total = pa.nsteps;
    Dev D = dev_view(t);
    for (int64_t done = 0; done < total; done += chunk) {
        PersistArgs a = pa;
        a.step0 = pa.step0 + done;
        a.nsteps = std::min<int64_t>(chunk, total - done);
        hipLaunchKernelGGL(zero_u32_kernel, dim3(64), dim3(256), 0, s, pa.flags - 64, (uint32_t)(CTRL_BYTES / 4));
        HIP_TRY(hipGetLastError());
        void *args[] = {&D, &a};
        HIP_TRY(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kern), dim3((uint32_t)nwg),
                                           dim3(t.tile_vars), args, t.lds_persist, s));
    }
    *used = true;
    return HEOM_OK;
}

int launch_persistent(const HostTables &t, hipStream_t s, const PersistArgs &pa, int prec, bool *used) {
    if (t.trcol) { *used = false; return HEOM_OK; }   // the persistent kernel keeps no transposed copies
#define HEOM_PCASE(MM) \
    case MM: return prec == HEOM_FP64 ? launch_persistent_m<MM, HEOM_FP64>(t, s, pa, used) \
                                      : launch_persistent_m<MM, HEOM_FP32>(t, s, pa, used);
    switch (t.m) {
        HEOM_PCASE(1) HEOM_PCASE(2) HEOM_PCASE(3) HEOM_PCASE(4)
        HEOM_PCASE(5) HEOM_PCASE(6) HEOM_PCASE(7) HEOM_PCASE(8)
        default: return fail(HEOM_E_UNSUPPORTED, "m out of range");
    }
#undef HEOM_PCASE
}

size_t work_bytes_for(const HostTables &t) { return vec_bytes(t) + CTRL_BYTES; }
size_t rhs_work_bytes_for(const HostTables &t) { return has_copies(t) ? (size_t)t.n_var * 16 : 0; }

// c_check_k = conj(c_k) for every channel: the condition under which the
// propagation maps Hermitian ADOs to Hermitian ADOs (Eq. adjoint-preservation).
bool adjoint_preserving(const HostTables &t) {
    for (int k = 0; k < t.m; ++k)
        if (t.cc[2 * k] != t.c[2 * k] || t.cc[2 * k + 1] != -t.c[2 * k + 1]) return false;
    return true;
}

bool adjoint_preserving(const heom_problem &p) {
    if (!p.c_check) return true;
    for (int k = 0; k < p.m; ++k)
        if (p.c_check[2 * k] != p.c[2 * k] || p.c_check[2 * k + 1] != -p.c[2 * k + 1]) return false;
    return true;
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

// One-slot-per-workgroup launch of a group: the group's only slot
// (batch_stage_single) or its tile list (batch_stage_kernel).
template <int M, int PREC, bool TOP, int CM>
void batch_launch_plain(const heom_batch *b, const heom_batch::Group &g, hipStream_t s, const SlotRec *recs,
                        const BatchTile *first, int stage, int sv, int64_t *ctr, uint32_t policy, uint32_t advance) {
    const dim3 grid(g.count), block(g.block);
    if (g.slot >= 0) {
        const SlotRec &R = b->recs[(size_t)g.slot];
        const uint32_t tile0 = g.tile0;
        if (sv == 0)
            hipLaunchKernelGGL((batch_stage_single<M, PREC, TOP, 0, CM>), grid, block, g.lds, s, R, tile0, stage, ctr,
                               policy, advance);
        else if (sv == 1)
            hipLaunchKernelGGL((batch_stage_single<M, PREC, TOP, 1, CM>), grid, block, g.lds, s, R, tile0, stage, ctr,
                               policy, advance);
        else if (PREC == HEOM_FP32)
            hipLaunchKernelGGL((batch_stage_single<M, PREC, TOP, 2, CM>), grid, block, g.lds, s, R, tile0, stage, ctr,
                               policy, advance);
        return;
    }
    if (sv == 0)
        hipLaunchKernelGGL((batch_stage_kernel<M, PREC, TOP, 0, CM>), grid, block, g.lds, s, recs, first, stage, ctr,
                           policy, advance);
    else if (sv == 1)
        hipLaunchKernelGGL((batch_stage_kernel<M, PREC, TOP, 1, CM>), grid, block, g.lds, s, recs, first, stage, ctr,
                           policy, advance);
    else if (PREC == HEOM_FP32)
        hipLaunchKernelGGL((batch_stage_kernel<M, PREC, TOP, 2, CM>), grid, block, g.lds, s, recs, first, stage, ctr,
                           policy, advance);
}

template <int M, int PREC, bool TOP>
void batch_launch_group(const heom_batch *b, const heom_batch::Group &g, hipStream_t s, const SlotRec *recs,
                        const BatchTile *first, int stage, int64_t *ctr, uint32_t policy, uint32_t advance) {
    const dim3 grid(g.count), block(g.shared ? 2u * g.block : g.block);
    const int sv = stage == 0 ? 0 : (PREC == HEOM_FP64 ? 1 : (stage < 3 ? 1 : 2));
    if (g.shared) {
        const uint32_t *lists = reinterpret_cast<const uint32_t *>(static_cast<const unsigned char *>(b->dev) +
                                                                   b->list_off);
        if (sv == 0)
            hipLaunchKernelGGL((batch_stage_pair<M, PREC, TOP, 0>), grid, block, g.lds, s, recs, first, lists, stage,
                               ctr, policy, advance);
        else if (sv == 1)
            hipLaunchKernelGGL((batch_stage_pair<M, PREC, TOP, 1>), grid, block, g.lds, s, recs, first, lists, stage,
                               ctr, policy, advance);
        else if (PREC == HEOM_FP32)
            hipLaunchKernelGGL((batch_stage_pair<M, PREC, TOP, 2>), grid, block, g.lds, s, recs, first, lists, stage,
                               ctr, policy, advance);
        return;
    }
    if (g.compact) batch_launch_plain<M, PREC, TOP, 1>(b, g, s, recs, first, stage, sv, ctr, policy, advance);
    else batch_launch_plain<M, PREC, TOP, 2>(b, g, s, recs, first, stage, sv, ctr, policy, advance);
}


template <int PREC>
int batch_launch(const heom_batch *b, hipStream_t s, int stage, uint32_t policy) {
    const SlotRec *recs = static_cast<const SlotRec *>(b->dev);
    const size_t tile_off = (sizeof(SlotRec) * b->slots.size() + 255) & ~(size_t)255;
    const BatchTile *tl = reinterpret_cast<const BatchTile *>(static_cast<const unsigned char *>(b->dev) + tile_off);
    int64_t *ctr = reinterpret_cast<int64_t *>(static_cast<unsigned char *>(b->dev) + b->ctr_off);
    uint32_t advance = stage == 0 ? 1u : 0u;   // the step's first launch advances the counter
    for (const auto &g : b->groups) {
        const BatchTile *first = tl + g.first;
        if (g.m == 0) {
            const dim3 grid(g.count), block(g.block);
            const int sv = stage == 0 ? 0 : (PREC == HEOM_FP64 ? 1 : (stage < 3 ? 1 : 2));
            if (sv == 0)
                hipLaunchKernelGGL((batch_stage_merged<PREC, 0>), grid, block, g.lds, s, recs, first, stage, ctr, policy, advance);
            else if (sv == 1)
                hipLaunchKernelGGL((batch_stage_merged<PREC, 1>), grid, block, g.lds, s, recs, first, stage, ctr, policy, advance);
            else if (PREC == HEOM_FP32)
                hipLaunchKernelGGL((batch_stage_merged<PREC, 2>), grid, block, g.lds, s, recs, first, stage, ctr, policy, advance);
            HIP_TRY(hipGetLastError());
            advance = 0u;
            continue;
        }
#define HEOM_BCASE(MM)                                                                         \
    case MM:                                                                                   \
        if (g.top) batch_launch_group<MM, PREC, true>(b, g, s, recs, first, stage, ctr, policy, advance);  \
        else batch_launch_group<MM, PREC, false>(b, g, s, recs, first, stage, ctr, policy, advance);       \
        break;
        switch (g.m) {
            HEOM_BCASE(1) HEOM_BCASE(2) HEOM_BCASE(3) HEOM_BCASE(4)
            HEOM_BCASE(5) HEOM_BCASE(6) HEOM_BCASE(7) HEOM_BCASE(8)
            default: return fail(HEOM_E_UNSUPPORTED, "m out of range");
        }
#undef HEOM_BCASE
        HIP_TRY(hipGetLastError());
        advance = 0u;
    }
    return HEOM_OK;
}

// One RK4 step of every slot: four stage launches per group.
int batch_step(const heom_batch *b, hipStream_t s, int precision) {
    // bit 3: Hermitian ADOs (slots with transposed tables read mirrored entries)
    const uint32_t policy = 6u | ((precision & HEOM_HERMITIAN) ? 8u : 0u);
    precision &= ~HEOM_HERMITIAN;
    for (int stage = 0; stage < 4; ++stage) {
        const int rc = precision == HEOM_FP64 ? batch_launch<HEOM_FP64>(b, s, stage, policy)
                                              : batch_launch<HEOM_FP32>(b, s, stage, policy);
        if (rc) return rc;
    }
    return HEOM_OK;
}

// Capture graph_steps steps on stream s into b->gexec. The capture is ended
// on every path, so the stream never stays in capture mode.
int batch_capture(heom_batch *b, hipStream_t s, int precision) {
    if (b->gexec) {
        HIP_TRY(hipGraphExecDestroy(b->gexec));
        b->gexec = nullptr;
    }
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    int rc = HEOM_OK;
    for (int32_t k = 0; k < b->graph_steps && rc == HEOM_OK; ++k) rc = batch_step(b, s, precision);
    const std::string launch_err = rc ? g_err : std::string();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return fail(rc, launch_err);
    }
    if (e != hipSuccess) return fail(HEOM_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
        b->gexec = nullptr;
        return fail(HEOM_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    b->gprec = precision;
    return HEOM_OK;
}

// heom_propagate without the persistent kernel: one launch per RK4 stage.
// Observable rows: row j holds the state after j*obs_every steps counted
// from step0 (the steps taken before this call), for rows below obs_cap.
// D: the device view (the tables' own, or a batch slot's).
int propagate_stages(const HostTables &t, hipStream_t s, double2 *y, const WorkView &wv, const PersistArgs &pa,
                     int precision, bool hermitian, double dt, int64_t nsteps, int64_t obs_every, double *obs_dev,
                     const Dev *D = nullptr, int64_t step0 = 0, int64_t obs_cap = INT64_MAX) {
    // one launch per stage; with transposed copies, y's copy is made once
    // here and each stage then writes the copy of its own output. Hermitian
    // ADOs need no copies: column gathers read the mirrored entry.
    const double h1 = dt / 4.0, h2 = dt / 3.0, h3 = dt / 2.0, h4 = dt;
    int rc;
    const bool mirror = hermitian && t.trcol;
    WorkView cv = wv;                       // the copies, or none
    if (mirror) cv.yT = cv.w0T = cv.w1T = nullptr, cv.u1T = cv.u2T = cv.u3T = nullptr;
    const uint32_t pol = mirror ? 8u : 0u;
    if (t.trcol && !mirror && (rc = launch_transpose(t, s, y, wv.yT))) return rc;
    if (precision == HEOM_FP64) {
        double2 *wa = pa.w0, *wbv = pa.w1, *waT = cv.w0T, *wbT = cv.w1T;
        for (int64_t st = 1; st <= nsteps; ++st) {
            const int64_t gs = step0 + st;
            double *ob = (obs_every > 0 && gs % obs_every == 0 && gs / obs_every < obs_cap)
                             ? obs_dev + (gs / obs_every) * HEOM_NOBS : nullptr;
            StageArgs a{};
            a.policy = pol;
            a.in64 = y; a.inT64 = cv.yT; a.out64 = wa; a.outT64 = waT; a.alpha = h1;
            if ((rc = launch_stage<true, false, BASE_IN, false, true>(t, s, a, D))) return rc;
            a = StageArgs{}; a.policy = pol;
            a.in64 = wa; a.inT64 = waT; a.ybase = y; a.out64 = wbv; a.outT64 = wbT; a.alpha = h2;
            if ((rc = launch_stage<true, false, BASE_Y, false, true>(t, s, a, D))) return rc;
            a = StageArgs{}; a.policy = pol;
            a.in64 = wbv; a.inT64 = wbT; a.ybase = y; a.out64 = wa; a.outT64 = waT; a.alpha = h3;
            if ((rc = launch_stage<true, false, BASE_Y, false, true>(t, s, a, D))) return rc;
            a = StageArgs{}; a.policy = pol;
            a.in64 = wa; a.inT64 = waT; a.ybase = y; a.out64 = y; a.outT64 = cv.yT; a.alpha = h4;
            a.obs = ob;
            if ((rc = launch_stage<true, false, BASE_Y, false, true>(t, s, a, D))) return rc;
        }
    } else {
        // u1 = h/4 M y, u2 = h/3 M (y + u1), u3 = h/2 M (y + u2) and
        // y += h M (y + u3), each from the FP32 increment it gathers plus
        // M y = (4/h) u1; the state is updated in place by its owner.
        float2 *u1 = pa.u1, *u2 = pa.u2, *u3 = pa.u3;
        const double inv_h1 = 1.0 / h1;
        for (int64_t st = 1; st <= nsteps; ++st) {
            const int64_t gs = step0 + st;
            double *ob = (obs_every > 0 && gs % obs_every == 0 && gs / obs_every < obs_cap)
                             ? obs_dev + (gs / obs_every) * HEOM_NOBS : nullptr;
            StageArgs a{};
            a.policy = pol;
            a.in64 = y; a.inT64 = cv.yT; a.out32 = u1; a.outT32 = cv.u1T; a.alpha = h1;
            if ((rc = launch_stage<true, false, BASE_NONE, false, false>(t, s, a, D))) return rc;
            a = StageArgs{}; a.policy = pol;
            a.in32 = u1; a.inT32 = cv.u1T; a.extra = u1; a.extra_scale = inv_h1; a.out32 = u2;
            a.outT32 = cv.u2T; a.alpha = h2;
            if ((rc = launch_stage<false, true, BASE_NONE, true, false>(t, s, a, D))) return rc;
            a = StageArgs{}; a.policy = pol;
            a.in32 = u2; a.inT32 = cv.u2T; a.extra = u1; a.extra_scale = inv_h1; a.out32 = u3;
            a.outT32 = cv.u3T; a.alpha = h3;
            if ((rc = launch_stage<false, true, BASE_NONE, true, false>(t, s, a, D))) return rc;
            a = StageArgs{}; a.policy = pol;
            a.in32 = u3; a.inT32 = cv.u3T; a.extra = u1; a.extra_scale = inv_h1; a.ybase = y;
            a.out64 = y; a.outT64 = cv.yT; a.alpha = h4; a.obs = ob;
            if ((rc = launch_stage<false, true, BASE_Y, true, true>(t, s, a, D))) return rc;
        }
    }
    return HEOM_OK;
}

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

int scratch_address(void **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(HEOM_E_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(HEOM_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HEOM_OK;
}

// heom_propagate on a given work buffer (the caller's, or the library's
// static scratch array for heom_propagate_noalloc).
int propagate_impl(const heom_tables *h, void *y_dev, void *work_dev, size_t work_bytes, double dt, int64_t nsteps,
                   int64_t obs_every, double *obs_dev, int precision, void *stream) {
    if (int rc = check_ready(h)) return rc;
    if (int rc = check_dev(y_dev, "y_dev")) return rc;
    if (int rc = check_dev(work_dev, "work_dev")) return rc;
    if (!(std::isfinite(dt)) || nsteps < 0 || obs_every < 0) return fail(HEOM_E_INVAL, "bad dt, nsteps or obs_every");
    if (obs_every > 0 && !obs_dev) return fail(HEOM_E_INVAL, "obs_dev is NULL");
    const bool hermitian = (precision & HEOM_HERMITIAN) != 0;
    precision &= ~HEOM_HERMITIAN;
    if (precision != HEOM_FP64 && precision != HEOM_FP32) return fail(HEOM_E_INVAL, "unknown precision");
    const HostTables &t = h->t;
    if (work_bytes < work_bytes_for(t)) return fail(HEOM_E_TOO_LARGE, "work buffer smaller than work_bytes");
    if (hermitian && !adjoint_preserving(t))
        return fail(HEOM_E_INVAL, "HEOM_HERMITIAN needs c_check = conj(c) for every channel");
    if (t.compact && !hermitian) return fail(HEOM_E_STATE, "compact tiles need HEOM_HERMITIAN");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double2 *y = static_cast<double2 *>(y_dev);
    if (obs_every > 0) {
        hipLaunchKernelGGL(observables_kernel, dim3(1), dim3(64), 0, s, dev_view(t), y, obs_dev);
        HIP_TRY(hipGetLastError());
    }
    if (nsteps == 0) return HEOM_OK;
    const WorkView wv = work_view(t, work_dev);
    PersistArgs pa{};
    pa.y = y;
    pa.dt = dt;
    pa.step0 = 0;
    pa.nsteps = nsteps;
    pa.obs_every = obs_every;
    pa.obs = obs_every > 0 ? obs_dev : nullptr;
    pa.timeout = reinterpret_cast<uint32_t *>(wv.ctrl + 4);
    pa.flags = reinterpret_cast<uint32_t *>(wv.ctrl + 256);
    pa.limit = t.tune.spin_limit > 0 ? (uint32_t)t.tune.spin_limit : (1u << 20);
    pa.policy = (uint32_t)t.tune.cache_policy;
    if (precision == HEOM_FP64) {
        pa.w0 = wv.w0;
        pa.w1 = wv.w1;
    } else {
        pa.u3 = wv.u3;
        pa.u1 = wv.u1;
        pa.u2 = wv.u2;
    }
    hipLaunchKernelGGL(zero_u32_kernel, dim3(64), dim3(256), 0, s, pa.timeout - 1, (uint32_t)(CTRL_BYTES / 4));
    HIP_TRY(hipGetLastError());
    const bool persist = t.tune.persistent == 1 || t.tune.persistent == 3 ||
                         (t.tune.persistent == 2 && t.tiles.size() <= 256);
    bool used = false;
    if (persist)
        if (int rc = launch_persistent(t, s, pa, precision, &used)) return rc;
    if (!used)
        if (int rc = propagate_stages(t, s, y, wv, pa, precision, hermitian, dt, nsteps, obs_every, obs_dev))
            return rc;
    // flag a non-finite tier-0 block or observable (heom_work_status reports it)
    const uint32_t n_obs = obs_every > 0 ? (uint32_t)((nsteps / obs_every + 1) * HEOM_NOBS) : 0u;
    hipLaunchKernelGGL(finite_check_kernel, dim3(1), dim3(256), 0, s, reinterpret_cast<const double *>(y),
                       (uint32_t)(2 * tier0_size(t)), obs_every > 0 ? obs_dev : nullptr, n_obs,
                       reinterpret_cast<uint32_t *>(wv.ctrl + 8));
    HIP_TRY(hipGetLastError());
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
    out->n_tiles = (int64_t)t.tiles.size();
    out->n_categories = (int64_t)t.cat.size();
    out->table_bytes = (int64_t)t.image.size();
    out->work_bytes_fp64 = (int64_t)work_bytes_for(t);
    out->work_bytes_fp32 = (int64_t)work_bytes_for(t);
    out->tier0_size = (int64_t)tier0_size(t);
    out->max_G = t.max_G;
    out->tile_vars = t.tile_vars;
    out->hier_gathers = t.hier_gathers;
    out->rhs_work_bytes = (int64_t)rhs_work_bytes_for(t);
    out->transposed = t.trcol ? 1 : 0;
    out->compact = t.compact ? 1 : 0;
    size_t covered = 0;
    for (const TileRec &r : t.tiles) covered += r.nv;
    out->stage_table_bytes = (int64_t)t.image.size() - (t.compact ? (int64_t)(sizeof(VarRec) * (t.n_var - covered)) : 0);
    out->own_entries = t.own_entries;
    out->read_entries = t.read_entries;
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

// Representative slot of tier-0 index idx (0 = cavity, q+1 = category q):
// distinguished molecules come first among the empty pattern's categories,
// in label order, then the pool.
static int tier0_slot(const HostTables &t, int idx) {
    if (idx == 0) return 0;
    const CatRec &c = t.cat[t.hdr[0].cat_base + idx - 1];
    return (c.flags & CAT_DIST) ? idx : t.d + 1;
}

int heom_tier0_operator(const heom_tables *h, const double *R, double *out) {
    if (!h || !R || !out) return fail(HEOM_E_INVAL, "NULL argument");
    const HostTables &t = h->t;
    const PatHdr &H = t.hdr[0];
    const int G = H.G, G1 = G + 1, ns = t.d + 3;
    auto put = [&](size_t pos, int a, int b) {
        out[2 * pos] = R[2 * (a * ns + b)];
        out[2 * pos + 1] = R[2 * (a * ns + b) + 1];
    };
    for (int A = 0; A < G1; ++A)
        for (int B = 0; B < G1; ++B) put((size_t)A * G1 + B, tier0_slot(t, A), tier0_slot(t, B));
    size_t pos = (size_t)G1 * G1;
    for (int q = 0; q < G; ++q)
        if ((H.tmask >> q) & 1u) put(pos++, t.d + 1, t.d + 2);   // two different pool molecules
    return HEOM_OK;
}

int heom_tier0_expand(const heom_tables *h, const double *tier0, double *R) {
    if (!h || !tier0 || !R) return fail(HEOM_E_INVAL, "NULL argument");
    const HostTables &t = h->t;
    const PatHdr &H = t.hdr[0];
    const int G = H.G, G1 = G + 1, ns = t.d + 3;
    std::fill(R, R + 2 * ns * ns, 0.0);
    auto get = [&](size_t pos, int a, int b) {
        R[2 * (a * ns + b)] = tier0[2 * pos];
        R[2 * (a * ns + b) + 1] = tier0[2 * pos + 1];
    };
    const int pa = t.d + 1, pb = t.d + 2;
    for (int A = 0; A < G1; ++A)
        for (int B = 0; B < G1; ++B) {
            const int a = tier0_slot(t, A), b = tier0_slot(t, B);
            get((size_t)A * G1 + B, a, b);
            // the second pool molecule has the same entries as the first
            // (the coherence between the two is the T variable, below)
            if (a == pa && b != pa) get((size_t)A * G1 + B, pb, b);
            if (b == pa && a != pa) get((size_t)A * G1 + B, a, pb);
            if (a == pa && b == pa) get((size_t)A * G1 + B, pb, pb);
        }
    size_t pos = (size_t)G1 * G1;
    for (int q = 0; q < G; ++q)
        if ((H.tmask >> q) & 1u) {
            get(pos, pa, pb);
            get(pos, pb, pa);
            ++pos;
        }
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

int heom_rhs(const heom_tables *h, const void *y_dev, void *dy_dev, void *work_dev, size_t work_bytes,
             int precision, void *stream) {
    if (int rc = check_ready(h)) return rc;
    if (int rc = check_dev(y_dev, "y_dev")) return rc;
    if (int rc = check_dev(dy_dev, "dy_dev")) return rc;
    if (y_dev == dy_dev) return fail(HEOM_E_INVAL, "y_dev and dy_dev must differ");
    const bool hermitian = (precision & HEOM_HERMITIAN) != 0;
    precision &= ~HEOM_HERMITIAN;
    if (precision != HEOM_FP64 && precision != HEOM_FP32) return fail(HEOM_E_INVAL, "unknown precision");
    const HostTables &t = h->t;
    if (hermitian && !adjoint_preserving(t))
        return fail(HEOM_E_INVAL, "HEOM_HERMITIAN needs c_check = conj(c) for every channel");
    if (t.compact && !hermitian) return fail(HEOM_E_STATE, "compact tiles need HEOM_HERMITIAN");
    // column moves of transposed tables read the mirrored entry (Hermitian
    // ADOs) or a transposed copy of y made here
    const bool mirror = hermitian && t.trcol;
    const bool copy = t.trcol && !mirror;
    const size_t need = copy ? rhs_work_bytes_for(t) : 0;
    if (need > 0 && !work_dev) return fail(HEOM_E_INVAL, "work_dev is NULL");
    if (work_bytes < need) return fail(HEOM_E_TOO_LARGE, "work buffer smaller than rhs_work_bytes");
    if (copy && (work_dev == y_dev || work_dev == dy_dev)) return fail(HEOM_E_INVAL, "work_dev overlaps y_dev or dy_dev");
    hipStream_t s = static_cast<hipStream_t>(stream);
    StageArgs a{};
    a.alpha = 1.0;
    a.policy = mirror ? 8u : 0u;
    if (precision == HEOM_FP64) {
        a.in64 = static_cast<const double2 *>(y_dev);
        a.out64 = static_cast<double2 *>(dy_dev);
        if (copy) {
            double2 *yT = static_cast<double2 *>(work_dev);
            if (int rc = launch_transpose(t, s, a.in64, yT)) return rc;
            a.inT64 = yT;
        }
        return launch_stage<true, false, BASE_NONE, false, true>(t, s, a);
    }
    // FP32 bulk: complex64 values in and out, FP64 weights and arithmetic
    a.in32 = static_cast<const float2 *>(y_dev);
    a.out32 = static_cast<float2 *>(dy_dev);
    if (copy) {
        float2 *yT = static_cast<float2 *>(work_dev);
        if (int rc = launch_transpose(t, s, a.in32, yT)) return rc;
        a.inT32 = yT;
    }
    return launch_stage<false, true, BASE_NONE, false, false>(t, s, a);
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
    return propagate_impl(h, y_dev, work_dev, work_bytes, dt, nsteps, obs_every, obs_dev, precision, stream);
}

int heom_propagate_noalloc(const heom_tables *h, void *y_dev, double dt, int64_t nsteps, int64_t obs_every,
                           double *obs_dev, int precision, void *stream) {
    if (int rc = check_ready(h)) return rc;
    if (work_bytes_for(h->t) > HEOM_NOALLOC_WORK_BYTES)
        return fail(HEOM_E_TOO_LARGE, "the tables' work_bytes exceed HEOM_NOALLOC_WORK_BYTES (use heom_propagate "
                                      "with a caller work buffer)");
    void *work = nullptr;
    if (int rc = scratch_address(&work)) return rc;
    return propagate_impl(h, y_dev, work, HEOM_NOALLOC_WORK_BYTES, dt, nsteps, obs_every, obs_dev, precision, stream);
}

int heom_set_tuning(heom_tables *h, const heom_tuning *tu) {
    if (!h || !tu) return fail(HEOM_E_INVAL, "NULL argument");
    HostTables &t = h->t;
    if (tu->persistent < 0 || tu->persistent > 3) return fail(HEOM_E_INVAL, "persistent must be 0, 1, 2 or 3");
    if (tu->cache_policy < 0 || tu->cache_policy > 7) return fail(HEOM_E_INVAL, "cache_policy must be 0..7");
    if (tu->transposed < -1 || tu->transposed > 1) return fail(HEOM_E_INVAL, "transposed must be -1, 0 or 1");
    if (tu->compact < 0 || tu->compact > 1) return fail(HEOM_E_INVAL, "compact must be 0 or 1");
    const bool compact = tu->compact != 0;
    const bool trcol = compact || (tu->transposed < 0 ? t.n_var >= TRANSPOSED_MIN_VARS : tu->transposed != 0);
    const int tv = tu->tile_vars != 0 ? tu->tile_vars : t.tile_vars;
    const int old_mode = t.tune.transposed, old_compact = t.tune.compact, old_tv = t.tile_vars;
    t.tune.transposed = tu->transposed;
    t.tune.compact = tu->compact;
    if (tv != t.tile_vars || trcol != t.trcol || compact != t.compact) {
        std::string err;
        if (int rc = make_tiles(&t, tv, &err)) {
            t.tune.transposed = old_mode;
            t.tune.compact = old_compact;
            // restore the previous tiles (the same arguments built them before)
            make_tiles(&t, old_tv, &err);
            return fail(rc, err);
        }
    }
    t.tune.persistent = tu->persistent;
    t.tune.xcd_map = tu->xcd_map ? 1 : 0;
    t.tune.max_workgroups = tu->max_workgroups;
    t.tune.spin_limit = tu->spin_limit;
    t.tune.cache_policy = tu->cache_policy;
    return HEOM_OK;
}

int heom_work_status(const heom_tables *h, const void *work_dev, size_t work_bytes, void *stream) {
    if (!h || !work_dev) return fail(HEOM_E_INVAL, "NULL argument");
    if (work_bytes < work_bytes_for(h->t)) return fail(HEOM_E_TOO_LARGE, "work buffer smaller than work_bytes");
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t flag[2] = {0u, 0u};            // timeout word, non-finite flag
    const unsigned char *p = static_cast<const unsigned char *>(work_dev) + vec_bytes(h->t) + 4;
    HIP_TRY(hipMemcpyAsync(flag, p, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (flag[0]) return fail(HEOM_E_TIMEOUT, "a grid barrier of the persistent kernel timed out");
    if (flag[1]) return fail(HEOM_E_NONFINITE, "the propagated tier-0 block or an observable is not finite");
    return HEOM_OK;
}

int heom_get_tuning(const heom_tables *h, heom_tuning *tu) {
    if (!h || !tu) return fail(HEOM_E_INVAL, "NULL argument");
    tu->tile_vars = h->t.tile_vars;
    tu->persistent = h->t.tune.persistent;
    tu->xcd_map = h->t.tune.xcd_map;
    tu->max_workgroups = h->t.tune.max_workgroups;
    tu->spin_limit = h->t.tune.spin_limit;
    tu->cache_policy = h->t.tune.cache_policy;
    tu->transposed = h->t.tune.transposed;
    tu->compact = h->t.tune.compact;
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

int heom_params_bytes(const heom_tables *h, size_t *bytes) {
    if (!h || !bytes) return fail(HEOM_E_INVAL, "NULL argument");
    const InstParams *ip = reinterpret_cast<const InstParams *>(h->t.image.data());
    *bytes = ip->off_hdr;
    return HEOM_OK;
}

int heom_upload_params(const heom_tables *h, const heom_problem *prob, void *dev, size_t bytes, void *stream) {
    if (!h || !prob || !dev) return fail(HEOM_E_INVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(dev) % 256) return fail(HEOM_E_INVAL, "params buffer must be 256-byte aligned");
    std::vector<unsigned char> blk;
    std::string err;
    if (int rc = pack_params(h->t, prob, &blk, &err)) return fail(rc, err);
    if (bytes < blk.size()) return fail(HEOM_E_TOO_LARGE, "params buffer smaller than heom_params_bytes");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(dev, blk.data(), blk.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::lock_guard<std::mutex> lk(g_params_mu);
    g_params[reinterpret_cast<uintptr_t>(dev)] = ParamsStamp{h->t.id, h->t.layout_gen, adjoint_preserving(*prob)};
    return HEOM_OK;
}

int heom_batch_create(int32_t capacity, heom_batch **out) {
    if (!out || capacity < 1) return fail(HEOM_E_INVAL, "bad capacity or NULL out");
    *out = nullptr;
    heom_batch *b = new (std::nothrow) heom_batch;
    if (!b) return fail(HEOM_E_NOMEM, "host allocation failed");
    b->slots.resize((size_t)capacity);
    *out = b;
    return HEOM_OK;
}

int heom_batch_set_slot(heom_batch *b, int32_t slot, const heom_tables *t, const void *params_dev, void *y_dev,
                        void *work_dev, size_t work_bytes, double dt, double *obs_dev, int64_t obs_every,
                        int64_t obs_capacity) {
    if (!b || slot < 0 || (size_t)slot >= b->slots.size()) return fail(HEOM_E_INVAL, "bad batch or slot");
    if (int rc = check_ready(t)) return rc;
    if (int rc = check_dev(y_dev, "y_dev")) return rc;
    if (int rc = check_dev(work_dev, "work_dev")) return rc;
    if (params_dev && reinterpret_cast<uintptr_t>(params_dev) % 256) return fail(HEOM_E_INVAL, "params_dev alignment");
    if (work_bytes < work_bytes_for(t->t)) return fail(HEOM_E_TOO_LARGE, "work buffer smaller than work_bytes");
    if (!std::isfinite(dt)) return fail(HEOM_E_INVAL, "dt not finite");
    if (obs_every < 0 || obs_capacity < 0 || (obs_every > 0 && !obs_dev)) return fail(HEOM_E_INVAL, "bad observables");
    BatchSlotHost &S = b->slots[(size_t)slot];
    S.used = true;
    S.tables = t;
    S.params = params_dev;
    S.y = y_dev;
    S.work = work_dev;
    S.work_bytes = work_bytes;
    S.dt = dt;
    S.obs = obs_dev;
    S.obs_every = obs_every;
    S.obs_cap = obs_capacity;
    S.steps = 0;
    b->committed = false;
    return HEOM_OK;
}

int heom_batch_clear_slot(heom_batch *b, int32_t slot) {
    if (!b || slot < 0 || (size_t)slot >= b->slots.size()) return fail(HEOM_E_INVAL, "bad batch or slot");
    b->slots[(size_t)slot] = BatchSlotHost{};
    b->committed = false;
    return HEOM_OK;
}

int heom_batch_device_bytes(const heom_batch *b, size_t *bytes) {
    if (!b || !bytes) return fail(HEOM_E_INVAL, "NULL argument");
    size_t nt = 0;
    for (const auto &S : b->slots)
        if (S.used) nt += S.tables->t.tiles.size();
    // slot records, tile list, slot lists of shared groups (each slot in at
    // most two lists, each list a count and its slots), then the 8-byte step
    // counter and the slots' non-finite flags (4 bytes each)
    const size_t ns = b->slots.size();
    *bytes = ((sizeof(SlotRec) * ns + 255) & ~(size_t)255) + ((sizeof(BatchTile) * nt + 255) & ~(size_t)255) +
             ((4 * (4 * ns + 4) + 255) & ~(size_t)255) + ((8 + 4 * ns + 255) & ~(size_t)255);
    return HEOM_OK;
}

int heom_batch_commit(heom_batch *b, void *dev, size_t bytes, void *stream) {
    if (!b || !dev) return fail(HEOM_E_INVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(dev) % 256) return fail(HEOM_E_INVAL, "batch buffer must be 256-byte aligned");
    size_t need = 0;
    heom_batch_device_bytes(b, &need);
    if (bytes < need) return fail(HEOM_E_TOO_LARGE, "batch buffer smaller than heom_batch_device_bytes");
    const size_t ns = b->slots.size();
    const size_t tile_off = (sizeof(SlotRec) * ns + 255) & ~(size_t)255;
    // the tables of a slot may have been re-tuned or re-uploaded since
    // heom_batch_set_slot: every pointer into their image is resolved here,
    // and a caller's parameter block must have been written for the tables'
    // current layout
    for (auto &S : b->slots) {
        if (!S.used) continue;
        if (int rc = check_ready(S.tables)) return rc;
        const HostTables &t = S.tables->t;
        if (S.work_bytes < work_bytes_for(t))
            return fail(HEOM_E_TOO_LARGE, "a slot's work buffer is smaller than its tables' work_bytes");
        if (!S.params) {
            S.adjoint = adjoint_preserving(t);
            continue;
        }
        std::lock_guard<std::mutex> lk(g_params_mu);
        const auto it = g_params.find(reinterpret_cast<uintptr_t>(S.params));
        if (it == g_params.end() || it->second.tables_id != t.id)
            return fail(HEOM_E_STATE, "a slot's parameter block was not written by heom_upload_params for its tables");
        if (it->second.layout_gen != t.layout_gen)
            return fail(HEOM_E_STATE, "a slot's parameter block predates a re-tuning of its tables "
                                      "(write it again with heom_upload_params)");
        S.adjoint = it->second.adjoint;
    }
    std::vector<unsigned char> img(need, 0);
    SlotRec *recs = reinterpret_cast<SlotRec *>(img.data());
    BatchTile *tl = reinterpret_cast<BatchTile *>(img.data() + tile_off);
    b->groups.clear();
    for (size_t i = 0; i < ns; ++i) {
        const BatchSlotHost &S = b->slots[i];
        if (!S.used) continue;
        const HostTables &t = S.tables->t;
        SlotRec &R = recs[i];
        R.img = static_cast<const unsigned char *>(t.dev);
        R.params = static_cast<const unsigned char *>(S.params ? S.params : t.dev);
        const Dev D = dev_view(t);
        R.hdr = D.hdr;
        R.cat = D.cat;
        R.gidx = D.gidx;
        R.tiles = D.tiles;
        R.vrec = D.vrec;
        R.lut = reinterpret_cast<const double *>(R.params + reinterpret_cast<const InstParams *>(t.image.data())->off_lut);
        const WorkView wv = work_view(t, S.work);
        R.y = static_cast<double2 *>(S.y);
        R.w0 = wv.w0;
        R.w1 = wv.w1;
        R.u1 = wv.u1;
        R.u2 = wv.u2;
        R.u3 = wv.u3;
        R.yT = wv.yT;
        R.w0T = wv.w0T;
        R.w1T = wv.w1T;
        R.u1T = wv.u1T;
        R.u2T = wv.u2T;
        R.u3T = wv.u3T;
        R.obs = S.obs;
        R.obs_every = S.obs_every;
        R.obs_cap = S.obs_cap;
        R.step0 = S.steps;
        R.dt = S.dt;
    }
    // Group the tiles by (m, tile size, tier class); within a group, slot by
    // slot in slot order and each slot's tiles in order (with interleave > 0
    // the slots of one structure image take turns, a chunk of tiles each, so
    // that workgroups running together read the same tables). Then the smallest
    // groups with m <= MERGE_MAX_M, up to merge_tiles tiles in all, become one
    // merged launch whose tiles come first in the list. In every other group,
    // with share_slots = 2, the slots that share one structure image are
    // computed in pairs (a shared launch of the group); the rest keep one
    // workgroup per slot and tile.
    std::vector<int> sizes;
    for (const auto &S : b->slots)
        if (S.used) sizes.push_back(S.tables->t.tile_vars);
    std::sort(sizes.begin(), sizes.end());
    sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
    struct Member {
        uint32_t slot, j0, j1;
    };
    struct Pending {
        heom_batch::Group g;
        std::vector<BatchTile> tiles;
        std::vector<Member> members;
    };
    std::vector<Pending> pend;
    size_t used = 0;
    for (const auto &S : b->slots) used += S.used ? 1 : 0;
    for (int m = 1; m <= HEOM_MAX_M; ++m)
        for (int tv : sizes)
            for (int top = 0; top < 2; ++top) {
                Pending P{{m, top != 0, (uint32_t)tv, 0u, 0u, 0u, -1, 0u}, {}, {}};
                bool all_compact = true;
                for (size_t i = 0; i < ns; ++i) {
                    const BatchSlotHost &S = b->slots[i];
                    if (!S.used || S.tables->t.m != m || S.tables->t.tile_vars != tv) continue;
                    const HostTables &t = S.tables->t;
                    const uint32_t T = (uint32_t)t.tiles.size();
                    // Top-tier tiles run with the top-tier variant: in a batch the extra
                    // launch is shared by every slot of the group, and small groups are
                    // merged below. A batch of one slot follows heom_propagate.
                    const bool split_ok = used > 1 || T >= TOP_SPLIT_TILES;
                    const uint32_t split = (split_ok && t.top_tile > 0 && t.top_tile < T) ? t.top_tile : T;
                    const uint32_t j0 = top ? split : 0, j1 = top ? T : split;
                    if (j1 <= j0) continue;
                    for (uint32_t j = j0; j < j1; ++j) P.tiles.push_back(BatchTile{(uint32_t)i, top ? (j | BTILE_TOP) : j});
                    P.members.push_back(Member{(uint32_t)i, j0, j1});
                    // LDS for the longest gather list among the group's tiles
                    // (the top tier's lists are about a third as long)
                    const uint32_t lds = split < T ? (top ? t.lds_top : t.lds_low) : t.lds_bytes;
                    P.g.lds = std::max<uint32_t>(P.g.lds, lds);
                    all_compact = all_compact && t.compact;
                }
                P.g.compact = all_compact;
                if (!P.tiles.empty()) pend.push_back(std::move(P));
            }
    std::vector<size_t> order(pend.size());
    for (size_t q = 0; q < order.size(); ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t x, size_t y) { return pend[x].tiles.size() < pend[y].tiles.size(); });
    std::vector<char> merged(pend.size(), 0);
    size_t mtiles = 0, mcount = 0;
    for (size_t q : order) {
        // large groups keep their own launch (and the occupancy of their own
        // kernel variant); only small ones are worth a shared launch
        if (pend[q].g.m > MERGE_MAX_M || pend[q].tiles.size() > (size_t)b->merge_tiles / 8) continue;
        if (mtiles + pend[q].tiles.size() > (size_t)b->merge_tiles) break;
        merged[q] = 1;
        mtiles += pend[q].tiles.size();
        ++mcount;
    }
    if (mcount < 2) std::fill(merged.begin(), merged.end(), 0);
    size_t k = 0;
    if (mcount >= 2) {
        heom_batch::Group M{0, false, 64u, 0u, 0u, 0u, -1, 0u};
        for (size_t q = 0; q < pend.size(); ++q)
            if (merged[q]) {
                for (const auto &bt : pend[q].tiles) tl[k++] = bt;
                M.block = std::max(M.block, pend[q].g.block);
                M.lds = std::max(M.lds, pend[q].g.lds);
            }
        M.count = (uint32_t)k;
        b->groups.push_back(M);
    }
    // slot lists of the shared groups, after the tile list (an upper bound
    // of its length: every slot's tiles once)
    size_t nt_all = 0;
    for (const auto &S : b->slots)
        if (S.used) nt_all += S.tables->t.tiles.size();
    const size_t list_off = tile_off + ((sizeof(BatchTile) * nt_all + 255) & ~(size_t)255);
    uint32_t *lists = reinterpret_cast<uint32_t *>(img.data() + list_off);
    uint32_t nl = 0;
    for (size_t q = 0; q < pend.size(); ++q) {
        if (merged[q]) continue;
        // members by structure image
        std::vector<std::vector<Member>> by_t;
        {
            std::vector<const heom_tables *> keys;
            for (const Member &mb : pend[q].members) {
                const heom_tables *t = b->slots[mb.slot].tables;
                size_t w = 0;
                while (w < keys.size() && keys[w] != t) ++w;
                if (w == keys.size()) {
                    keys.push_back(t);
                    by_t.emplace_back();
                }
                by_t[w].push_back(mb);
            }
        }
        heom_batch::Group SG = pend[q].g;
        SG.shared = true;
        SG.lds = 0;
        SG.first = (uint32_t)k;
        std::vector<char> plain_slot(ns, 0);
        // pairs of slots on one structure image (workgroups of twice the
        // tile size, so tiles of at most MAX_TILE / 2 variables); an odd slot
        // out keeps one-slot workgroups
        for (const auto &grp : by_t) {
            const InstParams *ip0 = reinterpret_cast<const InstParams *>(b->slots[grp[0].slot].tables->t.image.data());
            const bool fits = pend[q].g.block * 2u <= (uint32_t)MAX_TILE &&
                              pair_shared_bytes(*ip0) + 2u * pair_half_bytes(*ip0) <= 64u * 1024u;
            const size_t pairs = (b->share_slots >= 2 && fits) ? grp.size() / 2 : 0;
            for (size_t c = 2 * pairs; c < grp.size(); ++c) plain_slot[grp[c].slot] = 1;
            for (size_t c = 0; c < pairs; ++c) {
                const uint32_t off = nl;
                lists[nl++] = 2u;
                lists[nl++] = grp[2 * c].slot;
                lists[nl++] = grp[2 * c + 1].slot;
                for (uint32_t j = grp[2 * c].j0; j < grp[2 * c].j1; ++j)
                    tl[k++] = BatchTile{off, SG.top ? (j | BTILE_TOP) : j};
            }
            if (pairs > 0) SG.lds = std::max<uint32_t>(SG.lds, pair_shared_bytes(*ip0) + 2u * pair_half_bytes(*ip0));
        }
        SG.count = (uint32_t)(k - SG.first);
        if (SG.count > 0) b->groups.push_back(SG);
        heom_batch::Group G = pend[q].g;
        G.first = (uint32_t)k;
        if (b->interleave > 0) {
            // the members of one image have the same tile range (same tables)
            const uint32_t c = (uint32_t)b->interleave;
            for (const auto &grp : by_t) {
                const uint32_t j0 = grp[0].j0, j1 = grp[0].j1;
                for (uint32_t jc = j0; jc < j1; jc += c)
                    for (const Member &mb : grp) {
                        if (!plain_slot[mb.slot]) continue;
                        for (uint32_t j = jc; j < std::min(jc + c, j1); ++j)
                            tl[k++] = BatchTile{mb.slot, G.top ? (j | BTILE_TOP) : j};
                    }
            }
        } else {
            for (const auto &bt : pend[q].tiles)
                if (plain_slot[bt.slot]) tl[k++] = bt;
        }
        G.count = (uint32_t)(k - G.first);
        if (G.count == 0) continue;
        bool one_slot = true;
        for (uint32_t x = G.first; x < k; ++x) one_slot = one_slot && tl[x].slot == tl[G.first].slot;
        // a group of one slot: its record goes in the kernel arguments
        if (one_slot) {
            G.slot = (int32_t)tl[G.first].slot;
            G.tile0 = tl[G.first].tile & ~BTILE_TOP;
        }
        b->groups.push_back(G);
    }
    if (nl > 4 * ns + 4) return fail(HEOM_E_INVAL, "internal: slot lists exceed their section");
    b->list_off = list_off;
    b->recs.assign(recs, recs + ns);
    b->ctr_off = list_off + ((4 * (4 * ns + 4) + 255) & ~(size_t)255);   // counter = 0 in img
    if (b->gexec) {                        // the captured launches name the old layout
        HIP_TRY(hipGraphExecDestroy(b->gexec));
        b->gexec = nullptr;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(dev, img.data(), need, hipMemcpyHostToDevice, s));
    // Row 0 of a new slot's observables: the initial state, evaluated with
    // the slot's own parameter block (as heom_propagate does at its start).
    for (const auto &S : b->slots) {
        if (!S.used || S.steps != 0 || !S.obs || S.obs_every <= 0 || S.obs_cap <= 0) continue;
        Dev D = dev_view(S.tables->t);
        D.ip = static_cast<const InstParams *>(S.params ? S.params : S.tables->t.dev);
        hipLaunchKernelGGL(observables_kernel, dim3(1), dim3(64), 0, s, D, static_cast<const double2 *>(S.y), S.obs);
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(s));
    b->dev = dev;
    b->dev_bytes = bytes;
    b->committed = true;
    b->steps_since_commit = 0;
    return HEOM_OK;
}

int heom_batch_propagate(heom_batch *b, int64_t nsteps, int precision, void *stream) {
    if (!b) return fail(HEOM_E_INVAL, "batch is NULL");
    if (!b->committed) return fail(HEOM_E_STATE, "batch changed since the last heom_batch_commit");
    if (nsteps < 0) return fail(HEOM_E_INVAL, "nsteps < 0");
    const int base_prec = precision & ~HEOM_HERMITIAN;
    if (base_prec != HEOM_FP64 && base_prec != HEOM_FP32) return fail(HEOM_E_INVAL, "unknown precision");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (nsteps == 0) return HEOM_OK;
    for (const auto &S : b->slots) {
        if (!S.used) continue;
        if (S.tables->t.compact && !(precision & HEOM_HERMITIAN))
            return fail(HEOM_E_STATE, "a slot has compact tiles, which need HEOM_HERMITIAN");
        if ((precision & HEOM_HERMITIAN) && !S.adjoint)
            return fail(HEOM_E_INVAL, "HEOM_HERMITIAN needs c_check = conj(c) in every slot's parameters");
    }
    int64_t done = 0;
    // A batch of one slot (launched directly) takes heom_propagate's stage
    // launches with the slot's parameter block: one state gains nothing from
    // the batch kernels' slot records, which cost a little per launch.
    size_t used = 0, only = 0;
    for (size_t i = 0; i < b->slots.size(); ++i)
        if (b->slots[i].used) ++used, only = i;
    const int64_t K = b->graph_steps;
    const bool solo = used == 1 && !(K > 0 && s != nullptr && nsteps >= K);
    // slots with transposed copies: the copy of y, made once per call
    // (Hermitian ADOs use no copies; the one-slot path makes its own)
    for (size_t i = 0; i < b->slots.size() && !solo; ++i) {
        const BatchSlotHost &S = b->slots[i];
        if (!S.used || !S.tables->t.trcol || (precision & HEOM_HERMITIAN)) continue;
        if (int rc = launch_transpose(S.tables->t, s, b->recs[i].y, b->recs[i].yT)) return rc;
    }
    if (solo) {
        const BatchSlotHost &S = b->slots[only];
        const HostTables &t = S.tables->t;
        Dev D = dev_view(t);
        D.ip = static_cast<const InstParams *>(b->recs[only].params ? static_cast<const void *>(b->recs[only].params)
                                                                     : t.dev);
        D.lut = b->recs[only].lut;
        const WorkView wv = work_view(t, S.work);
        PersistArgs pa{};
        pa.w0 = wv.w0;
        pa.w1 = wv.w1;
        pa.u1 = wv.u1;
        pa.u2 = wv.u2;
        pa.u3 = wv.u3;
        if (int rc = propagate_stages(t, s, static_cast<double2 *>(S.y), wv, pa, base_prec,
                                      (precision & HEOM_HERMITIAN) != 0, S.dt, nsteps, S.obs_every, S.obs, &D, S.steps,
                                      S.obs_cap))
            return rc;
        unsigned char *cb = static_cast<unsigned char *>(b->dev);
        hipLaunchKernelGGL(counter_add_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<int64_t *>(cb + b->ctr_off),
                           nsteps);
        HIP_TRY(hipGetLastError());
        done = nsteps;
    }
    // Whole graphs of graph_steps steps where possible (not on the null
    // stream, which cannot be captured), single launches for the rest.
    if (done == 0 && K > 0 && s != nullptr && nsteps >= K) {
        if (!b->gexec || b->gprec != precision)
            if (int rc = batch_capture(b, s, precision)) return rc;
        for (; done + K <= nsteps; done += K) HIP_TRY(hipGraphLaunch(b->gexec, s));
    }
    for (; done < nsteps; ++done)
        if (int rc = batch_step(b, s, precision)) return rc;
    // flag slots whose tier-0 block is no longer finite (heom_batch_status)
    unsigned char *base = static_cast<unsigned char *>(b->dev);
    hipLaunchKernelGGL(batch_finite_kernel, dim3((uint32_t)b->slots.size()), dim3(64), 0, s,
                       static_cast<const SlotRec *>(b->dev), reinterpret_cast<uint32_t *>(base + b->ctr_off + 8));
    HIP_TRY(hipGetLastError());
    b->steps_since_commit += nsteps;
    for (auto &S : b->slots)
        if (S.used) S.steps += nsteps;
    return HEOM_OK;
}

int heom_batch_status(const heom_batch *b, int32_t *slot_flags, int32_t cap, void *stream) {
    if (!b || cap < 0 || (cap > 0 && !slot_flags)) return fail(HEOM_E_INVAL, "bad argument");
    if (!b->committed) return fail(HEOM_E_STATE, "batch changed since the last heom_batch_commit");
    const size_t ns = b->slots.size();
    std::vector<uint32_t> fl(ns, 0u);
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(fl.data(), static_cast<const unsigned char *>(b->dev) + b->ctr_off + 8, 4 * ns,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    bool any = false;
    for (size_t i = 0; i < ns; ++i) {
        if (i < (size_t)cap) slot_flags[i] = fl[i] ? 1 : 0;
        any |= fl[i] != 0u;
    }
    return any ? fail(HEOM_E_NONFINITE, "a slot's tier-0 block is not finite") : HEOM_OK;
}

int heom_batch_slot_steps(const heom_batch *b, int32_t slot, int64_t *steps) {
    if (!b || !steps || slot < 0 || (size_t)slot >= b->slots.size()) return fail(HEOM_E_INVAL, "bad argument");
    *steps = b->slots[(size_t)slot].steps;
    return HEOM_OK;
}

int heom_batch_set_graph(heom_batch *b, int32_t steps) {
    if (!b || steps < 0 || steps > 4096) return fail(HEOM_E_INVAL, "bad batch or graph step count");
    if (steps != b->graph_steps && b->gexec) {
        HIP_TRY(hipGraphExecDestroy(b->gexec));
        b->gexec = nullptr;
    }
    b->graph_steps = steps;
    return HEOM_OK;
}

int heom_batch_set_share(heom_batch *b, int32_t max_slots) {
    if (!b || max_slots < 1 || max_slots > 2) return fail(HEOM_E_INVAL, "bad batch, or slots per workgroup not 1 or 2");
    b->share_slots = max_slots;
    b->committed = false;
    return HEOM_OK;
}

int heom_batch_set_interleave(heom_batch *b, int32_t tiles) {
    if (!b || tiles < 0) return fail(HEOM_E_INVAL, "bad batch or chunk length");
    b->interleave = tiles;
    b->committed = false;
    return HEOM_OK;
}

int heom_batch_set_merge(heom_batch *b, int32_t max_tiles) {
    if (!b || max_tiles < 0) return fail(HEOM_E_INVAL, "bad batch or tile count");
    b->merge_tiles = max_tiles;
    b->committed = false;
    return HEOM_OK;
}

void heom_batch_free(heom_batch *b) { delete b; }

const char *heom_last_error(void) { return g_err.c_str(); }

const char *heom_version(void) { return "heom-mi355x 0.1 (gfx950)"; }

}  // extern "C"
