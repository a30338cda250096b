// Internal definitions shared by the host table builder (tables.cpp) and the
// gfx950 kernels (device.hip): the device image of the tables and the
// category remap rule of a connection record.
#pragma once

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "heom.h"

#ifdef __HIPCC__
#define HEOM_HD __host__ __device__ __forceinline__
#else
#define HEOM_HD inline
#endif

namespace heom {

// One canonical pattern (Sec. IV.A). 32 bytes.
struct PatHdr {
    uint32_t off;        // first unique variable of the block
    uint32_t cat_base;   // index of the first CatRec of the pattern
    uint32_t conn_base;  // index of the first Conn of the pattern
    uint16_t tmask;      // bit q: category q has M_q >= 2 and owns a T_q
    uint8_t  G;          // number of categories
    uint8_t  tier;       // |Lambda|
    uint64_t cnt;        // byte k: sum over molecules of n_ik (for Gamma_Lambda)
    uint32_t r;          // nonzero pool molecules; M_0 = (N - d) - r
    uint32_t size;       // (G+1)^2 + h
};
static_assert(sizeof(PatHdr) == 32, "PatHdr layout");

enum : uint16_t { CAT_ZERO = 1, CAT_DIST = 2 };

// One occupation category of a pattern (Sec. V.A). 16 bytes.
struct CatRec {
    uint64_t vec;        // byte k: component k of the local vector
    uint32_t mult;       // M_q (0 for the zero category: its M_0 is per instance)
    uint16_t conn_off;   // first Conn of this category, relative to conn_base
    uint16_t flags;      // CAT_ZERO, CAT_DIST
};
static_assert(sizeof(CatRec) == 16, "CatRec layout");

// One connection: moving one molecule of a category by +-e_k
// (Eqs. raw-target-*, canonical-target-*). 8 bytes.
//   info bits 0-4   G' of the target
//        bits 5-8   q', category of the moved molecule in the target
//        bit  9     the source category vanishes (its only molecule moved)
//        bit  10    q' is a category the source did not have
//        bits 16-31 tmask of the target
// Records of a category: the m up moves (if tier < L) then the down moves of
// the channels with v_k > 0, in channel order.
struct Conn {
    uint32_t off;
    uint32_t info;
};
static_assert(sizeof(Conn) == 8, "Conn layout");

HEOM_HD uint32_t conn_G(uint32_t info) { return info & 31u; }
HEOM_HD uint32_t conn_q(uint32_t info) { return (info >> 5) & 15u; }
HEOM_HD bool conn_vanish(uint32_t info) { return (info >> 9) & 1u; }
HEOM_HD bool conn_new(uint32_t info) { return (info >> 10) & 1u; }
HEOM_HD uint32_t conn_tmask(uint32_t info) { return info >> 16; }

// Category in the target of the unmoved molecules of source category r, for
// a move of one molecule of source category q. Unmoved categories keep their
// vectors and relative order; the target list is the source list without q
// (if it vanished) with q' inserted (if new).
HEOM_HD int conn_remap(uint32_t info, int q, int r) {
    int r1 = r - ((conn_vanish(info) && r > q) ? 1 : 0);
    return r1 + ((conn_new(info) && r1 >= (int)conn_q(info)) ? 1 : 0);
}

// One workgroup tile: a run of whole patterns and the contiguous ranges of
// their variables, categories and hierarchy gather indices. 32 bytes.
// With compact tiles (Hermitian ADOs) the tile's threads cover only the
// entries of the upper triangle (row <= column) and the T_q of its blocks:
// nv counts those, and the decode record of thread t is at v0 + t of the
// records (its entry follows from the record and the block's header).
struct TileRec {
    uint32_t p0, np;     // patterns
    uint32_t v0, nv;     // unique variables (compact: the covered entries)
    uint32_t c0, nc;     // category records
    uint32_t g0, ng;     // gather indices (see expand_gathers)
};

// Hierarchy gather slots of one unique variable (Eqs. uvar-up, uvar-down):
// for each channel k the row molecule raised (slot k), lowered (M+k), the
// column molecule raised (2M+k), lowered (3M+k). A variable's live slots,
// in slot order, each hold the index of the target variable they read.
enum { KIND_Z = 0, KIND_X = 1, KIND_Y = 2, KIND_P = 3, KIND_S = 4 };
HEOM_HD uint32_t live_slots(int kind, bool chi, uint64_t vq, uint64_t vr, int M) {
    const bool rowmv = kind == KIND_X || kind == KIND_P || kind == KIND_S;
    const bool colmv = kind == KIND_Y || kind == KIND_S;
    uint32_t live = 0;
    for (int k = 0; k < M; ++k) {
        const bool nq = ((vq >> (8 * k)) & 0xffu) != 0, nr = ((vr >> (8 * k)) & 0xffu) != 0;
        live |= ((uint32_t)(rowmv && kind != KIND_P && chi) << k) | ((uint32_t)(rowmv && nq) << (M + k)) |
                ((uint32_t)(colmv && chi) << (2 * M + k)) | ((uint32_t)(colmv && nr) << (3 * M + k));
    }
    return live;
}
static_assert(sizeof(TileRec) == 32, "TileRec layout");

// Per-variable decode record, relative to the variable's tile:
//   x = p | A << 7 | B << 12 | isT << 17 | goff << 18
//   y = live hierarchy slots (bit j, slot order as in live_slots)
// p: pattern index within the tile (< VREC_MAX_NP; every block has at least
// four variables, so a 512-variable tile holds at most 128 patterns); A, B:
// row and column category + 1 (0 = cavity); isT: the variable is T_{A-1};
// goff: position of its first gather index in the tile's list.
struct VarRec {
    uint32_t x, y;
};
static_assert(sizeof(VarRec) == 8, "VarRec layout");
constexpr uint32_t VREC_MAX_NP = 128u, VREC_MAX_GOFF = 16383u;
HEOM_HD VarRec vrec_pack(uint32_t p, uint32_t A, uint32_t B, bool isT, uint32_t goff, uint32_t live) {
    return VarRec{p | (A << 7) | (B << 12) | ((uint32_t)isT << 17) | (goff << 18), live};
}

// Per-instance numeric parameters (device image header). 256-byte aligned.
struct InstParams {
    double g;          // single-molecule coupling
    double delta;      // eps - omega_c
    double kappa;      // cavity loss rate
    double term;       // terminator Delta
    double npool;      // N - d as double
    double Nd;         // N as double
    double inv_sqrtN;  // 1/sqrt(N)
    double cos_th, sin_th;  // polariton mixing angle (Eq. polariton-states)
    double nu[HEOM_MAX_M];
    double cr[HEOM_MAX_M], ci[HEOM_MAX_M];      // c_k
    double ccr[HEOM_MAX_M], cci[HEOM_MAX_M];    // c_check_k
    int32_t m, L, d, n_pat;
    uint32_t n_var, n_tiles, tile_vars, max_np, max_nc, max_ng, lds_bytes;
    uint32_t val_len;  // tile values held in LDS: tile_vars, or the largest compact tile's variables
    uint32_t compact;  // 1: compact tiles (see TileRec)
    uint32_t tcol;     // 1: column moves name transposed positions
    // byte offsets of the sections from the image base
    uint64_t off_lut, off_hdr, off_cat, off_gidx, off_tile, off_vrec, off_end;
};

struct HostTables {
    heom_problem prob;                 // copy (array pointers cleared)
    std::vector<double> c, cc, nu;
    int m = 0, L = 0, d = 0;
    int64_t N = 0;
    int32_t tile_vars = 256;
    // local vectors, nonzero, descending; id nv = zero vector
    std::vector<uint64_t> vecs;
    // patterns
    std::vector<PatHdr> hdr;
    std::vector<CatRec> cat;
    std::vector<Conn> conn;
    std::vector<uint32_t> conn_target;  // target pattern index per Conn
    std::vector<TileRec> tiles;         // workgroup tiles
    std::vector<uint32_t> gidx;         // per-tile lists of gather target indices
    std::vector<VarRec> vrec;           // per-variable decode records
    std::vector<uint16_t> vloc;         // compact tiles: tile-relative variable of each thread (host
                                        // only: the element counts and the tile checker; not in the image)
    uint32_t max_np = 0, max_nc = 0, max_ng = 0, lds_bytes = 0, val_len = 0;
    uint32_t lds_low = 0, lds_top = 0;      // LDS of a launch over the tiles below / in the top tier
    uint32_t lds_persist = 0;               // LDS of the persistent kernel (lists kept for every stage)
    uint32_t own_entries = 0;           // entries loaded as threads' own values (compact: the covered ones)
    uint32_t read_entries = 0;          // distinct positions one right-hand side reads (own values, gather targets)
    std::vector<uint16_t> pat_ids;      // flat: d dist ids + pool ids
    std::vector<uint32_t> pat_start;    // per pattern start in pat_ids, then end
    uint32_t n_var = 0;
    int max_G = 0;
    int64_t hier_gathers = 0;
    std::vector<double> lut;            // up[k][n] then dn[k][n]
    std::vector<unsigned char> image;   // device image (host staging)
    heom_tuning tune{0, 0, 0, 0, 0, 6, -1, 0};  // tile_vars unused here; persistent, xcd_map, max_workgroups, spin_limit, cache_policy, transposed, compact
    bool trcol = false;                 // column gathers name transposed positions (tune.transposed, or compact)
    bool compact = false;               // compact tiles (tune.compact): Hermitian ADOs only
    uint32_t top_tile = 0;              // first tile whose patterns are all in tier L
    void *dev = nullptr;                // uploaded image
    size_t dev_bytes = 0;
    bool uploaded = false;
    uint64_t id = 0;                    // unique per built handle (never reused in a process)
    uint64_t layout_gen = 0;            // advanced whenever the tiles, and so the image layout, change
};

// States of at least this many variables keep transposed copies by default.
constexpr uint32_t TRANSPOSED_MIN_VARS = 1u << 19;

// Sets the calling thread's error message (heom_last_error) and returns code.
int set_error(int code, const std::string &msg);

// host-side helpers implemented in tables.cpp
int build(const heom_problem *p, HostTables *t, std::string *err);
int set_params(HostTables *t, const heom_problem *p, std::string *err);
int make_tiles(HostTables *t, int tile_vars, std::string *err);
void expand_gathers(const HostTables &t, uint32_t p, std::vector<uint32_t> *out);
void pack_image(HostTables *t);
size_t image_bytes(const HostTables &t);
// [InstParams + coefficient tables] of problem p on the structure of t, laid
// out as the head of t's device image (bytes [0, off_hdr)).
int pack_params(const HostTables &t, const heom_problem *p, std::vector<unsigned char> *out, std::string *err);
size_t tier0_size(const HostTables &t);

inline uint32_t vcomp(uint64_t v, int k) { return (uint32_t)((v >> (8 * k)) & 0xffu); }

}  // namespace heom
