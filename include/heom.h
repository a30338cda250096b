/*
 * heom.h -- C ABI of libheom: symmetry-adapted HEOM for the permutationally
 * invariant Holstein-Tavis-Cummings model on AMD Instinct MI355X (gfx950).
 *
 * Method: Mondal & Huo, "Symmetry Adapted Hierarchical Equations of Motion
 * for Exact Simulations of Large Polariton Systems" (arXiv 2608.20657).
 * The library propagates the unique complex variables Z, X_q, Y_q, P_q,
 * S_{q,r}, T_q (Sec. V.A) of every canonical occupation pattern (Sec. IV)
 * with the matrix-free right-hand side of Sec. V.C and classical RK4.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Return value: HEOM_OK (0) or a negative HEOM_E_* code; the message of the
 *   last failure on the calling thread is heom_last_error(). No entry point
 *   aborts or throws. Asynchronous device errors surface at the next call that
 *   synchronizes or checks the stream.
 * - Pointers named *_dev are device memory owned by the caller (for example
 *   torch tensors); the library never allocates device memory itself. Host
 *   pointers are caller-owned and only read during the call unless stated.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream). All
 *   device work is enqueued on it; calls return before it completes.
 * - Complex numbers are interleaved (re, im) doubles (torch complex128) or
 *   floats (complex64).
 * - State vector layout (Eq. global-R): one block per canonical pattern, in
 *   the library's pattern order (tier ascending; within a tier the
 *   distinguished molecules' local vectors, smaller first, then the pool
 *   vectors compared entry by entry, larger first; local vectors are ordered
 *   by (|v|, v_0, .., v_{m-1})). A block is the (G+1)x(G+1) category matrix
 *   row-major with index 0 = cavity -- Z at (0,0), Y_q at (0,q), X_q at
 *   (q,0), P_q at (q,q), S_{q,r} at (q,r) -- followed by T_q for each
 *   category with M_q >= 2. Categories: the d distinguished molecules, the
 *   distinct nonzero pool vectors in pattern order, then the zero pool vector
 *   if present. Block length (G+1)^2 + h (Eq. uvar-count).
 */
#ifndef HEOM_H
#define HEOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HEOM_OK             0
#define HEOM_E_INVAL       -1   /* invalid argument */
#define HEOM_E_NOMEM       -2   /* host allocation failed */
#define HEOM_E_TOO_LARGE   -3   /* structure or buffer exceeds a stated limit */
#define HEOM_E_HIP         -4   /* a HIP runtime call failed */
#define HEOM_E_NONFINITE   -5   /* a non-finite observable was detected */
#define HEOM_E_UNSUPPORTED -6   /* outside the implemented parameter range */
#define HEOM_E_STATE       -7   /* call order violated (e.g. not uploaded) */
#define HEOM_E_TIMEOUT     -8   /* a grid barrier of the persistent kernel gave up waiting */

#define HEOM_MAX_M   8     /* exponentials per bath */
#define HEOM_MAX_L   63    /* hierarchy depth */
#define HEOM_MAX_G   16    /* categories per pattern */
#define HEOM_NOBS    10    /* observables per sample, see heom_observables */

#define HEOM_FP64    0     /* precision: complex FP64 throughout */
#define HEOM_FP32    1     /* precision: complex FP32 RK4 increments, FP64 state */
#define HEOM_HERMITIAN 2   /* flag OR-ed into precision: every ADO is Hermitian (see heom_propagate) */

/* One problem (Sec. II, Eqs. HS, BCF-exp, scaled-HEOM; Sec. VI.B for d).
 * Units are the caller's, with hbar = 1. */
typedef struct heom_problem {
    int64_t N;               /* molecules, >= 1 (Eq. basis) */
    int32_t m;               /* exponentials per local bath, 1..HEOM_MAX_M (Eq. BCF-exp) */
    int32_t L;               /* hierarchy depth, 0..HEOM_MAX_L (hard cutoff, Sec. II.C) */
    int32_t d;               /* distinguished molecules 1..d kept explicit, 0 <= d <= N (Eq. N-symmetric-pool) */
    int32_t reserved;        /* must be 0 */
    const double *c;         /* 2m doubles: (re, im) of c_k (Eq. BCF-exp) */
    const double *c_check;   /* 2m doubles: c_check_k, or NULL for conj(c_k) (real rates) */
    const double *nu;        /* m real decay rates nu_k >= 0 (Eq. tier-damping) */
    double eps;              /* molecular transition energy (Eq. HS) */
    double omega_c;          /* cavity frequency (Eq. HS) */
    double g;                /* single-molecule coupling (Eq. HS) */
    double kappa;            /* cavity loss rate: -(kappa/2){|c><c|, .} on every ADO */
    double terminator;       /* Ishizaki-Tanimura Delta: -Delta sum_i [Q_i,[Q_i, .]] (0 = off) */
} heom_problem;

typedef struct heom_tables heom_tables;   /* opaque host handle */

typedef struct heom_sizes {
    int64_t n_patterns;      /* canonical patterns (Eq. canonical-count-one for m = 1) */
    int64_t n_var;           /* unique variables = state vector length (Eq. Du-one) */
    int64_t n_conn;          /* connection records (one per pattern, category, channel, direction) */
    int64_t n_tiles;         /* workgroup tiles of whole patterns */
    int64_t n_categories;    /* sum of G over patterns */
    int64_t table_bytes;     /* device bytes heom_upload needs */
    int64_t work_bytes_fp64; /* device work bytes heom_propagate needs at HEOM_FP64 */
    int64_t work_bytes_fp32; /* device work bytes heom_propagate needs at HEOM_FP32 */
    int64_t tier0_size;      /* unique variables of the empty pattern */
    int32_t max_G;           /* largest category count */
    int32_t tile_vars;       /* variables per tile (workgroup size) */
    int64_t hier_gathers;    /* hierarchy reads of one right-hand side */
    int64_t rhs_work_bytes;  /* device work bytes heom_rhs needs (0 without transposed copies) */
    int32_t transposed;      /* 1 if column moves name transposed positions (see heom_tuning) */
    int32_t compact;         /* 1 if the tiles are compact (see heom_tuning) */
    int64_t stage_table_bytes; /* bytes of the table image one stage reads (compact tiles leave the
                                  record slots of their mirrored entries unread) */
    int64_t own_entries;     /* state entries one right-hand side loads as threads' own values
                                (n_var; compact tiles: the covered entries) */
    int64_t read_entries;    /* distinct state positions one right-hand side reads: own values and
                                hierarchy gather targets (element level; at 128-byte line level a
                                compact RHS still touches nearly every line of the state) */
} heom_sizes;

/* Build the pattern list, unique-variable layout and connection tables of
 * Sec. IV-V on the host (the precomputation of Sec. V.C.4). Reads `prob` and
 * its arrays during the call only. On success *out owns a new handle (free
 * with heom_free_tables). Errors: E_INVAL for out-of-range arguments,
 * E_UNSUPPORTED if a pattern has more than HEOM_MAX_G categories, E_TOO_LARGE
 * if the state exceeds 2^32-1 variables, E_NOMEM. No device call is made. */
int heom_build_tables(const heom_problem *prob, heom_tables **out);

/* Change the numeric parameters (c, c_check, nu, eps, omega_c, g, kappa,
 * terminator, and N when the structure is unchanged) of built tables. The
 * structure key (min(N, L+d+2), m, L, d) must be unchanged: beyond
 * saturation N enters only through M_0 (Sec. V.C.4). Takes effect at the next
 * heom_upload. Errors: E_INVAL if the structure would change. */
int heom_set_params(heom_tables *t, const heom_problem *prob);

/* Sizes of built tables (host only). */
int heom_table_info(const heom_tables *t, heom_sizes *out);

/* Copy the device image of the tables (pattern headers, categories,
 * connection records, tiles, coefficient look-up tables) into caller device
 * memory `dev` of `bytes` >= table_bytes, 256-byte aligned, on `stream`. The
 * handle remembers `dev`; the caller keeps it alive and unchanged while the
 * handle is used. The host staging copy stays owned by the handle. */
int heom_upload(heom_tables *t, void *dev, size_t bytes, void *stream);

/* Tier-0 unique variables of the pure initial state
 *   |psi> = a_c |c> + sum_{j<d} a_dist[j] |e_{j+1}> + a_pool sum_{pool i} |e_i>,
 * rho_S(0) = |psi><psi|, which is invariant under every relabeling of the
 * pool (Eqs. symmetric-initial-density, localized-residual-symmetry). This
 * covers the photon, bright, upper/lower polariton states (Eqs.
 * cavity-initial-uvar ... lower-polariton-initial), a localized excitation
 * and the cavity-site superposition of Sec. VII. Amplitudes are complex
 * (re, im) pairs; a_dist has 2d doubles (may be NULL if d = 0).
 * out: 2*tier0_size doubles (host). Mixtures follow by linearity. */
int heom_tier0_pure(const heom_tables *t, const double a_c[2], const double *a_dist,
                    const double a_pool[2], double *out);

/* Tier-0 unique variables of any operator A on the single-excitation space
 * that is invariant under relabelings of the pool molecules (Hermitian or
 * not, e.g. the representative operators |e_1><c|, |e_1><e_2| of the
 * linear reconstruction of Sec. VI.C, Table II). A is given by its
 * entries between representative basis states, R[a][b] = <a|A|b>, on the
 * d+3 slots 0 = cavity, 1..d = distinguished molecules e_1..e_d, d+1 = a
 * pool molecule, d+2 = a second pool molecule: R is (d+3)x(d+3) complex,
 * row-major (re, im) pairs, host. Read are the entries among slots
 * 0..d+1 and R[d+1][d+2] (the coherence between two different pool
 * molecules); the others follow from pool invariance and are ignored.
 * out: 2*tier0_size doubles (host). */
int heom_tier0_operator(const heom_tables *t, const double *R, double *out);

/* Inverse of heom_tier0_operator: the (d+3)x(d+3) slot matrix R (host,
 * every entry written; entries of slot d+2 mirror slot d+1 except the
 * pool-pool coherence) of the operator whose tier-0 block is `tier0`
 * (2*tier0_size doubles, host), e.g. rho_S(t) read back from a propagated
 * state. Entries of absent slots (a pool with fewer than two molecules)
 * are 0. */
int heom_tier0_expand(const heom_tables *t, const double *tier0, double *R);

/* Dense rho_S(t) of one output time by linear reconstruction (Sec. VI.C,
 * Table II; Eqs. Gt-linearity, Gt-covariance, arbitrary-initial-expansion):
 * the reduced map is linear in rho_S(0) and covariant under relabelings, so
 * rho_S(t) is the sum over the five operator types of rho_S(0) of the
 * representatives' responses, relabeled and weighted by rho_S(0)'s entries
 * of that type:
 *   type |c><c|       weight rho0[c][c]         representative d = 0
 *   type |e_k><c|     weights rho0[k][c]        representative |e_1><c|, d = 1
 *   type |c><e_k|     weights rho0[c][k]        representative |c><e_1|, d = 1
 *   type |e_k><e_k|   weights rho0[k][k]        representative |e_1><e_1|, d = 1
 *   type |e_k><e_l|   weights rho0[k][l], k!=l  representative |e_1><e_2|, d = 2
 * N: molecules, 1..HEOM_RECON_MAX_N. rho0_dev: device, (N+1)x(N+1) complex
 * doubles, row-major, index 0 = cavity, 1..N = molecules. R: host, the five
 * responses at this time as slot matrices (heom_tier0_expand of each
 * representative's propagated tier-0 block), complex row-major (re, im)
 * pairs packed in the order above: 3x3, 4x4, 4x4, 4x4, 5x5
 * (HEOM_RECON_R_DOUBLES doubles); read during the call only. mask: bit t set
 * = type t (order above) contributes; HEOM_RECON_CE_ADJOINT with bit 2: the
 * |c><e_1| response is taken as the adjoint of the |e_1><c| one (Eq.
 * adjoint-preservation; valid when c_check_k = conj(c_k)) and R's third
 * block is not read. work_dev: device, at least heom_reconstruct_work_bytes(N)
 * bytes (row and column sums of rho0's molecule block, totals), overwritten.
 * out_dev: device, (N+1)x(N+1) complex doubles, overwritten; may not alias
 * rho0_dev or work_dev. Stream-ordered on `stream`, nothing allocated.
 * Errors: HEOM_E_INVAL (N out of range, NULL pointer, a device buffer not
 * 16-byte aligned, unknown mask bits, the adjoint flag without bit 2),
 * HEOM_E_TOO_LARGE (work too small). */
#define HEOM_RECON_MAX_N 4096
#define HEOM_RECON_R_DOUBLES 164
#define HEOM_RECON_CE_ADJOINT 32u
int heom_reconstruct_dense(int64_t N, const void *rho0_dev, const double *R, uint32_t mask, void *work_dev,
                           size_t work_bytes, void *out_dev, void *stream);
/* Work bytes heom_reconstruct_dense needs for N molecules (0 if N is out of range). */
size_t heom_reconstruct_work_bytes(int64_t N);

/* Factorized initial condition (Eqs. factorized-initial-zero/-higher):
 * y_dev (n_var complex128) gets the tier-0 variables `tier0` (host,
 * 2*tier0_size doubles) and zeros elsewhere. Requires heom_upload. */
int heom_init_state(const heom_tables *t, const double *tier0, void *y_dev, void *stream);

/* One matrix-free right-hand side dy = M_u y (Eq. uvar-propagator): the
 * commutator with H_S through grouped multiplicity sums (Eqs.
 * grouped-row-sum, grouped-column-sum, HZ, HX), -Gamma_Lambda damping
 * (Eq. Gamma-Lambda-one and its m-channel form), cavity loss, the terminator
 * if set, and the hierarchy couplings read through the connection records
 * (Eqs. uvar-up, uvar-down). y_dev and dy_dev: n_var values each, distinct.
 *   precision HEOM_FP64: complex128 in and out, FP64 arithmetic.
 *   precision HEOM_FP32: complex64 in and out (the FP32 bulk of
 *     heom_propagate); multiplicities, square-root weights, damping and the
 *     arithmetic are FP64, the result is rounded to complex64 once.
 *   | HEOM_HERMITIAN: the caller asserts that every ADO of y is Hermitian
 *     (see heom_propagate). Tables with transposed column targets then read
 *     the conjugated mirrored entry of y for column moves; compact tables
 *     (heom_tuning.compact), which need this flag, compute each block's upper
 *     triangle and T_q and write every entry of dy (the lower triangle as
 *     the conjugates). Errors: E_INVAL if c_check != conj(c).
 * work_dev: scratch for the transposed copy of y, needed only by tables with
 * transposed column targets without HEOM_HERMITIAN (rhs_work_bytes; may be
 * NULL otherwise). Requires heom_upload. Errors: E_TOO_LARGE if work_bytes
 * is too small, E_STATE for compact tables without HEOM_HERMITIAN. */
int heom_rhs(const heom_tables *t, const void *y_dev, void *dy_dev, void *work_dev, size_t work_bytes,
             int precision, void *stream);

/* Propagate y_dev in place by nsteps classical RK4 steps of size dt (the
 * integrator of Sec. VII.E). The linear generator is autonomous, so a step
 * is evaluated as y + h M (y + h/2 M (y + h/3 M (y + h/4 M y))), the same
 * degree-4 polynomial in hM as the k1..k4 form, with four fused
 * right-hand-side + combination stages.
 *   precision HEOM_FP64: all stages in complex FP64; work_dev holds
 *     work_bytes_fp64 bytes (two state vectors, and with transposed copies
 *     (heom_tuning) three more: the copies of y and of the two).
 *   precision HEOM_FP32: y stays complex FP64; the increments
 *     u1 = h/4 M y, u2 = h/3 M (y + u1), u3 = h/2 M (y + u2) are stored as
 *     complex FP32, and each later stage gathers only its FP32 increment,
 *     using linearity (M y = (4/h) u1); y += h M (y + u3) is applied in
 *     place. Multiplicities, square-root weights, damping, the arithmetic
 *     and the combination with y stay FP64; work_dev holds work_bytes_fp32
 *     bytes.
 * precision | HEOM_HERMITIAN: the caller asserts that every ADO of y is
 *   Hermitian (rho_n^dagger = rho_n: a Hermitian rho_S(0) propagated with
 *   c_check = conj(c), Eq. adjoint-preservation), so that the entry a
 *   column-molecule move needs is the complex conjugate of the entry with
 *   row and column exchanged. Tables with transposed copies (heom_tuning)
 *   then read that mirrored entry of y's own row-major layout and keep no
 *   copies; other tables ignore the flag. Results agree with the general
 *   path to rounding (the two mirrored entries are computed by different
 *   threads), not bitwise. Errors: E_INVAL if c_check != conj(c).
 * If obs_every > 0, obs_dev (device, (nsteps/obs_every + 1)*HEOM_NOBS
 * doubles) receives the observables of heom_observables before the first
 * step and after every obs_every steps. obs_dev may be NULL if obs_every is 0.
 * Requires heom_upload. */
int heom_propagate(const heom_tables *t, void *y_dev, void *work_dev, size_t work_bytes,
                   double dt, int64_t nsteps, int64_t obs_every, double *obs_dev,
                   int precision, void *stream);

/* Bytes of the library's own work array used by heom_propagate_noalloc:
 * 64 MiB on each GPU the library runs on, held until the process ends. Tables
 * whose work_bytes_fp64 exceed it (about 2.09 M unique variables, or 0.84 M
 * with transposed copies) are refused. */
#define HEOM_NOALLOC_WORK_BYTES ((size_t)64 << 20)

/* heom_propagate without a caller work buffer, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation. Arguments and results as heom_propagate
 * (the caller still passes y_dev and obs_dev); the stage vectors and the
 * control area live in a static device array of HEOM_NOALLOC_WORK_BYTES in
 * the library, so this call allocates nothing (no hipMalloc, no hipFree).
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams or threads) race and must be serialized by the caller;
 * the array keeps the last call's contents, and what must start at zero is
 * cleared by each call with a fill kernel. heom_work_status cannot inspect
 * this array (the caller has no pointer to it); a non-finite result shows in
 * the observables. Errors: as heom_propagate, plus E_TOO_LARGE if the tables
 * need more than HEOM_NOALLOC_WORK_BYTES of work memory. */
int heom_propagate_noalloc(const heom_tables *t, void *y_dev, double dt, int64_t nsteps, int64_t obs_every,
                           double *obs_dev, int precision, void *stream);

/* Observables of the physical reduced density operator, the tier-0 block
 * (Sec. V.D, generalized to d distinguished molecules by grouping each
 * category with its multiplicity). obs_dev receives HEOM_NOBS doubles:
 *   0 Tr rho_S (real part)   1 P_cav = Z        2 P_exc = sum_q M_q P_q
 *   3 P_B                    4 P_D = P_exc - P_B
 *   5 P_+                    6 P_-  (Eq. polariton-states, theta = atan2(2 g sqrt N, omega_c - eps)/2)
 *   7 population of molecule 1   8 population of molecules 2..N   9 Im Tr rho_S
 * (Eqs. trace-uvar, Pcav-uvar, Pexc-uvar, PB-uvar, PD-uvar, Pplus-uvar,
 * Pminus-uvar). Requires heom_upload. */
int heom_observables(const heom_tables *t, const void *y_dev, double *obs_dev, void *stream);

/* Serialized canonical form of the tables, for bit-exact comparison on the
 * host. Writes int64 values to `out` (capacity `cap` entries, may be NULL to
 * query) and the required count to *needed:
 *   [n_patterns, n_var, m, d]
 *   per pattern: [offset, G, tier] then per category [dist label or -1,
 *     multiplicity, v_0 .. v_{m-1}]
 *   then per pattern, per category q, per channel k, up (if tier < L) then
 *   down (if v_k(q) > 0): [target pattern, q', r'_0 .. r'_{G-1}] where q' is
 *   the moved molecule's category in the target and r'_r the category of
 *   the unmoved members of source category r (-1 if none remain). */
int heom_export_layout(const heom_tables *t, int64_t *out, size_t cap, size_t *needed);

/* Coefficient look-up tables as used by the kernels (host copy):
 * out[k*(L+1) + n] = sqrt((n+1)|c_k|) (up, n = 0..L) followed by
 * out[m*(L+1) + k*(L+1) + n] = sqrt(n/|c_k|) (down, n = 0..L); zero for a
 * channel with c_k = 0. Capacity cap doubles; *needed = 2m(L+1). */
int heom_export_coefficients(const heom_tables *t, double *out, size_t cap, size_t *needed);

/* Launch configuration of the kernels (the autotuner's knobs). */
typedef struct heom_tuning {
    int32_t tile_vars;       /* variables per workgroup tile: 64, 128, 256 or 512 (0 = keep) */
    int32_t persistent;      /* 1: heom_propagate runs all steps in one cooperative launch with a
                                grid barrier after each stage (check heom_work_status afterwards:
                                a barrier that times out leaves the state mid-step); 0 (default):
                                one launch per stage; 2: persistent when the state has at most
                                256 tiles; 3: persistent, the grid barrier counting arrivals in
                                per-group counters instead of every workgroup polling every
                                workgroup's flag */
    int32_t xcd_map;         /* 1: map workgroups to tiles so each XCD streams a contiguous run */
    int32_t max_workgroups;  /* cap on resident workgroups of the persistent launch (0 = occupancy limit) */
    int32_t spin_limit;      /* polls before a grid barrier gives up (0 = default, about 4 s) */
    int32_t cache_policy;    /* streaming (non-temporal) hints: bit 0 own-value loads, bit 1 loads of
                                the RK4 base vector, bit 2 stores (default 6) */
    int32_t transposed;      /* transposed copies: 1 on, 0 off, -1 (default) on for states of
                                2^19 or more variables. With copies on, every stage also writes its
                                output with each block's category matrix transposed, and the
                                column-molecule moves (Eqs. uvar-up, uvar-down, column terms) gather
                                from that copy, where the entries one column move reads are
                                contiguous; work_bytes grow from 32 to 80 bytes per variable and the
                                persistent launch is not used. */
    int32_t compact;         /* 1: compact tiles for Hermitian ADOs (default 0). Each block's lower
                                triangle (row > column) is the conjugate of its upper triangle, so
                                the threads cover only the entries with row <= column and the T_q;
                                each writes its entry and the conjugate into the mirrored position,
                                and the column sums of the Hamiltonian bracket are taken as the
                                conjugates of the row sums (Eqs. grouped-row-sum,
                                grouped-column-sum). About half the gathers and arithmetic of a
                                stage. Implies transposed column targets, with no copies (work_bytes
                                stay 32 per variable). The upper triangle of y is taken as the
                                state. Only heom_propagate / heom_batch_propagate with
                                HEOM_HERMITIAN run on such tables (E_STATE otherwise, heom_rhs
                                included). */
} heom_tuning;

/* Set or read the launch configuration. A new tile_vars or a change of the
 * effective `transposed` rebuilds the tiles and needs a new heom_upload
 * (table_bytes and the work sizes may change). Results do not
 * depend on the configuration (every variable has one writer, and the sum
 * order inside a variable is fixed). Errors: E_INVAL if tile_vars is not
 * allowed or smaller than the largest pattern block. */
int heom_set_tuning(heom_tables *t, const heom_tuning *tuning);
int heom_get_tuning(const heom_tables *t, heom_tuning *tuning);

/* Wait for `stream` and report how the last heom_propagate that used this
 * work buffer ended: HEOM_OK; HEOM_E_TIMEOUT if a grid barrier of the
 * persistent kernel gave up (the state is then invalid); HEOM_E_NONFINITE if
 * the tier-0 block of the final state or an observable row written by that
 * call is NaN or infinite (an unstable dt, for instance). heom_propagate
 * itself returns before the device finishes, so it cannot report these.
 * Reads 8 bytes of work_dev. */
int heom_work_status(const heom_tables *t, const void *work_dev, size_t work_bytes, void *stream);

/* Release a handle (NULL is allowed). Device memory is the caller's. */
void heom_free_tables(heom_tables *t);

/* ---------------------------------------------------------------------
 * Many independent problems (the batched and served workloads).
 *
 * Problems with the same structure key (min(N, L+d+2), m, L, d) share one
 * uploaded structure (Sec. V.C.4: beyond saturation only M_0 and the
 * numeric parameters differ). Each problem then needs only a parameter
 * block: heom_params_bytes bytes written by heom_upload_params.
 * ------------------------------------------------------------------- */

/* Bytes of one parameter block (scalars and coefficient look-up tables). */
int heom_params_bytes(const heom_tables *t, size_t *bytes);

/* Write the parameter block of `prob` on the structure of `t` into caller
 * device memory `dev` (256-byte aligned, >= heom_params_bytes), synchronously
 * on `stream`. Errors: E_INVAL if prob's structure key differs from t's. */
int heom_upload_params(const heom_tables *t, const heom_problem *prob, void *dev, size_t bytes, void *stream);

typedef struct heom_batch heom_batch;   /* opaque host handle */

/* An empty batch with `capacity` slots. */
int heom_batch_create(int32_t capacity, heom_batch **out);

/* Put a problem into a slot (replacing what was there): its structure `t`
 * (uploaded, kept alive and unmoved by the caller), its parameter block
 * (written by heom_upload_params for t and t's current tiles; NULL = the
 * parameters in t's own image, wherever t is uploaded at the next commit),
 * its state y_dev (t's layout,
 * complex128, initialized e.g. by heom_init_state), a work buffer of at least
 * work_bytes_fp64 bytes, its time step, and optionally an observable buffer
 * of obs_capacity samples of HEOM_NOBS doubles: sample j holds the
 * observables after j*obs_every steps of this slot; sample 0, the initial
 * state evaluated with the slot's own parameters, is written by the next
 * heom_batch_commit, so y_dev must be initialized before it. All pointers
 * are caller device memory. The slot's step count restarts at 0. Takes
 * effect at the next heom_batch_commit. */
int heom_batch_set_slot(heom_batch *b, int32_t slot, const heom_tables *t, const void *params_dev, void *y_dev,
                        void *work_dev, size_t work_bytes, double dt, double *obs_dev, int64_t obs_every,
                        int64_t obs_capacity);

/* Empty a slot (its buffers are no longer touched after the next commit). */
int heom_batch_clear_slot(heom_batch *b, int32_t slot);

/* Device bytes heom_batch_commit needs for the current slots. */
int heom_batch_device_bytes(const heom_batch *b, size_t *bytes);

/* Upload the slot records and the tile list (grouped by m) into caller
 * device memory (256-byte aligned, >= heom_batch_device_bytes), and write
 * observable sample 0 of every slot that has not stepped yet, synchronously
 * on `stream`. Required after any set/clear, and after re-tuning or
 * re-uploading a slot's tables. Errors: E_STATE if a slot's tables are not
 * uploaded, or its parameter block was not written by heom_upload_params for
 * those tables and their current tiles (re-tuning tiles makes earlier blocks
 * stale); E_TOO_LARGE if a slot's work buffer is smaller than its tables'
 * work_bytes now. */
int heom_batch_commit(heom_batch *b, void *dev, size_t bytes, void *stream);

/* Advance every occupied slot by nsteps RK4 steps of its own dt (the same
 * fused stages as heom_propagate; one launch per stage and per m covers the
 * tiles of all slots; slots whose tables keep transposed copies get the copy
 * of y made at the start of each call). Each problem's trajectory is bitwise the same as with
 * heom_propagate alone (no slot reads another slot's memory). precision as
 * in heom_propagate, HEOM_HERMITIAN included (E_INVAL unless every slot's
 * parameters have c_check = conj(c)). A batch with one occupied slot runs
 * heom_propagate's stage launches with that slot's parameter block (unless a
 * HIP graph replays the call, heom_batch_set_graph). Errors: E_STATE if not
 * committed since the last change. Non-finite states are reported by
 * heom_batch_status. */
int heom_batch_propagate(heom_batch *b, int64_t nsteps, int precision, void *stream);

/* Replay whole groups of `steps` RK4 steps from a HIP graph captured on the
 * stream of heom_batch_propagate (0, the default, launches every kernel
 * directly; at most 4096). Small problems are bound by the host's launch
 * rate, which a replayed graph avoids. The graph is captured at the first
 * heom_batch_propagate with at least `steps` steps after a commit (or a
 * change of precision or of this setting) and replayed for as many whole
 * groups as fit; the remaining steps are launched directly. The step
 * index that selects observable rows is kept on the device, so replays and
 * direct launches give bitwise the same results. Not used on the null
 * stream, which cannot be captured. */
int heom_batch_set_graph(heom_batch *b, int32_t steps);

/* Launch shape: the batch's tiles fall into groups of one m, tile size and
 * tier class. The smallest groups with m <= 4 and at most max_tiles/8
 * tiles each, up to max_tiles tiles in all, are run as one launch per RK4
 * stage (each workgroup picks the kernel
 * variant of its slot's m and tier class); every other group has its own
 * launch. Small problems are bound by the latency of dependent launches,
 * which the merged launch avoids; large groups keep their own kernels, whose
 * register use allows more waves. 0 = one launch per group. Default 16384.
 * Results are bitwise the same either way. Takes effect at the next
 * heom_batch_commit (required). */
int heom_batch_set_merge(heom_batch *b, int32_t max_tiles);

/* Launch shape: the order of the tiles in the groups that run one workgroup
 * per slot and tile. 0: slot by slot. tiles > 0: the slots that use the same
 * uploaded structure take turns, `tiles` consecutive tiles each, so that
 * workgroups resident together read the same connection tables (beyond
 * saturation problems of one structure key share them, Sec. V.C.4) and one
 * fetch of them serves several problems. Default 32. Results are bitwise the
 * same either way. Takes effect at the next heom_batch_commit (required). Errors: E_INVAL
 * if tiles < 0. */
int heom_batch_set_interleave(heom_batch *b, int32_t tiles);

/* Wait for `stream` and report whether any occupied slot's tier-0 block
 * became NaN or infinite during a heom_batch_propagate since the last
 * heom_batch_commit (which clears the flags): HEOM_E_NONFINITE if so, else
 * HEOM_OK. slot_flags (host, may be NULL when cap is 0) receives 1 or 0 for
 * the first `cap` slots. Errors: E_STATE if not committed since the last
 * change. */
int heom_batch_status(const heom_batch *b, int32_t *slot_flags, int32_t cap, void *stream);

/* Launch shape: with max_slots = 2, slots that use the same uploaded
 * structure (the same heom_tables, each with its own parameter block) are
 * computed in pairs, side by side in one workgroup of twice the tile size:
 * each half computes the tile for one slot, and the tile's metadata (pattern
 * headers, categories, gather lists) is staged into LDS once for both
 * (beyond saturation the structure is N-independent, Sec. V.C.4, so problems
 * of one structure key read the same tables). Structures with 512-variable
 * tiles, or whose pair would need more than 64 KiB of LDS, and an odd slot
 * out keep one workgroup per slot. 1 = off (default). Applies to the groups
 * that are not merged (heom_batch_set_merge). Results are bitwise the same
 * either way. Takes effect at the next heom_batch_commit (required). Errors:
 * E_INVAL unless max_slots is 1 or 2. */
int heom_batch_set_share(heom_batch *b, int32_t max_slots);

/* Steps a slot has taken since it was set. */
int heom_batch_slot_steps(const heom_batch *b, int32_t slot, int64_t *steps);

/* Release a batch handle (NULL is allowed). */
void heom_batch_free(heom_batch *b);

/* Message of the last failure on this thread ("" if none). */
const char *heom_last_error(void);

/* Library version string. */
const char *heom_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HEOM_H */
