/*
 * wick.h -- C ABI of the MI355X (gfx950) library for light-nucleus two-point
 * correlators by Wick contraction with baryon blocks.
 *
 * What is computed (arXiv 2411.08962):
 *   C(t) = sum over Wick terms of  coef * prod_{a=1..A} B_{k_a}(t)[iota_a]
 * where the baryon blocks are (Eq. 2.4, App. D)
 *   B_k(t)[i1,i2,i3] = sum_x sum_j w_k(j) S_f1(x,t)[j1,i1] S_f2(x,t)[j2,i2] S_f3(x,t)[j3,i3]
 * antisymmetrised in the two same-flavor source slots (as Eq. 2.4 writes it),
 * and the signed, deduplicated term table comes from the host planner
 * (randomised identity testing, Sec. 3.2 and App. C, done exactly in F_p).
 *
 * Conventions
 *   - spin-color index chi = 3*spin + color in [0, 12) (Sec. 2.1).
 *   - propagator S[cfg][t][z][y][x][j][i]: j = sink index (row), i = source
 *     index (column); complex128 (WICK_C128) or complex64 (WICK_C64),
 *     interleaved (re, im). One array per flavor (u, d).
 *   - quark flavors: 0 = u, 1 = d.
 *   - a block kind has flavors (f, g, f) with f != g (nucleon-like: two slots
 *     of one flavor, slots 1 and 3). Its block is stored antisymmetrised in
 *     compact form: B[c] with c = pair(i1,i3)*12 + i2 for i1 < i3, where
 *     pair(i1,i3) = i3*(i3-1)/2 + i1 (66 pairs, 792 entries per kind), and
 *     B[c] = Braw[i1,i2,i3] - Braw[i3,i2,i1].
 *   - block array: double B[n_cfg][T][n_kinds][792][2] (device memory).
 *   - correlator array: double C[n_cfg][T][2] (device memory), already
 *     multiplied by the operator's scale.
 *
 * Ownership and errors
 *   - The caller owns every array passed in. The library owns plans and an
 *     internal device workspace (released by wick_shutdown or at exit).
 *   - Every GPU entry point validates its arguments on the host first and
 *     returns WICK_EINVAL before launching anything. GPU work is queued on
 *     the given stream (a hipStream_t; NULL = default stream) and is
 *     asynchronous unless stated otherwise. HIP failures return WICK_EHIP.
 *     No C++ exception crosses this interface; wick_last_error() returns a
 *     thread-local message for the last failing call.
 *   - Plans are immutable after creation and may be used from several
 *     threads and streams at once.
 */
#ifndef WICK_H
#define WICK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wick_plan_s *wick_plan_t;
typedef void *wick_stream_t; /* a hipStream_t */

typedef enum {
    WICK_OK = 0,
    WICK_EINVAL = -1,      /* bad argument (shape, pointer, enum, index) */
    WICK_ENOMEM = -2,      /* host or device allocation failed */
    WICK_EHIP = -3,        /* a HIP call failed */
    WICK_EUNSUPPORTED = -4,/* valid input this build does not handle */
    WICK_ECORRUPT = -5,    /* plan file checksum / version mismatch */
    WICK_ETOOBIG = -6      /* a size exceeds an internal limit */
} wick_status;

typedef enum { WICK_C128 = 0, WICK_C64 = 1 } wick_dtype;

/* Arithmetic of the block build. The term sum and C(t) are always FP64. */
typedef enum {
    WICK_P64 = 0,  /* FP64 MFMA, FP64 accumulation */
    WICK_P32 = 1,  /* FP32 MFMA on power-of-two scaled tiles, FP64 across chunks */
    WICK_PB3 = 2,  /* split-BF16: 2 limbs, 3 products, FP32 MFMA accumulate */
    WICK_PB6 = 3   /* split-BF16: 3 limbs, 6 products, FP32 MFMA accumulate */
} wick_precision;

/* One nucleon-like operator with a fixed sink spin: its quark flavors and its
 * nonzero weights w(j1, j2, j3) as exact Gaussian integers (Eq. 2.2-2.3 and
 * the projected forms of Sec. 3.3 are all of this form). */
typedef struct {
    int32_t flavor[3];
    int32_t n_w;
    const int8_t *j;       /* [n_w][3] sink spin-color indices */
    const int64_t *w_re;   /* [n_w] */
    const int64_t *w_im;   /* [n_w] */
} wick_kind;

/* A nuclear operator: sums of products of A kinds with Gaussian-integer
 * coefficients, at the sink and at the source (Sec. 3.1, Eq. 2.7 with the
 * coefficient tensor written as products of nucleon weights). */
typedef struct {
    int32_t A;                   /* nucleons, 1..5 */
    int32_t n_kinds;
    const wick_kind *kinds;
    int32_t n_snk;
    const int32_t *snk_kind;     /* [n_snk][A] kind of each sink nucleon */
    const int64_t *snk_re, *snk_im;
    int32_t n_src;
    const int32_t *src_kind;     /* [n_src][A] kind (weights) of each source nucleon */
    const int64_t *src_re, *src_im;
    double scale;                /* real factor applied to C (irrational normalisations) */
    uint64_t hash_seed;          /* seed of the random F_p propagators (0: default) */
    int32_t hash_trials;         /* independent identity tests (0: default 2) */
    int32_t hash_sites;          /* sites of the toy lattice, >= A (0: default 8) */
} wick_nucleus_desc;

/* ---------------------------------------------------------------- planning */

/* Build the deduplicated Wick-term table of an operator on the host
 * (Sec. 3.2 "computation of non-redundant minimal set", App. C identity
 * testing): antisymmetrise the source per flavor, enumerate every
 * assignment of source indices to block slots with its sign, evaluate each
 * term on random F_p propagators and merge terms whose values agree up to
 * sign in every trial, summing their integer coefficients exactly.
 * Deterministic for a given desc. Returns WICK_EINVAL for inconsistent
 * flavor contents, WICK_EUNSUPPORTED for a sink kind that is not
 * nucleon-like, WICK_ETOOBIG past internal limits. */
wick_status wick_plan(const wick_nucleus_desc *desc, wick_plan_t *out);

/* Built-in operators of Sec. 3.3: "1H" (proton, spin J), "2H", "3He",
 * "3H", "4He"; also "2H-" and "2H0" (the deuteron operator with P_- and with
 * no projector). J is the spin of the last nucleon where the operator has one
 * (3He, 3H) or the proton's sink and source spin (1H); ignored otherwise. */
wick_status wick_plan_std(const char *nucleus, int32_t J, wick_plan_t *out);

/* An off-diagonal correlator of built-in operators: `sink` (spin J_sink) at
 * the sink and `source` (spin J_source) at the source, normalised by
 * sqrt(scale_sink * scale_source); one element of a correlation matrix
 * (Eq. E1) planned on its own. */
wick_status wick_plan_std_pair(const char *sink, int32_t J_sink, const char *source, int32_t J_source,
                               wick_plan_t *out);

/* Sizes: A, number of block kinds, number of terms. */
wick_status wick_plan_info(wick_plan_t plan, int32_t *A, int32_t *n_kinds, int64_t *n_terms);

/* Planner statistics: enumerated terms, source groups, table terms, and the
 * union bound on a false merge (Thm. 1 of App. C with the trials used). */
wick_status wick_plan_stats(wick_plan_t plan, int64_t *n_enumerated, int64_t *n_groups,
                            int64_t *n_terms, double *false_merge_bound);

/* Work of the plan's term sum per time slice, for pricing the term-sum
 * kernel (Eq. 2.9's signed sum over the deduplicated table, Sec. 3.2). form:
 * 0 plain, 1 packed (one word per term), 2 segmented with a coefficient
 * palette, 3 segmented with integer coefficients, 4 factored (A = 4: each
 * list of terms shared by several index prefixes is summed once and
 * weighted by the sum of its prefix products); words2 / words1: table words
 * gathering two leaves / one leaf (padding not counted; for forms 0 and 1,
 * words1 = n_terms); segments: lanes holding a segment (forms 2-4). Builds
 * the table on the host when the plan has not been used on a device yet
 * (seconds for 4He). Any output pointer may be NULL. */
wick_status wick_plan_sum_work(wick_plan_t plan, int32_t *form, int64_t *words2, int64_t *words1,
                               int64_t *segments);

/* Copy the table out (host arrays): kidx[A][n_terms] with
 * kidx = kind*792 + c, and coef[n_terms][2] (scale included). */
wick_status wick_plan_table(wick_plan_t plan, uint16_t *kidx, double *coef);

/* Block kind k of a plan: block kinds are the desc's kinds used at the sink,
 * numbered in order of first use in the sink patterns (the kind axis of B
 * and the kind part of kidx). Writes its slot flavors and its number of
 * weight entries n_w; if j / w_re / w_im are not NULL, also its weights as
 * given in the desc (host arrays of n_w*3, n_w, n_w entries). */
wick_status wick_plan_kind(wick_plan_t plan, int32_t k, int32_t flavor[3], int32_t *n_w,
                           int8_t *j, int64_t *w_re, int64_t *w_im);

/* Store / reuse a plan (the look-up table of App. C): a versioned file with a
 * checksum; load returns WICK_ECORRUPT on any mismatch. */
wick_status wick_plan_save(wick_plan_t plan, const char *path);
wick_status wick_plan_load(const char *path, wick_plan_t *out);
void wick_plan_destroy(wick_plan_t plan);

/* Important-term truncation (Sec. 5 "distributions of terms in determinants
 * and blocks", App. D): the few terms with large values carry the correlator
 * and which terms they are is fixed by the operator, so they can be chosen
 * once from blocks of a small calibration lattice (even a single site) and
 * reused on any ensemble with the same kernels.
 *   B_cal: host double [n_slices][n_kinds][792][2], blocks as written by
 *          wick_blocks (any calibration configurations and time slices,
 *          e.g. [n_cfg][T] flattened); n_slices >= 1.
 *   keep_fraction in (0, 1]: the new plan keeps
 *          M = clamp(ceil(keep_fraction * N - 1e-6), 1, N) of the N terms.
 * Ranking: term n has value v_n(s) = coef_n prod_a B_cal[s][kidx_{a,n}] on
 * slice s; with m_s = max_n |v_n(s)|, its score is the largest
 * |v_n(s)| / m_s over the slices with m_s > 0. The M highest scores are kept
 * (equal scores in table order) and stay in table order, with their
 * coefficients unchanged. If dropped is not NULL it receives, per slice
 * (host double [n_slices]), the sum of |v_n(s)| over the dropped terms: a
 * bound on |C_full(s) - C_kept(s)| on the calibration slices.
 * *out is a new plan (destroy it with wick_plan_destroy); the input plan is
 * not changed. Blocking, host only. Errors: WICK_EINVAL (null pointers,
 * n_slices < 1, keep_fraction outside (0, 1] or NaN, non-finite blocks),
 * WICK_ENOMEM. */
wick_status wick_plan_truncate(wick_plan_t plan, const double *B_cal, int32_t n_slices,
                               double keep_fraction, wick_plan_t *out, double *dropped);

/* ------------------------------------------------------------ GPU compute */

/* Baryon blocks of every kind of the plan on every configuration and time
 * slice (Eq. 2.4): S_u, S_d are device arrays [n_cfg][T][Z][Y][X][12][12]
 * of dtype (sink index first), 16-byte aligned; dims = {X, Y, Z, T}; B is
 * device double [n_cfg][T][n_kinds][792][2], entry c = pair(i1, i3)*12 + i2
 * with pair(i1, i3) = i3(i3-1)/2 + i1, i1 < i3 (the block antisymmetrised in
 * its two same-flavor slots). Sums over sites in a fixed order
 * (deterministic: bitwise repeatable). Errors: WICK_EINVAL (null or
 * misaligned pointers, bad sizes), WICK_EUNSUPPORTED (split precision for
 * kinds not of nucleon form), WICK_ENOMEM, WICK_EHIP. Asynchronous on
 * stream; the caller keeps S_u, S_d and B alive until it completes. */
wick_status wick_blocks(wick_plan_t plan, const void *S_u, const void *S_d, wick_dtype dtype,
                        const int32_t dims[4], int32_t n_cfg, wick_precision prec,
                        wick_stream_t stream, double *B);

/* C[cfg][t] = sum_n coef_n prod_a B[cfg][t][kidx_{a,n}] in FP64 (Eq. 2.6 /
 * App. D), deterministic tree reduction. B as written by wick_blocks. */
wick_status wick_contract(wick_plan_t plan, const double *B, int32_t n_cfg, int32_t T,
                          wick_stream_t stream, double *C);

/* wick_contract for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and launch shape, so C is bitwise equal to wick_contract's,
 * but the partial sums go to a static device array of 131072 complex FP64
 * entries (2 MiB) that the library holds on each GPU until the process ends,
 * and nothing is allocated (no hipMalloc / hipFree, no profiling events).
 * Preconditions: the plan's table is already on the current device (one
 * wick_contract or wick_blocks call with this plan on this device, made
 * beforehand, puts it there; else WICK_EINVAL). A launch that needs more
 * than 131072 partial sums (n_cfg * T * table slices) is WICK_ETOOBIG. Every
 * call on one GPU uses that GPU's single array: calls that overlap on one
 * GPU (several streams or threads) race and give wrong C; serialise them.
 * Each call writes every partial sum it reads, so nothing needs clearing.
 * Asynchronous on stream; the caller owns B and C. */
wick_status wick_contract_noalloc(wick_plan_t plan, const double *B, int32_t n_cfg, int32_t T,
                                  wick_stream_t stream, double *C);

/* Both steps for a batch of (plan, configuration) items, which may mix
 * nuclei: C is device double [n_items][T][2]. use_graph = 1 captures the
 * launches in a hipGraph on first use of this (plans, items, dims, prec)
 * and replays it afterwards. */
typedef struct { int32_t plan, cfg; } wick_item;
wick_status wick_correlator(const wick_plan_t *plans, int32_t n_plans, const wick_item *items,
                            int32_t n_items, const void *S_u, const void *S_d, wick_dtype dtype,
                            const int32_t dims[4], int32_t n_cfg, wick_precision prec,
                            int32_t use_graph, wick_stream_t stream, double *C);

/* Pick the block kernel's sites per workgroup (single and batched launches)
 * and the term sum's terms per workgroup for a plan and lattice by timing
 * candidates on the current device, on scratch propagators of one
 * configuration that the call allocates and frees (blocking; it uses a
 * stream of its own). Later wick_blocks / wick_contract / wick_correlator
 * calls with the same (dims, dtype, precision, plan sizes) use the choice.
 * The choice is kept in memory and, if cache_path is not NULL, merged into
 * that text file (created if missing); a cache that already holds the shape
 * is used without timing. Errors: WICK_EINVAL (bad arguments),
 * WICK_ECORRUPT (unreadable cache file), WICK_ENOMEM, WICK_EHIP. */
wick_status wick_autotune(wick_plan_t plan, const int32_t dims[4], wick_dtype dtype,
                          wick_precision prec, const char *cache_path);

/* Tune a batched launch as a whole (wick_correlator with these plans, item
 * tables, dims, dtype and precision): the block kernel's sites per
 * workgroup and the term sum's terms per workgroup, each picked by timing
 * eager launches of the whole batch on the caller's propagators S_u, S_d
 * (device, as for wick_correlator; read only). Blocking; it uses a stream of
 * its own and a C buffer it allocates and frees. The choice is kept under a
 * key of (dims, dtype, prec, multiset of the items' tables) and used by every
 * later wick_correlator call with that key (a batch already cached by
 * wick_correlator keeps its shape); with a cache_path it is merged into that
 * text file as for wick_autotune. Errors as for wick_correlator and
 * wick_autotune. */
wick_status wick_autotune_batch(const wick_plan_t *plans, int32_t n_plans, const wick_item *items,
                                int32_t n_items, const void *S_u, const void *S_d, wick_dtype dtype,
                                const int32_t dims[4], int32_t n_cfg, wick_precision prec,
                                const char *cache_path);

/* ------------------------------------------------- correlation matrices */

/* Correlation matrix for the generalized eigenvalue problem (Eqs. E1-E3):
 * C_ij(t) with operator i at the sink and operator j at the source, for
 * n_ops <= 4 operators that share A and flavor content (each desc as for
 * wick_plan; element (i, j) is normalised by sqrt(scale_i * scale_j), scales
 * must be positive). Every element is planned like wick_plan; the element
 * tables are united into one table whose terms are distinct block-entry
 * monomials with one coefficient per element, so a monomial shared by
 * several elements is evaluated once (the cross-element common
 * sub-expressions of Sec. E). Host only; errors as wick_plan. */
typedef struct wick_gevp_s *wick_gevp_t;
wick_status wick_gevp_plan(const wick_nucleus_desc *ops, int32_t n_ops, wick_gevp_t *out);

/* The same for built-in operators (names as for wick_plan_std, spins J[i]
 * or all 0 if J is NULL); "2H-" and "2H0" are the deuteron operator with P_-
 * and with no projector, a basis with "2H". */
wick_status wick_gevp_plan_std(const char *const *names, const int32_t *J, int32_t n_ops, wick_gevp_t *out);

/* Sizes: operators, A, block kinds, terms of the union table, and the sum of
 * the element tables' sizes. */
wick_status wick_gevp_info(wick_gevp_t plan, int32_t *n_ops, int32_t *A, int32_t *n_kinds, int64_t *n_terms,
                           int64_t *n_element_terms);

/* Copy the union table out: kidx[A][n_terms] as for wick_plan_table (each
 * term's indices ascending), coef[n_terms][n_ops * n_ops][2] (element
 * e = i * n_ops + j; zero where the term does not occur). */
wick_status wick_gevp_table(wick_gevp_t plan, uint16_t *kidx, double *coef);

/* A borrowed plan handle with the matrix's block kinds and no terms, valid
 * while the GEVP plan lives (do not destroy it): use it with wick_blocks
 * (the blocks of every element at once), wick_plan_kind and wick_autotune. */
wick_status wick_gevp_kinds(wick_gevp_t plan, wick_plan_t *blocks_plan);

/* C[cfg][t][i][j][2] (device double) = sum over union terms of
 * coef[n][i * n_ops + j] * prod_a B[cfg][t][kidx_{a,n}], FP64, deterministic;
 * B as written by wick_blocks for the wick_gevp_kinds plan. Errors:
 * WICK_EINVAL (null or misaligned pointers, bad sizes), WICK_ENOMEM,
 * WICK_EHIP. Asynchronous on stream. */
wick_status wick_gevp_contract(wick_gevp_t plan, const double *B, int32_t n_cfg, int32_t T,
                               wick_stream_t stream, double *C);
void wick_gevp_destroy(wick_gevp_t plan);

/* ------------------------------------------------------- point sinks */

/* Point-sink correlators by the determinant method (Sec. 3.1 Eq. 2.9,
 * improved method B of Sec. 3.3, the form of App. A Eq. A1): all quarks of
 * the sink operator sit at one site x, summed over x,
 *   C(t) = scale * sum_x sum_{g, h} W_g W'_h det S_u(x,t)[U_g; U'_h] det S_d(x,t)[D_g; D'_h]
 * where (U_g, D_g) runs over the sink operator's coefficient tensor
 * antisymmetrised per flavor (sorted sink index lists with the sign of the
 * sorting, including the flavor-grouping sign) and (U'_h, D'_h) over the
 * source's, and det S[R; K] is the determinant of the rows R (sink indices)
 * and columns K (source indices) of the 12x12 propagator at (x, t). The
 * minimal set of determinants is the set of distinct (row set, column set)
 * pairs per flavor. Uses the same wick_nucleus_desc as wick_plan (the sink
 * patterns are read at one point; kinds need not be nucleon-like). Up to 6
 * quarks of each flavor (WICK_EUNSUPPORTED beyond). */
typedef struct wick_point_s *wick_point_t;
wick_status wick_point_plan(const wick_nucleus_desc *desc, wick_point_t *out);
wick_status wick_point_plan_std(const char *nucleus, int32_t J, wick_point_t *out);

/* Sizes: quarks per flavor, sink and source groups, distinct sink row sets
 * and source column sets per flavor (the minimal set has n_rows_u * n_cols_u
 * u determinants and n_rows_d * n_cols_d d determinants per site). */
wick_status wick_point_info(wick_point_t plan, int32_t *n_u, int32_t *n_d, int64_t *n_sink_groups,
                            int64_t *n_src_groups, int64_t *n_rows_u, int64_t *n_cols_u,
                            int64_t *n_rows_d, int64_t *n_cols_d);

/* C[cfg][t] (device double [n_cfg][T][2]) from propagators laid out as for
 * wick_blocks (device, 16-byte aligned, complex128 or complex64), FP64
 * arithmetic throughout, deterministic. Errors: WICK_EINVAL (null or
 * misaligned pointers, bad sizes), WICK_ENOMEM, WICK_EHIP. Asynchronous on
 * stream; the caller keeps S_u, S_d and C alive until it completes. */
wick_status wick_point_correlator(wick_point_t plan, const void *S_u, const void *S_d, wick_dtype dtype,
                                  const int32_t dims[4], int32_t n_cfg, wick_stream_t stream, double *C);
void wick_point_destroy(wick_point_t plan);

/* The same point-sink correlator in the block form (Eq. 3.1): at every site
 * the blocks of that site alone and the plane-wave plan's signed term table
 * on them, summed over sites (C[cfg][t] = sum_x sum_n coef_n prod_a
 * B_x[kidx_{a,n}], scale included). The per-site blocks are built in chunks
 * of site-slices and summed with the wick_contract kernels (the site-slices
 * take the place of time slices). On the 24^3 lattice it is the faster route
 * for deuteron, helium-3 and helium-4 (whose table takes the factored form
 * there as everywhere). Same
 * arguments and errors as wick_point_correlator, with a plan from wick_plan /
 * wick_plan_std; it allocates a second per-stream workspace for the site
 * blocks (at most 512 MB) and the per-site sums. */
wick_status wick_point_blocks_correlator(wick_plan_t plan, const void *S_u, const void *S_d, wick_dtype dtype,
                                         const int32_t dims[4], int32_t n_cfg, wick_stream_t stream, double *C);

/* Release the device workspace (blocking). */
wick_status wick_shutdown(void);

/* Kernel timing with HIP events, recorded on the stream each kernel runs on.
 * enable = 1 starts recording (and clears earlier records), 0 stops.
 * wick_profile_read waits for the recorded events and returns, for the
 * kernel named `kernel` ("blocks", "blocks_reduce", "contract",
 * "contract_finalize"), the number of launches and their total time. */
wick_status wick_profile(int32_t enable);
wick_status wick_profile_read(const char *kernel, int64_t *launches, double *total_ms);

/* Message of the last failing call on this thread ("" if none). */
const char *wick_last_error(void);

/* Library version string. */
const char *wick_version(void);

#ifdef __cplusplus
}
#endif
#endif /* WICK_H */
