/*
 * spamm.h -- C ABI of the MI355X (gfx950) Sparse Approximate Matrix Multiply.
 *
 * Method: Challacombe & Bock, "Fast Multiplication of Matrices with Decay"
 * (arXiv:1011.3534).  A matrix is held as a quadtree (section 2, Eq. 1):
 * 2x2 recursive blocking down to dense b x b leaves, with the Frobenius norm
 * (section 3) carried at every node.  The product C = A B is formed by the
 * SpAMM recursion of Eq. (4): a block product is dropped when
 * ||A^k|| ||B^k|| < tau, taken densely at the leaves, and otherwise assembled
 * from its 8 sub-products.
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 *  - All functions return spamm_status; SPAMM_OK (0) on success.  Nothing is
 *    thrown or aborted across the ABI.  On a non-OK status
 *    spamm_last_error() returns a thread-local message.
 *  - Arguments are validated on the host before anything is enqueued; a
 *    SPAMM_EINVAL return leaves every output untouched.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it in order; calls do not synchronise the device
 *    except where stated (non-NULL stats/log pointers, the host read-back
 *    helpers).
 *  - Device pointers are caller-owned, are read in stream order and may be
 *    released once the stream has passed the call.  spamm_matrix handles are
 *    library-owned and released with spamm_free().
 *  - Norms are FP64 squared Frobenius norms S; the cull test is
 *    fl(S_A * S_B) < fl(tau * tau) (ties kept), so no square root decides a
 *    product.  A leaf's S is summed in a fixed order: per column, over rows
 *    in ascending order with fused multiply-add; then over columns by the
 *    pairwise tree s_c += s_{c+h}, h = b/2 .. 1.  A parent's S is
 *    (S_00 + S_01) + (S_10 + S_11), absent children counting +0.
 *  - The kept leaf triples (I, J, K) are therefore fixed by the stored input
 *    values, the leaf size and tau alone -- not by leaf precision, schedule or
 *    padding -- and equal the flat rule keep <=> !(S_A[I,K] S_B[K,J] < tau^2)
 *    (the tier tests are monotone because parent norms dominate children).
 */
#ifndef SPAMM_H
#define SPAMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spamm_matrix spamm_matrix;

typedef enum {
    SPAMM_OK = 0,
    SPAMM_EINVAL = 1,       /* invalid argument (nothing enqueued)                  */
    SPAMM_ENOMEM = 2,       /* device allocation failed                             */
    SPAMM_EHIP = 3,         /* a HIP runtime call failed (message names it)         */
    SPAMM_ECAPACITY = 4,    /* a device-side buffer would overflow                  */
    SPAMM_ENONFINITE = 5,   /* an operand holds an inf or NaN (its root norm is     *
                             * not finite), reported by the syncing calls         */
    SPAMM_ENOCONV = 6,      /* SP2 did not meet its stopping rule within max_iter   */
    SPAMM_EUNSUPPORTED = 7  /* valid request the library does not implement         */
} spamm_status;

/* Element type of the caller's dense matrix and of the stored tiles. */
typedef enum { SPAMM_F64 = 0, SPAMM_F32 = 1 } spamm_dtype;

/* Arithmetic of the dense leaf products (section 3 uses single precision
 * 4x4 products; the MFMA variants here accumulate in FP32, FP64 in FP64).
 *   F64    : FP64 inputs, FP64 MFMA, FP64 result (also the exact reference)
 *   F32    : FP32 MFMA, FP32 result
 *   BF16   : operands rounded to bfloat16 (RNE), FP32 accumulation
 *   BF16X3 : x = hi + lo with hi = bf16(x), lo = bf16(x - hi); the product
 *            hi*hi + hi*lo + lo*hi on bf16 MFMA (lo*lo dropped)
 *   F16    : operands scaled per tile by a power of two, rounded to fp16
 *   F16X3  : as BF16X3 with fp16 halves of the per-tile power-of-two scaled
 *            operand; the scale is undone exactly after each leaf product.
 * The result of every precision other than F64 is stored as FP32. */
typedef enum {
    SPAMM_LEAF_F64 = 0,
    SPAMM_LEAF_F32 = 1,
    SPAMM_LEAF_BF16 = 2,
    SPAMM_LEAF_BF16X3 = 3,
    SPAMM_LEAF_F16 = 4,
    SPAMM_LEAF_F16X3 = 5
} spamm_leaf_prec;

#define SPAMM_MAX_LEVELS 24

/* Statistics of one product (filled by a syncing call). */
typedef struct {
    int64_t n;                                /* matrix dimension                              */
    int32_t leaf;                             /* leaf size b                                   */
    int32_t levels;                           /* tiers above the leaves, L = ceil(log2 nb)     */
    int64_t nb;                               /* leaves per dimension, ceil(n / b)             */
    int64_t survivors[SPAMM_MAX_LEVELS];      /* kept octree nodes per tier (0 = leaf triples) */
    int64_t tasks;                            /* leaf products T (= survivors[0])              */
    int64_t nonempty_tiles;                   /* C tiles with at least one kept product        */
    double flops;                             /* algorithmic leaf flops 2 b^3 T                */
    double culled_bound;                      /* sum over culled octree nodes of
                                                 ||A^k||_F ||B^k||_F (Eq. 3 bound on ||dC||_F) */
} spamm_stats;

/* Per-iteration record of spamm_sp2. */
#define SPAMM_SP2_MAX_ITER 256
typedef struct {
    int32_t iterations;                       /* steps executed                                */
    int32_t converged;                        /* 1: ||X^2-X||_F <= idem_tol was met            */
    int32_t stagnated;                        /* 1: stopped by the stagnation rule             */
    int32_t result_step;                      /* P = X_{result_step}                           */
    double trace[SPAMM_SP2_MAX_ITER];         /* tr(X_m), FP64                                 */
    double idem[SPAMM_SP2_MAX_ITER];          /* ||X_m^2 - X_m||_F, FP64                       */
    int32_t branch[SPAMM_SP2_MAX_ITER];       /* 0: X <- X^2, 1: X <- 2X - X^2                 */
    int64_t tasks[SPAMM_SP2_MAX_ITER];        /* leaf products of step m                       */
    double final_trace;                       /* tr(P)                                         */
    double energy;                            /* tr(P H), FP64                                 */
    double eps_min, eps_max;                  /* Gershgorin bounds of H                        */
} spamm_sp2_log;

/* ------------------------------------------------------------------ build */

/* Quadtree representation of a dense matrix (section 2, Eq. 1).
 *   dev_a : device pointer, n x n row-major, leading dimension lda (elements)
 *   dt    : element type of dev_a; the tiles are stored in the same type
 *   leaf  : b in {32, 64, 128}
 *   out   : in/out.  If *out is NULL it receives a new handle: zero-padded
 *           tile-major storage (b x b tiles, row-major inside, tiles in
 *           (I, K) row-major order) and the FP64 squared-norm pyramid of all
 *           tiers.  If *out is a handle of the same n, leaf and dtype it is
 *           rebuilt in place (no allocation).
 * One pass over dev_a computes the packed tiles and the leaf norms.  The
 * tiers above the leaves are formed when a call first reads them (a product
 * that descends the tiers, spamm_norms, the tau calls), on that call's
 * stream; calls on one handle must be ordered (one stream, or events), as
 * for every other use of it.  Errors: EINVAL (n < 1, lda < n, bad
 * leaf/dtype, null pointers), ENOMEM, EHIP. */
spamm_status spamm_build(const void* dev_a, int64_t n, int64_t lda, spamm_dtype dt, int32_t leaf,
                         void* stream, spamm_matrix** out);

/* spamm_build of count matrices in one pass (the concatenated tile pools of
 * a batch): one launch packs every matrix's tiles and leaf norms, and each
 * upper tier is formed for all matrices by one launch, so a batch of small
 * matrices costs a few launches instead of a few per matrix.  Results are
 * the same bits as count calls of spamm_build.
 *   dev_a[m], n[m], lda[m] : as spamm_build, per matrix (host arrays)
 *   dt, leaf               : shared by the batch
 *   out[m]                 : in/out as for spamm_build (NULL entries are
 *                            allocated; existing handles must match n[m],
 *                            leaf and dt, and be distinct)
 * Errors: EINVAL (count outside [1, 128], null pointers, bad n/lda/leaf,
 * mismatched or repeated handles), ENOMEM, EHIP.  On error no handle of
 * out[] is changed. */
spamm_status spamm_build_batched(int32_t count, const void* const* dev_a, const int64_t* n,
                                 const int64_t* lda, spamm_dtype dt, int32_t leaf, void* stream,
                                 spamm_matrix** out);

/* spamm_build for operands of products with leaf precision `prec`.  For the
 * 16-bit precisions (FP32 input only) the same pass also writes the handle's
 * split tiles: x = hi + lo per element in FP16 (tile scaled by a power of two
 * that puts its largest |x| in [2^14, 2^15)) or BF16, rounded to nearest,
 * which the 16-bit leaf products read (4 more bytes of device memory per tile
 * element, owned by the handle) instead of splitting each operand tile again
 * for every product that reads it; worth it when an operand feeds several
 * products.  Products of operands without current split tiles (built by
 * spamm_build, rebuilt since, or products of other calls) split on the fly;
 * the results are the same bits either way.  For the FP32 and FP64
 * precisions it is spamm_build.  Errors: as spamm_build;
 * EINVAL for an unknown prec; EUNSUPPORTED for a 16-bit prec with FP64 input. */
spamm_status spamm_build_ex(const void* dev_a, int64_t n, int64_t lda, spamm_dtype dt, int32_t leaf,
                            spamm_leaf_prec prec, void* stream, spamm_matrix** out);

/* spamm_build without the copy (section 2, Eq. 1: the tree's leaves are the
 * b x b blocks of the matrix, wherever they are stored).  The handle keeps
 * dev_a itself as its tile storage (tile (I, K) is rows I*b.. and columns
 * K*b.. of dev_a) and owns only the norm pyramid, so the build reads dev_a
 * once and writes no tiles.  dev_a must outlive the handle and must not be
 * written while the handle is in use (rebuild after every change).
 * A view is an operand of spamm_multiply*, spamm_tau_*, spamm_to_dense,
 * spamm_diff_norms and spamm_norms; it cannot receive a product (EINVAL) and
 * is not an SP2 Hamiltonian (EUNSUPPORTED).  Norms and products of a view are
 * the same bits as those of a spamm_build handle of the same array.
 *   out : in/out as for spamm_build; an existing handle must be a view of
 *         the same n, leaf and dtype, and is re-pointed at dev_a.
 * Errors: as spamm_build; EINVAL also for n not a multiple of leaf, dev_a or
 * lda * element size not a multiple of 16 bytes, leaf * lda * element size
 * >= 2^31 bytes, or an existing handle that is not a view (and spamm_build
 * on an existing view). */
spamm_status spamm_build_view(const void* dev_a, int64_t n, int64_t lda, spamm_dtype dt, int32_t leaf,
                              void* stream, spamm_matrix** out);

/* spamm_build_view for operands of products with leaf precision `prec`: no
 * copy of the FP32 tiles, but for the 16-bit precisions the handle owns
 * split hi/lo tiles of the array, written as in spamm_build_ex (4 bytes per
 * element, tile-major).  The leaf products read the split tiles instead of
 * the array, so the build costs one pass that reads the array and writes the
 * split tiles, and every product of the handle skips the split.  Products
 * are the same bits as those of spamm_build_view operands.  For the FP32 and
 * FP64 precisions it is spamm_build_view.
 *   out  : in/out as for spamm_build_view (a rebuild refreshes the split)
 * Errors: as spamm_build_view; EINVAL for an unknown prec; EUNSUPPORTED for
 * a 16-bit prec with FP64 input. */
spamm_status spamm_build_view_ex(const void* dev_a, int64_t n, int64_t lda, spamm_dtype dt, int32_t leaf,
                                 spamm_leaf_prec prec, void* stream, spamm_matrix** out);

/* spamm_build_view of count matrices, one launch for all leaf norms and one
 * per upper tier, as spamm_build_batched.  Arguments, errors and the
 * no-change-on-error rule as spamm_build_batched, with the view conditions
 * of spamm_build_view applying to every matrix. */
spamm_status spamm_build_view_batched(int32_t count, const void* const* dev_a, const int64_t* n,
                                      const int64_t* lda, spamm_dtype dt, int32_t leaf, void* stream,
                                      spamm_matrix** out);

/* ------------------------------------------------------------------ multiply */

/* C ~= A B by Eq. (4) with absolute threshold tau.
 *   A, B  : handles with equal n and leaf (dtypes may differ; F64 leaves
 *           promote FP32 tiles exactly)
 *   tau   : finite, tau == 0 (dense product) or tau >= 1e-150
 *   prec  : leaf arithmetic (spamm_leaf_prec)
 *   C     : in/out.  If *C is NULL a new handle is allocated.  If *C is a
 *           handle of the same n, leaf and result type it is overwritten in
 *           place, reusing its product scratch (no allocation).  C may not
 *           alias A or B.
 *   st    : optional; when non-NULL the call synchronises the stream and
 *           fills the statistics.
 * The result carries its own norm pyramid (leaf norms from the product,
 * the tiers above formed when first read), so it can be an operand of the
 * next product.  Every C tile with no kept product is exactly zero.
 * Errors: EINVAL, ENOMEM, EHIP; with st, ENONFINITE when A or B holds an
 * inf or NaN (the product is still written) and ECAPACITY. */
spamm_status spamm_multiply(const spamm_matrix* A, const spamm_matrix* B, double tau,
                            spamm_leaf_prec prec, void* stream, spamm_matrix** C,
                            spamm_stats* st);

/* Threshold schedules of spamm_multiply_ex. */
#define SPAMM_TAU_FLAT 0          /* tau at every tier: Eq. (4) (spamm_multiply)  */
#define SPAMM_TAU_DEPTH_SCALED 1  /* tau / 8^k at depth k below the root          */

/* spamm_multiply with a threshold schedule.  SPAMM_TAU_DEPTH_SCALED is the
 * rigorous variant section 2 mentions beside its round-off comparison: the
 * threshold is divided by 8 at every level of the recursion, so a node of
 * the product octree at depth k (the root is depth 0, the leaf triples
 * depth L) is kept iff !(S_A * S_B < fl(tau_k * tau_k)) with tau_k =
 * tau / 8^k, and every ancestor was kept.  (S are the FP64 squared norms of
 * the node's blocks; fl(tau_k * tau_k) = fl(tau * tau) 2^-6k exactly.)  The
 * kept leaf triples then contain those of the flat rule at tau and lie within
 * those of the flat rule at tau / 8^L, and the omitted part of the product is
 * below (L + 1) tau in Frobenius norm.  The flat rule at tau equals its own
 * leaf-level test; the depth-scaled one does not, so its cull is truly
 * tier-by-tier.
 *   tau_schedule : SPAMM_TAU_FLAT or SPAMM_TAU_DEPTH_SCALED
 *   tau          : as spamm_multiply; for the depth-scaled schedule also
 *                  tau == 0 or tau / 8^L >= 1e-150, so that every tier's tau^2
 *                  is a normal FP64 number
 * Other arguments, ownership and results as spamm_multiply.
 * Errors: as spamm_multiply; EINVAL for an unknown schedule or a tau below
 * the depth-scaled limit. */
spamm_status spamm_multiply_ex(const spamm_matrix* A, const spamm_matrix* B, double tau,
                               spamm_leaf_prec prec, int32_t tau_schedule, void* stream,
                               spamm_matrix** C, spamm_stats* st);

/* Phase durations of one product, from HIP events on the caller's stream. */
typedef struct {
    double ms_cull;    /* counter reset, mask clear and every cull tier      */
    double ms_leaf;    /* the leaf-product launch (incl. its epilogue)       */
    double ms_norms;   /* upper tiers of the result's norm pyramid           */
    double ms_total;   /* first to last event                                */
} spamm_timing;

/* spamm_multiply with phase timing: same arguments and result; records HIP
 * events between the phases on `stream`, synchronises, and fills *t.
 * Errors: as spamm_multiply; EINVAL if t is NULL. */
spamm_status spamm_multiply_timed(const spamm_matrix* A, const spamm_matrix* B, double tau,
                                  spamm_leaf_prec prec, void* stream, spamm_matrix** C,
                                  spamm_timing* t);

/* spamm_multiply_timed with options.  SPAMM_TIMED_DESCENT: the cull
 * descends level-synchronously from the root, tier by tier (each tier's
 * survivors compacted by prefix scans), as a product with statistics does,
 * instead of testing every leaf triple in one pass -- the same kept triples
 * and the same result bits, for timing the descent itself.  flags = 0 is
 * spamm_multiply_timed.  Errors: as spamm_multiply_timed; EINVAL for unknown
 * flags. */
#define SPAMM_TIMED_DESCENT 1
spamm_status spamm_multiply_timed_ex(const spamm_matrix* A, const spamm_matrix* B, double tau,
                                     spamm_leaf_prec prec, int32_t flags, void* stream, spamm_matrix** C,
                                     spamm_timing* t);

/* Leaf-product schedule. */
typedef enum {
    SPAMM_SCHED_STATIC = 0,  /* one block per C tile, tiles split into 8 contiguous
                                ranges, one per XCD (the default of spamm_multiply) */
    SPAMM_SCHED_LPT = 1,     /* persistent blocks pull tiles from a device queue in
                                order of decreasing kept-K count (largest first)     */
    SPAMM_SCHED_LIST = 2     /* one pass lists the C tiles that need a write (a kept
                                product, or stored values not known to be zero);
                                persistent blocks take the list in a static stride,
                                so the many empty tiles of banded products cost no
                                block at all                                         */
} spamm_schedule;

typedef struct {
    int32_t leaf;            /* leaf size the operands were built with (autotuner output) */
    int32_t schedule;        /* spamm_schedule                                           */
    int32_t split;           /* autotuner output: 1 = build the operands with split
                                16-bit tiles (spamm_build_ex with the leaf precision),
                                0 = plain builds (split while staging); ignored by
                                spamm_multiply_batched, whose operands decide        */
    int32_t reserved[5];
} spamm_tune;

/* count independent products C_m ~= A_m B_m in one pass: one cull over every
 * root (products enter at their own root tier) and ONE leaf-product launch
 * over the union of all C tiles.  All operands share the leaf size and leaf
 * precision; n may differ between products.
 *   tau[m]       : per-product threshold (host array of count doubles)
 *   tune         : schedule; NULL = SPAMM_SCHED_LPT (tune->leaf is ignored
 *                  here: it must equal the operands' leaf if set)
 *   C[m]         : in/out as for spamm_multiply
 *   st           : optional host array of count spamm_stats (syncs)
 * Batch scratch (frontiers, counters, schedule) is allocated for the call and
 * released at its end.
 * Errors: EINVAL (count < 1 or > 128, mismatched pairs, mixed leaf sizes),
 * ENOMEM, EHIP; with st, ECAPACITY and ENONFINITE as spamm_multiply. */
spamm_status spamm_multiply_batched(int32_t count, const spamm_matrix* const* A,
                                    const spamm_matrix* const* B, const double* tau,
                                    spamm_leaf_prec prec, const spamm_tune* tune, void* stream,
                                    spamm_matrix** C, spamm_stats* st);

/* spamm_multiply_batched for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same cull, schedule and leaf kernels, with the batch
 * scratch (descriptors, counters, schedule arrays) in a static 16 MiB
 * device array of the library -- one per device, kept until the process
 * ends.  It calls no allocator: no hipMalloc, hipFree or allocator hook.
 *   C[m]   : existing result handles (same n, leaf and result type as for
 *            spamm_multiply_batched), each of which has already received a
 *            product, so that its own product scratch is in place; the
 *            handles are overwritten, the array itself is not written
 *   other arguments as spamm_multiply_batched; no statistics.
 * Limits: at most 2^27 leaf triples over the batch (sum of nb^3: the direct
 * leaf pass, no frontier) and a batch plan within 16 MiB.
 * Every call on a device shares that device's array and leaves its contents
 * behind; calls that overlap on one device (different streams or host
 * threads with no ordering between them) race.  Calls on one stream are
 * ordered and safe.
 * Errors: EINVAL as spamm_multiply_batched, also for a NULL C[m], a handle
 * with no product scratch or on another device than the current one;
 * ECAPACITY beyond the limits (nothing enqueued); EHIP. */
spamm_status spamm_multiply_batched_noalloc(int32_t count, const spamm_matrix* const* A,
                                            const spamm_matrix* const* B, const double* tau,
                                            spamm_leaf_prec prec, const spamm_tune* tune, void* stream,
                                            spamm_matrix* const* C);

/* ------------------------------------------------------------------ autotuner */

#define SPAMM_TUNE_MAX_LEAVES 3
#define SPAMM_TUNE_MAX_TRIALS 18
typedef struct {
    int32_t trials;                              /* candidates timed (0 if from cache)     */
    int32_t from_cache;                          /* 1: answer read from the cache file     */
    int32_t leaf[SPAMM_TUNE_MAX_TRIALS];
    int32_t schedule[SPAMM_TUNE_MAX_TRIALS];
    int32_t split[SPAMM_TUNE_MAX_TRIALS];        /* operands built with split tiles        */
    int32_t qualified[SPAMM_TUNE_MAX_TRIALS];    /* met max_rel_err                        */
    double ms[SPAMM_TUNE_MAX_TRIALS];            /* median of reps batched products        */
    double max_rel_err[SPAMM_TUNE_MAX_TRIALS];   /* worst product of the batch             */
    double best_ms;
} spamm_tune_report;

/* Autotuner of spamm_multiply_batched for the products C_m = A_m A_m of the
 * caller's dense operands (dev_a[m]: n[m] x n[m] row-major, leading
 * dimension n[m], element type dt).  For every leaf size in leaves[] (each
 * 32, 64 or 128; at most 3) the operands are built and the three schedules
 * are timed (median of reps products, HIP events on `stream`); with a 16-bit
 * leaf precision and FP32 operands every leaf size is tried twice, with plain
 * builds and with split tiles (spamm_build_ex), so up to 18 candidates.
 * Because the leaf size changes which block products are kept, a candidate
 * qualifies only if every product stays within max_rel_err (relative
 * Frobenius error) of the exact product, formed once with FP64 leaves at
 * tau = 0.  The fastest qualifying candidate is returned in *best and, if
 * cache_path is non-NULL, appended to that text file, one line per key.  The
 * key describes the batch by buckets: the count in octaves, the mean n in
 * half-octaves and the kept fraction of the leaf triples at leaves[0] (one
 * product with statistics, in octaves), with dt, prec, max_rel_err and the
 * candidate leaves; a later call whose batch falls in the same buckets
 * returns the cached answer after that one product, without trials.
 * report (optional) lists every trial.  Synchronises.  Errors: EINVAL (bad
 * arguments, no candidate qualifies), ENOMEM, EHIP. */
spamm_status spamm_autotune_batched(int32_t count, const void* const* dev_a, const int64_t* n,
                                    spamm_dtype dt, const double* tau, spamm_leaf_prec prec,
                                    const int32_t* leaves, int32_t n_leaves, double max_rel_err,
                                    int32_t reps, const char* cache_path, void* stream,
                                    spamm_tune* best, spamm_tune_report* report);

/* ------------------------------------------------------------------ SP2 / TC2 */

/* Density matrix P = theta[mu I - H] with n_occ occupied states by TC2
 * purification (section 3; Niklasson 2002), every squaring a SpAMM at tau:
 *   X_0 = (eps_max I - H)/(eps_max - eps_min) from Gershgorin bounds (FP64);
 *   step m: Y = SpAMM(X_m, X_m); X_{m+1} = Y if tr(X_m) > n_occ else 2X_m - Y;
 *           e_m = ||Y - X_m||_F; traces and e_m in FP64 on the device;
 *   stop after the step with e_m <= idem_tol (P = X_{m+1}), or when
 *   e_m >= e_{m-2} while e_{m-2} < 0.1 (stagnation; P = X_m), or after
 *   max_iter steps.
 * All max_iter steps are captured in one hipGraph; steps after the stop are
 * no-ops decided on the device, so the host synchronises once.
 *   H       : symmetric operand (FP32 or FP64 tiles)
 *   prec    : leaf arithmetic of the squarings (not F64 unless H is FP64)
 *   P       : receives a new handle
 *   log     : optional per-step record
 * Errors: EINVAL (n_occ outside [0, n], max_iter outside [1, 256]), ENOMEM,
 * EHIP, ENOCONV (no stop rule met; P then holds X_max_iter). */
spamm_status spamm_sp2(const spamm_matrix* H, int64_t n_occ, double tau, int32_t max_iter,
                       double idem_tol, spamm_leaf_prec prec, void* stream, spamm_matrix** P,
                       spamm_sp2_log* log);

/* spamm_sp2 with options.  SPAMM_SP2_SYMMETRIC: every squaring is a
 * symmetric squaring, the TC2 iteration's X being symmetric: only the C
 * tiles with I <= J are formed by Eq. (4) (kept K of tile (I, J) by the flat
 * rule), and tile (J, I) is written as the transpose of tile (I, J), with the
 * norm of the stored values in the canonical order; X stays exactly
 * symmetric off the diagonal tiles and the leaf work about halves.  H must be
 * exactly symmetric (checked: EINVAL otherwise).  Other arguments, results
 * and errors as spamm_sp2; the per-step task counts are those formed. */
#define SPAMM_SP2_SYMMETRIC 1
/* SPAMM_SP2_DROPPING: the block-dropping scheme that section 3 compares
 * SpAMM with.  tau is then the drop threshold: every squaring is exact over
 * the tiles present (a tile is absent once dropped, so it takes part in no
 * product; the per-step task counts are the pairs of present tiles), and
 * after each step every tile of the new iterate with squared norm
 * S < fl(tau * tau) is dropped (set to zero, norm 0), so the trace that
 * decides the next branch is that of the filtered iterate.  X_0 is not
 * filtered.  Presence is the cull test at threshold 1e-150: a non-zero FP32
 * tile has S >= 2^-298, so two present tiles always pass it.  Not combined
 * with SPAMM_SP2_SYMMETRIC (EUNSUPPORTED): the two mirrored tiles' norms are
 * summed in different orders and could be filtered differently. */
#define SPAMM_SP2_DROPPING 2
spamm_status spamm_sp2_ex(const spamm_matrix* H, int64_t n_occ, double tau, int32_t max_iter,
                          double idem_tol, spamm_leaf_prec prec, int32_t flags, void* stream,
                          spamm_matrix** P, spamm_sp2_log* log);

/* ------------------------------------------------------------------ learned tau */

/* The paper sets tau by hand to match energy errors (section 3).  The
 * selector maps the norm structure of A and B and a target relative error
 * ||C~ - C||_F / ||C||_F to a threshold with a small network trained on
 * (matrix, tau, error) samples that SpAMM itself produces.
 *
 * Features (SPAMM_TAU_NFEAT floats): for operand X in (A, B) and tier
 * l = 0..7 counted from the leaves (tiers above the root are all zero), the
 * fraction of the tier's nodes in bin k = #{j in 1..31 : S < S_root * 1e-j}
 * (32 bins; 1e-j the correctly rounded decimal constants); then
 * log10(target), log2(nb) / 10, log2(b) / 7.
 * Network: 515 -> 128 -> 128 -> 128 -> 1, ReLU on hidden layers, FP32;
 * parameters flat as W1 (in x out, row-major), b1, W2, b2, W3, b3, W4, b4.
 * Output y = log10(tau / (||A||_F ||B||_F)).  Training minimises the mean
 * squared error of y with Adam (beta 0.9 / 0.999, eps 1e-8) over fixed-order
 * minibatches. */
#define SPAMM_TAU_NFEAT 515
#define SPAMM_TAU_HIDDEN 128
#define SPAMM_TAU_NPARAM (515 * 128 + 128 + 2 * (128 * 128 + 128) + 128 + 1)

typedef struct spamm_tau_model spamm_tau_model;  /* device weights + Adam moments */

typedef struct {
    double tau_pred;      /* the network's threshold                         */
    double err_pred;      /* relative error of the product at tau_pred       */
    double tau;           /* returned threshold (tau_pred unless fallback)   */
    double rel_err;       /* relative error at tau                           */
    int64_t tasks;        /* leaf products at tau                            */
    int32_t evaluations;  /* SpAMM + error evaluations performed             */
    int32_t fallback;     /* 1: tau_pred missed the target, bisection ran    */
} spamm_tau_info;

/* Model from SPAMM_TAU_NPARAM host floats (initial or trained weights). */
spamm_status spamm_tau_model_create(const float* host_params, spamm_tau_model** out);
/* Copy the current weights to host_params (SPAMM_TAU_NPARAM floats); syncs. */
spamm_status spamm_tau_model_params(const spamm_tau_model* m, float* host_params);
void spamm_tau_model_free(spamm_tau_model* m);

/* Features of (A, B, target) into dev_out (SPAMM_TAU_NFEAT device floats). */
spamm_status spamm_tau_features(const spamm_matrix* A, const spamm_matrix* B, double target,
                                float* dev_out, void* stream);
/* y for count feature rows dev_x (count x 515, device) into dev_y; syncs. */
spamm_status spamm_tau_forward(const spamm_tau_model* m, const float* dev_x, int64_t count,
                               float* dev_y, void* stream);
/* Gradient of the mean squared error over the count rows (host_grad:
 * SPAMM_TAU_NPARAM floats) and the loss; syncs.  For checking. */
spamm_status spamm_tau_grad(const spamm_tau_model* m, const float* dev_x, const float* dev_y,
                            int64_t count, float* host_grad, float* host_loss, void* stream);
/* epochs passes of Adam over minibatches of `batch` consecutive rows;
 * host_loss (optional, epochs floats) receives each epoch's mean loss. */
spamm_status spamm_tau_train(spamm_tau_model* m, const float* dev_x, const float* dev_y,
                             int64_t count, int32_t epochs, int32_t batch, float lr, void* stream,
                             float* host_loss);
/* tau = 10^y ||A||_F ||B||_F for the target relative error; syncs. */
spamm_status spamm_tau_predict(const spamm_matrix* A, const spamm_matrix* B, double target,
                               const spamm_tau_model* m, void* stream, double* tau_out);
/* Threshold that meets the target, checked against the exact product (FP64
 * leaves at tau = 0): the starting tau -- the network's prediction for half
 * the target (m non-NULL), else 10 target ||A||_F ||B||_F -- is checked; if
 * its error exceeds the target, tau steps down until the target holds (from
 * a prediction by log10(err / target) + 0.1 decades, at least 0.1, since the
 * error grows about in proportion to tau; a decade at a time otherwise) and
 * is then bisected in log10(tau) to resolution_decades between the tau that
 * met the target and the last one that missed.  *C (in/out as for spamm_multiply) holds the product at
 * the returned tau.  Syncs.  Errors: EINVAL, ENOMEM, EHIP, ENOCONV (no tau
 * within 12 decades met the target). */
spamm_status spamm_tau_select(const spamm_matrix* A, const spamm_matrix* B, double target,
                              const spamm_tau_model* m, spamm_leaf_prec prec,
                              double resolution_decades, void* stream, spamm_matrix** C,
                              spamm_tau_info* info);

/* ------------------------------------------------------------------ helpers */

/* Dense row-major copy of M (n x n, leading dimension ldo, M's element type)
 * into caller-owned device memory. */
spamm_status spamm_to_dense(const spamm_matrix* M, void* dev_out, int64_t ldo, void* stream);

/* Shape queries. */
spamm_status spamm_info(const spamm_matrix* M, int64_t* n, int32_t* leaf, spamm_dtype* dt,
                        int32_t* levels);

/* Squared norms of tier `level` (0 = leaves) copied to host_out
 * (m_l x m_l row-major, m_l = ceil(nb / 2^level)); cap in elements.
 * Synchronises the stream.  ENONFINITE (after the copy) when the matrix
 * holds an inf or NaN. */
spamm_status spamm_norms(const spamm_matrix* M, int32_t level, double* host_out, int64_t cap,
                         void* stream);

/* The kept leaf triples of the product that last wrote C, as keys
 * I << 42 | J << 21 | K, sorted ascending, copied to host (up to cap);
 * *count receives T.  Synchronises the stream. */
spamm_status spamm_task_list(const spamm_matrix* C, uint64_t* host_keys, int64_t cap,
                             int64_t* count, void* stream);

/* ||X - Y||_F^2 and ||Y||_F^2 in FP64 over two handles of equal n (any
 * element types and leaf sizes), e.g. X = SpAMM result, Y = exact product.
 * Synchronises. */
spamm_status spamm_diff_norms(const spamm_matrix* X, const spamm_matrix* Y, double* diff2,
                              double* ref2, void* stream);

/* Seeded synthetic decay matrix on the device (input generation only; the
 * multiply never calls it).  a_ij = round(f(|i-j|) * (lo + (hi - lo) u_ij))
 * with u_ij = (h >> 11) 2^-53, h = SplitMix64(SplitMix64(seed) ^ (i << 32 | j))
 * (counter (min(i,j), max(i,j)) when symmetric), f = host_table[0..n) in
 * FP64; host_diag (optional, n entries) overrides the diagonal.  The same
 * definition as the host-side generator, so both draw identical matrices.
 * dev_out: n x n row-major, leading dimension ld, element type dt.
 * Synchronises.  Errors: EINVAL, ENOMEM, EHIP. */
spamm_status spamm_generate_decay(int64_t n, int64_t ld, spamm_dtype dt, const double* host_table,
                                  uint64_t seed, double lo, double hi, int32_t symmetric,
                                  const double* host_diag, void* dev_out, void* stream);

/* Device allocation hook, stream-ordered.
 *   alloc(bytes, stream, ctx)  : device memory for work enqueued on `stream`
 *                                (a hipStream_t as void*, NULL = null stream),
 *                                or NULL on failure (the call then returns
 *                                SPAMM_ENOMEM)
 *   dealloc(ptr, stream, ctx)  : release ptr once the work enqueued on
 *                                `stream` before this call is done with it: the
 *                                block may go to later work on that stream at
 *                                once (stream order), to other streams only
 *                                after this stream passes the call
 * Every device allocation of the library goes through the hook: handle
 * storage and product scratch (allocated on the stream of the call that
 * creates them, released by spamm_free after it synchronises the handle's
 * last stream), per-call workspaces of the batched, SP2, autotune, tau,
 * diff-norm and generator calls (allocated and released on the stream of the
 * call, the release enqueued right after the kernels that read them), and
 * tau models (allocated on the null stream, released by
 * spamm_tau_model_free after a device synchronisation).
 * NULL functions restore hipMalloc / hipFree (hipFree waits for the device).
 * Handles and models keep the pair they were allocated with, so the
 * functions must stay callable until every such object is freed; ctx is
 * passed through unchanged.  Errors: EINVAL if exactly one function is NULL. */
typedef void* (*spamm_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*spamm_dealloc_fn)(void* ptr, void* stream, void* ctx);
spamm_status spamm_set_allocator(spamm_alloc_fn alloc, spamm_dealloc_fn dealloc, void* ctx);

/* Release a handle (NULL is a no-op).  Synchronises the handle's last stream. */
void spamm_free(spamm_matrix* M);

/* Thread-local description of the last non-OK status. */
const char* spamm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SPAMM_H */
