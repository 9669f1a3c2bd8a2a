/*
 * mra.h -- C ABI of the MI355X (gfx950) library for the multi-resolution
 * approximation (MRA) of a Gaussian process: partition build, log-likelihood
 * and kriging.
 *
 * The method is the one whose CPU implementation is described by Huang, Blake
 * & Hammerling ("Pushing the Limit: A Hybrid Parallel Implementation of the
 * Multi-resolution Approximation for Massive Data"):
 *   - the process and its remainder covariances, Sec. 1.1;
 *   - the J-ary partition, half-open regions, the one-percent extension of
 *     the root and the grid knots, Sec. 1.2 and Appendix A;
 *   - the calculation modes (build structure, likelihood, prediction) and the
 *     covariance parameters sill/range/nugget, Sec. 2.2 (user parameters);
 *   - the data file layout (n, then longitudes, latitudes, values as 64-bit
 *     reals), Sec. 2.2.
 *
 * All arithmetic is FP64.  Status codes are returned; no exception crosses
 * the ABI.  mra_last_error() gives a thread-local message for the last
 * failing call on the calling thread.
 */
#ifndef MRA_H
#define MRA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mra_tree mra_tree;

/* status codes */
#define MRA_OK 0
#define MRA_EINVAL (-1)  /* invalid argument */
#define MRA_ENOTPD (-2)  /* a Cholesky pivot was not positive: matrix not positive definite */
#define MRA_ENOMEM (-3)  /* device or host allocation failed */
#define MRA_EDEVICE (-4) /* HIP runtime error, or no gfx950 device */
#define MRA_EDOMAIN (-5) /* a location lies outside the root region */

/* covariance families; distance t = |a - b| / range (Euclidean, in the plane)
 *   MRA_EXP           : sill * exp(-t)                  (the paper's exponential)
 *   MRA_MATERN nu=0.5 : sill * exp(-t)
 *   MRA_MATERN nu=1.5 : sill * (1 + t) * exp(-t)
 *   MRA_MATERN nu=2.5 : sill * (1 + t + t^2/3) * exp(-t)
 *   MRA_GAUSS         : sill * exp(-t^2)   (nu ignored; its knot matrices become
 *                       singular in FP64 once the knot spacing is well below the
 *                       range, which mra_loglik reports as MRA_ENOTPD)           */
#define MRA_EXP 0
#define MRA_MATERN 1
#define MRA_GAUSS 2

/* mra_build_tree flags */
#define MRA_DEVICE_PTRS (1u << 0)  /* x, y, z are device pointers (else host) */
#define MRA_ELIM_DUPLICATES (1u << 1)    /* drop repeated locations, keep the first (Sec. 2.2,
                                            ELIMINATION_DUPLICATES_FLAG) */
#define MRA_ALLOW_ZERO_NUGGET (1u << 2)  /* mra_loglik accepts tau = 0 (noise-free data) */
#define MRA_FURTHER_APPROX (1u << 3)     /* r knots at the finest level too (Sec. 1.2, the further
                                            approximation): the finest-level remainder of each leaf is
                                            represented by its knots' predictive process instead of
                                            being kept exact; mra_predict refuses such a tree */
#define MRA_FOLD_GRAM (1u << 4)    /* fold every region in knot space (Gram form) */
#define MRA_FOLD_FACTOR (1u << 5)  /* fold in observation space wherever scratch allows */

/*
 * Build the multi-resolution partition (Sec. 1.2).
 *   x, y, z : n locations and values (host memory, or device memory with
 *             MRA_DEVICE_PTRS).  Read during the call only; the library keeps
 *             its own device copy, so the caller may free them on return.
 *             A NaN value marks a location without an observation: it is left
 *             out of the likelihood.  Non-finite locations -> MRA_EINVAL.
 *   J       : 2 (split the longer side, x on a tie) or 4 (halve both sides).
 *   r       : requested knots per region above the finest level; the knots
 *             form a ceil(sqrt r) x floor(r / ceil(sqrt r)) grid, so
 *             r_hat = that product knots are placed.  The library supports
 *             r_hat <= 64 (MRA_EINVAL beyond).
 *   M       : number of levels, >= 1.  The finest level holds the observations
 *             as its knots.  M <= 0 selects the default of Sec. 2.2: the M for
 *             which the finest level's average count per region, n_obs /
 *             J^(M-1), is closest on a log scale to r_hat (n_obs: inputs with
 *             a value; M = 1 when n_obs <= r_hat), i.e.
 *             M = 1 + max(0, floor(log_J(n_obs / r_hat) + 1/2)).
 *   offset  : knot offset as a fraction of the region side; <= 0 selects the
 *             default e/100 (Sec. 1.2, Appendix A).
 *   domain4 : {xmin, xmax, ymin, ymax} of the root region, used verbatim, or
 *             NULL for the data bounding box with its right and top sides
 *             pushed out by one percent of the side length.  An observation
 *             outside the half-open root region -> MRA_EDOMAIN.
 *   out     : receives an opaque, immutable, library-owned handle; release it
 *             with mra_free_tree.
 * Observations that coincide exactly with a knot of an ancestor region above
 * the finest level are dropped (Sec. 1.2).  With MRA_ELIM_DUPLICATES, an
 * observation whose two coordinates equal (==) those of an earlier observation
 * with a value is dropped too, the first one kept (Sec. 2.2, the duplicate
 * elimination user parameter); without it repeated locations stay, and the
 * likelihood needs a positive nugget.  Requires a gfx950 device (the current
 * HIP device); the tree's device arrays live on it.
 */
int mra_build_tree(const double *x, const double *y, const double *z, int64_t n, int J, int r, int M,
                   double offset, uint32_t flags, const double *domain4, mra_tree **out);

/*
 * MRA log-likelihood for B covariance-parameter vectors (likelihood mode,
 * Sec. 2.2): loglik[b] = log N(z; 0, Sigma_MRA(theta_b) + tau_b I), where
 * Sigma_MRA is the covariance of tau_1 + ... + tau_M of Sec. 1.1 at the
 * observations, including the -n/2 log(2 pi) constant.
 *   family, nu : MRA_EXP (nu ignored) or MRA_MATERN with nu = 0.5 or 1.5.
 *   theta      : B x 3 row-major {sill alpha, range beta, nugget tau}, all > 0
 *                (tau = 0 allowed for a tree built with MRA_ALLOW_ZERO_NUGGET).
 *   loglik     : B outputs.  theta and loglik are both host or both device
 *                pointers.
 *   stream     : hipStream_t (NULL = the null stream).  With device pointers
 *                the call is asynchronous on the stream; with host pointers it
 *                returns after the results are written.
 * The tree is read-only: concurrent calls on different streams are allowed.
 * Errors: MRA_EINVAL (bad family/nu/theta), MRA_ENOTPD (message names theta
 * index, level and region), MRA_ENOMEM, MRA_EDEVICE.  With device pointers
 * the call returns before the kernels run: a theta whose factorisation fails
 * (or a device theta that is not valid) yields NaN in its output, and
 * mra_loglik_status reports the failure as MRA_ENOTPD / MRA_EINVAL.
 */
int mra_loglik(const mra_tree *tree, int family, double nu, const double *theta, int64_t B,
               double *loglik, void *stream);

/*
 * The two terms of the log-likelihood per theta, besides loglik itself:
 *   loglik = -1/2 [ n_used log(2 pi) + logdet + quad ],
 *   logdet = log det (Sigma_MRA + tau I),  quad = z^T (Sigma_MRA + tau I)^{-1} z.
 * Since Sigma_MRA scales with the sill, at fixed range and nugget-to-sill
 * ratio the log-likelihood is maximised over the sill in closed form from
 * these two terms (sill_hat = sill * quad / n_used).  logdet and quad are
 * optional (NULL); memory space, stream and errors as for mra_loglik.
 */
int mra_loglik_terms(const mra_tree *tree, int family, double nu, const double *theta, int64_t B,
                     double *loglik, double *logdet, double *quad, void *stream);

/*
 * Per-level breakdown of the log-determinant term, to localise a
 * disagreement with another implementation: level_logdet[b * M + (m - 1)] is
 * the sum over the level-m regions of their log-determinant contributions
 * (finest level: log det of each region's finest-level covariance plus nugget;
 * above it: log det (B + At) - log det B of each fold, in the notation of the
 * prior/posterior recursion), for m = 1 .. M; the M values add up to
 * log det(Sigma_MRA + tau I).  loglik as for mra_loglik.  Memory spaces,
 * stream and errors as for mra_loglik (host outputs: the call is synchronous);
 * these calls are not graph-captured.
 */
int mra_loglik_levels(const mra_tree *tree, int family, double nu, const double *theta, int64_t B,
                      double *loglik, double *level_logdet, void *stream);

/*
 * mra_loglik for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * same kernels as mra_loglik, but every buffer beyond the inputs and outputs
 * lives in one fixed array of 64 MiB of device memory per GPU, created when
 * the library is loaded and held until the process ends; this call allocates
 * nothing and creates no HIP object.
 *   theta, loglik : device pointers (B x 3 and B), on the tree's device, which
 *                   must be the current device; the call is asynchronous on
 *                   `stream`.
 * Trees whose one-theta working set (V stores, finest-level factors, Gram
 * blocks, one workgroup slot) exceeds 64 MiB -> MRA_ENOMEM, with the size in
 * the message (a tree of a few thousand observations at r = 32 fits; the
 * theta batch is processed in chunks that fit).  Every call on a GPU uses that
 * GPU's array: calls that overlap in time on one GPU (different streams or
 * threads) race and must be serialised by the caller.  A failed factorisation
 * gives NaN for that theta (no status is kept).
 */
int mra_loglik_noalloc(const mra_tree *tree, int family, double nu, const double *theta, int64_t B,
                       double *loglik, void *stream);

/*
 * Status of the most recent mra_loglik / mra_loglik_terms call on this tree
 * (for callers that pass device pointers, whose calls return before the
 * kernels run).  Waits for that call's work on its stream, then returns
 * MRA_OK, MRA_ENOTPD (a Cholesky pivot was not positive; mra_last_error names
 * the first such theta index, level and region) or MRA_EINVAL (a theta that
 * is not finite and positive).  MRA_EINVAL with "no evaluation" if the tree
 * has none.  MRA_EDEVICE if a finest-level task of a theta that shares its
 * prior gave up its bounded wait for the others of its group (an internal
 * scheduling fault, not expected; the group's outputs are NaN).
 */
int mra_loglik_status(const mra_tree *tree);

/*
 * Kriging (prediction mode, Sec. 2.2): posterior mean and variance of the
 * latent process X (no nugget) at np locations given the tree's observations.
 * Each location joins the finest-level region that contains it.
 *   theta    : 3 values {alpha, beta, tau}.
 *   px, py   : np locations; mean, var : np outputs.  All host or all device
 *              pointers (same memory space).
 * A location outside the root region -> MRA_EDOMAIN (nothing is clamped).
 */
int mra_predict(const mra_tree *tree, int family, double nu, const double *theta, const double *px,
                const double *py, int64_t np, double *mean, double *var, void *stream);

/* Release a tree and its device memory.  NULL is allowed. */
void mra_free_tree(mra_tree *tree);

/* Thread-local description of the last error on this thread ("" if none). */
const char *mra_last_error(void);

typedef struct mra_info {
    int64_t n_in, n_nan, n_elim, n_used; /* inputs, NaN values, knot coincidences dropped, used */
    int32_t J, M, r, r_hat, P;           /* P = r_hat padded to the kernel tile (16, 32 or 64) */
    int64_t n_regions, n_leaves;
    int64_t leaf_min, leaf_max;          /* observations per finest-level region */
    int64_t n_gram_regions;              /* regions folded in knot space */
    int64_t n_dup;                       /* repeated locations dropped (MRA_ELIM_DUPLICATES) */
    int64_t leaf_hist[16];               /* finest-level regions by observation count c:
                                            [0] c = 0, [b] 2^(b-1) <= c < 2^b (b = 1..14),
                                            [15] c >= 2^14 */
} mra_info;

/* Structure summary (the build-structure-only mode of Sec. 2.2). */
int mra_tree_info(const mra_tree *tree, mra_info *info);

/*
 * Copy of the tree's used observations in the library's internal order
 * (grouped by finest-level region, input order kept inside a region), the
 * input index of each, and the per-leaf offsets (n_leaves + 1).  Host
 * pointers; any may be NULL.
 */
int mra_tree_arrays(const mra_tree *tree, double *x, double *y, double *z, int64_t *orig,
                    int64_t *leaf_off);

/*
 * Execution plan (scheduling only: results change by rounding at most).
 * Each region above the finest level folds either in observation space
 * (regions whose subtree holds few observations) or in knot space; leaves
 * and small folds of up to small_max rows run on one-wave finishers, larger
 * ones on workgroup kernels.
 *
 * mra_autotune times one evaluation of a host sample theta (B x 3) under
 * candidate plans -- per level, the observation-space threshold in
 * {0, 64, ..., 768}, then per level the tile shape of the knot-space Schur
 * blocks, then small_max in {64, 32, 16} -- keeps each choice that
 * is at least 2 % faster, installs the best plan in the tree and reports it.
 * mra_set_plan installs a plan directly (fold_max: M - 1 entries for levels
 * 1 .. M-1, -1 = the default rule; or NULL), e.g. one cached from an earlier
 * autotune.  Both drop the tree's evaluation workspace; they must not run
 * concurrently with other calls on the same tree.  Trees built with
 * MRA_FOLD_GRAM or MRA_FOLD_FACTOR cannot be tuned (MRA_EINVAL).
 */
typedef struct mra_tune_result {
    int32_t levels;        /* M */
    int32_t small_max;     /* 16, 32 or 64 */
    int64_t fold_max[16];  /* [m - 1]: threshold of level m = 1 .. M-1 */
    double ms_before;      /* one evaluation of the sample with the plan on entry */
    double ms_after;       /* ... with the plan installed */
    int32_t trials;        /* plans timed */
    int32_t tile[16];      /* [m - 1]: tile shape of level m's knot-space Schur blocks:
                              0 64 x 64 blocks (one wave each), 1 128 x 128 super-blocks
                              (one workgroup each, rows staged through LDS) */
} mra_tune_result;

int mra_autotune(mra_tree *tree, int family, double nu, const double *theta, int64_t B, mra_tune_result *out);
int mra_set_plan(mra_tree *tree, const int64_t *fold_max, int small_max);

/*
 * Tile shape of each level's knot-space Schur blocks (tile: M - 1 entries
 * for levels 1 .. M-1: -1 the default rule -- super-blocks when the level's
 * median region has at least 128 rows of observation-space children -- 0
 * 64 x 64 blocks, 1 128 x 128 super-blocks; NULL: all default).  mra_autotune
 * also times the alternative shape of every level with knot-space folds.
 * Same workspace rules as mra_set_plan.
 */
int mra_set_tile_shapes(mra_tree *tree, const int32_t *tile);

/*
 * Parameter vectors that share alpha and the range share the prior (every
 * level above the finest and the observations' whitened rows: the nugget
 * enters the finest level only, Sec. 1.1).  Within each chunk of theta that
 * device memory allows, mra_loglik computes the prior once per distinct
 * (alpha, range) -- found on the device, so captured graphs follow new values
 * -- and the other theta of the chunk reuse it, with results identical to
 * evaluating each theta alone.  A caller whose theta come in consecutive
 * groups of g with the same (alpha, range) (for instance a grid with g
 * nuggets per range) calls this with multiple = g, so that chunk sizes are
 * multiples of g and no group is split between chunks (multiple = 1: no
 * rounding, the default).  The environment variable MRA_SHARE_PRIOR=0
 * switches the sharing off.  Returns MRA_EINVAL for multiple < 1.  Same
 * workspace rules as mra_set_plan.
 */
int mra_set_chunk_multiple(mra_tree *tree, int64_t multiple);

/*
 * Optional per-launch timing, for measurement.  While enabled, every kernel
 * launch of mra_loglik is bracketed by HIP events on the caller's stream, or,
 * with only_kernel non-NULL, only the launches of that kernel at only_level
 * (the names mra_profile_read reports; MRA_EINVAL for an unknown name).
 * mra_profile_read waits for the recorded events, aggregates them by kernel
 * and level (elapsed milliseconds, launch count, and the algorithmic FP64
 * flops of what those launches computed, padding excluded), writes up to
 * cap entries, sets *count to the number of entries and clears the record.
 * Process-wide; not meant to be toggled while other threads run mra_loglik.
 */
typedef struct mra_kernel_stat {
    char name[32];
    int32_t level;
    int64_t launches;
    double ms;
    double flops;
} mra_kernel_stat;

int mra_profile_enable(int on, const char *only_kernel, int only_level);
int mra_profile_read(mra_kernel_stat *out, int cap, int *count);

/*
 * Achievable FP64 matrix-core rate of the current device, for measurement:
 * 8 workgroups of 4 waves per compute unit each issue `iters` rounds of 8
 * independent 16x16x4 FP64 matrix instructions on register operands; *tflops
 * receives (flops issued) / (kernel time).  Allocates and frees a small
 * output buffer.  Errors: MRA_EINVAL, MRA_EDEVICE, MRA_ENOMEM.
 */
int mra_bench_mfma_f64(int64_t iters, double *tflops);

#ifdef __cplusplus
}
#endif
#endif /* MRA_H */
