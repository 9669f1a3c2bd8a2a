/*
 * mra_oracle.c -- CPU oracle for the multi-resolution approximation (MRA)
 * log-likelihood and kriging.  TEST INFRASTRUCTURE ONLY: only the test
 * suite, the smoke check and the CPU baseline of the benchmark may load it.
 * The product path never calls into this file and shares no code with it.
 *
 * Plain C, FP64 everywhere, no BLAS, no blocking.  Every function names the
 * passage of the paper (Huang, Blake & Hammerling, "Pushing the Limit: A
 * Hybrid Parallel Implementation of the Multi-resolution Approximation for
 * Massive Data") that it follows.
 *
 * Two independent routes to the same number:
 *  (i)  oracle_dense_*  : the definition.  The remainder covariances
 *       C_{m+1} = C_m - C_m(.,Q) C_m(Q,Q)^{-1} C_m(Q,.) inside each region,
 *       zero across regions (Sec. 1.1, the C_2 ... C_M display), summed into
 *       the MRA covariance of the observations (the tau_1+...+tau_M
 *       expansion), and the Gaussian log-density of the data under it.
 *       O(n^3); used for n of a few thousand.
 *  (ii) oracle_mra_loglik : the prior/posterior recursion that reaches the
 *       same number region by region.  The paper names its statistics
 *       (ATilde: conditional (co)variances of the ancestors, Sec. 4.2 and
 *       Appendix B) but does not print the algebra; it is derived from the
 *       definitions with the Woodbury identity and the matrix determinant
 *       lemma and written here in its plain form (B, K = B^{-1}, A, omega).
 *       Pinned against (i) by the test suite.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>

#define O_OK 0
#define O_EINVAL (-1)
#define O_ENOTPD (-2)
#define O_ENOMEM (-3)
#define O_EDOMAIN (-5)

#define O_MAXLEV 24

static char o_err[512];
const char *oracle_last_error(void) { return o_err; }
static int fail(int code, const char *msg) {
    snprintf(o_err, sizeof o_err, "%s", msg);
    return code;
}

/* build flags (same values as the library's) */
#define O_ELIM_DUPLICATES (1u << 1) /* drop repeated locations, keep the first (Sec. 2.2) */
#define O_ALLOW_ZERO_NUGGET (1u << 2) /* accept tau = 0 in the likelihood */
/* r knots at the finest level too (Sec. 1.2, the further approximation):
 * the finest-level remainder is represented by its knots, not kept exact */
#define O_FURTHER_APPROX (1u << 3)

typedef struct otree {
    int J, M, r, nx, ny, rhat;
    double offset;
    uint32_t flags;
    int64_t n_in, n_nan, n_elim, n_used, n_dup;
    int64_t nreg, nleaf;
    int64_t lvl_start[O_MAXLEV + 1]; /* first level-order index of each level (0-based level) */
    double *box;                     /* nreg x 4 : xlo xhi ylo yhi */
    int64_t *leaf_off;               /* nleaf + 1 */
    double *x, *y, *z;               /* used observations, grouped by leaf, input order kept */
    int64_t *orig;                   /* input index of each used observation */
} otree;

/* ------------------------------------------------------------------------ */
/* Structure (Sec. 1.2)                                                      */
/* ------------------------------------------------------------------------ */

/* Number of x and y grid bars: ceil(sqrt(r)) and floor(r / ceil(sqrt(r))),
 * Sec. 1.2 (knot placement).  Integer arithmetic only. */
static void grid_dims(int r, int *nx, int *ny) {
    int a = 1;
    while ((int64_t)a * a < r) a++;
    *nx = a;
    *ny = r / a;
}

/* Grid bar positions along one axis of a region [lo, hi): the first bar sits
 * offset*length from lo, consecutive bars are length*(1-2*offset)/(nb-1)
 * apart (relative-offset form of Appendix A; the last bar lands at
 * hi - offset*length).  A single bar sits at lo + offset*length. */
static void grid_bars(double lo, double hi, int nb, double f, double *out) {
    double L = hi - lo;
    for (int p = 0; p < nb; p++) {
        if (nb == 1)
            out[p] = lo + f * L;
        else
            out[p] = (lo + f * L) + (((double)p * L) * (1.0 - 2.0 * f)) / (double)(nb - 1);
    }
}

int oracle_grid_dims(int r, int *nx, int *ny) {
    if (r < 1) return fail(O_EINVAL, "r < 1");
    grid_dims(r, nx, ny);
    return O_OK;
}

/* Knots of a box: index q*nx + p (x fastest). */
int oracle_box_knots(double xlo, double xhi, double ylo, double yhi, int r, double offset,
                     double *kx, double *ky) {
    int nx, ny;
    if (r < 1) return fail(O_EINVAL, "r < 1");
    grid_dims(r, &nx, &ny);
    double xb[4096], yb[4096];
    if (nx > 4096 || ny > 4096) return fail(O_EINVAL, "r too large");
    grid_bars(xlo, xhi, nx, offset, xb);
    grid_bars(ylo, yhi, ny, offset, yb);
    for (int q = 0; q < ny; q++)
        for (int p = 0; p < nx; p++) {
            kx[q * nx + p] = xb[p];
            ky[q * nx + p] = yb[q];
        }
    return O_OK;
}

/* Child box j of a parent box (Sec. 1.2).  J = 4: both sides halved, children
 * numbered (x-lo,y-lo), (x-hi,y-lo), (x-lo,y-hi), (x-hi,y-hi).  J = 2: the
 * longer side is halved (x on a tie), children (lo, hi). */
static void child_box(const double *pb, int J, int j, double *cb) {
    double xlo = pb[0], xhi = pb[1], ylo = pb[2], yhi = pb[3];
    double mx = 0.5 * (xlo + xhi), my = 0.5 * (ylo + yhi);
    if (J == 4) {
        cb[0] = (j & 1) ? mx : xlo;
        cb[1] = (j & 1) ? xhi : mx;
        cb[2] = (j & 2) ? my : ylo;
        cb[3] = (j & 2) ? yhi : my;
    } else {
        int splitx = (xhi - xlo) >= (yhi - ylo);
        cb[0] = xlo; cb[1] = xhi; cb[2] = ylo; cb[3] = yhi;
        if (splitx) { if (j) cb[0] = mx; else cb[1] = mx; }
        else        { if (j) cb[2] = my; else cb[3] = my; }
    }
}

/* Which child of box pb holds (px, py): regions are half-open, a coordinate
 * equal to the midpoint belongs to the upper child (Sec. 1.2). */
static int child_of(const double *pb, int J, double px, double py) {
    double xlo = pb[0], xhi = pb[1], ylo = pb[2], yhi = pb[3];
    double mx = 0.5 * (xlo + xhi), my = 0.5 * (ylo + yhi);
    if (J == 4) return (px >= mx ? 1 : 0) + (py >= my ? 2 : 0);
    int splitx = (xhi - xlo) >= (yhi - ylo);
    return splitx ? (px >= mx) : (py >= my);
}

static int64_t ipow(int64_t b, int e) {
    int64_t v = 1;
    while (e-- > 0) v *= b;
    return v;
}

void oracle_mra_free_tree(otree *t) {
    if (!t) return;
    free(t->box); free(t->leaf_off); free(t->x); free(t->y); free(t->z); free(t->orig);
    free(t);
}

/* Build the partition (Sec. 1.2).  NaN-valued observations are prediction
 * locations and do not enter the likelihood.  The root box is the data box
 * with its top and right sides pushed out by one percent of the side length
 * (one percent of 1.0 for a degenerate side) unless domain4 is given, which is
 * used verbatim.  An observation that coincides exactly with a knot of one of
 * its ancestors above the finest level is dropped. */
/* Order of observation indices by location, then input index (for the
 * duplicate search: equal locations become neighbours, first one first). */
static const double *g_dx, *g_dy;
static int cmp_loc(const void *pa, const void *pb) {
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    if (g_dx[a] < g_dx[b]) return -1;
    if (g_dx[a] > g_dx[b]) return 1;
    if (g_dy[a] < g_dy[b]) return -1;
    if (g_dy[a] > g_dy[b]) return 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

int oracle_mra_build_tree(const double *x, const double *y, const double *z, int64_t n, int J,
                          int r, int M, double offset, uint32_t flags, const double *domain4,
                          otree **out) {
    *out = NULL;
    if (n < 0 || (J != 2 && J != 4) || r < 1 || M < 1 || M > O_MAXLEV)
        return fail(O_EINVAL, "bad n/J/r/M");
    if (!(offset > 0.0)) offset = exp(1.0) / 100.0;
    for (int64_t i = 0; i < n; i++)
        if (!isfinite(x[i]) || !isfinite(y[i])) return fail(O_EINVAL, "non-finite location");
    otree *t = calloc(1, sizeof *t);
    if (!t) return fail(O_ENOMEM, "oom");
    t->J = J; t->M = M; t->r = r; t->offset = offset; t->flags = flags;
    grid_dims(r, &t->nx, &t->ny);
    t->rhat = t->nx * t->ny;
    t->n_in = n;
    t->nleaf = ipow(J, M - 1);
    t->nreg = 0;
    for (int m = 0; m < M; m++) { t->lvl_start[m] = t->nreg; t->nreg += ipow(J, m); }
    t->lvl_start[M] = t->nreg;
    t->box = malloc(sizeof(double) * 4 * t->nreg);
    t->leaf_off = calloc(t->nleaf + 1, sizeof(int64_t));
    if (!t->box || !t->leaf_off) { oracle_mra_free_tree(t); return fail(O_ENOMEM, "oom"); }

    double rb[4];
    if (domain4) {
        rb[0] = domain4[0]; rb[1] = domain4[1]; rb[2] = domain4[2]; rb[3] = domain4[3];
        if (!(rb[1] > rb[0]) || !(rb[3] > rb[2])) { oracle_mra_free_tree(t); return fail(O_EINVAL, "bad domain"); }
    } else {
        double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
        for (int64_t i = 0; i < n; i++) {
            if (x[i] < xmin) xmin = x[i];
            if (x[i] > xmax) xmax = x[i];
            if (y[i] < ymin) ymin = y[i];
            if (y[i] > ymax) ymax = y[i];
        }
        if (n == 0) { xmin = ymin = 0.0; xmax = ymax = 1.0; }
        double lx = xmax - xmin, ly = ymax - ymin;
        rb[0] = xmin; rb[1] = xmax + 0.01 * (lx > 0.0 ? lx : 1.0);
        rb[2] = ymin; rb[3] = ymax + 0.01 * (ly > 0.0 ? ly : 1.0);
    }
    memcpy(t->box, rb, sizeof rb);
    for (int m = 0; m + 1 < M; m++)
        for (int64_t k = 0; k < ipow(J, m); k++)
            for (int j = 0; j < J; j++)
                child_box(t->box + 4 * (t->lvl_start[m] + k), J, j,
                          t->box + 4 * (t->lvl_start[m + 1] + J * k + j));

    /* repeated locations (optional, the ELIMINATION_DUPLICATES_FLAG of
     * Sec. 2.2): among observations with a value, one whose two coordinates
     * equal those of an earlier one is dropped; the first is kept */
    char *dup = calloc(n > 0 ? n : 1, 1);
    if (!dup) { oracle_mra_free_tree(t); return fail(O_ENOMEM, "oom"); }
    if (flags & O_ELIM_DUPLICATES) {
        int64_t *ord = malloc(sizeof(int64_t) * (n > 0 ? n : 1));
        int64_t nv = 0;
        for (int64_t i = 0; i < n; i++) if (!isnan(z[i])) ord[nv++] = i;
        g_dx = x; g_dy = y;
        qsort(ord, nv, sizeof(int64_t), cmp_loc);
        for (int64_t s2 = 1; s2 < nv; s2++) {
            int64_t a = ord[s2 - 1], b = ord[s2];
            if (x[a] == x[b] && y[a] == y[b]) dup[b] = 1; /* b comes later in the input than a */
        }
        free(ord);
    }

    /* assign every observation to its leaf, eliminating knot coincidences */
    int64_t *leaf = malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    if (!leaf) { free(dup); oracle_mra_free_tree(t); return fail(O_ENOMEM, "oom"); }
    double *xb = malloc(sizeof(double) * t->nx), *yb = malloc(sizeof(double) * t->ny);
    int64_t used = 0;
    for (int64_t i = 0; i < n; i++) {
        leaf[i] = -1;
        if (isnan(z[i])) { t->n_nan++; continue; }
        if (x[i] < rb[0] || x[i] >= rb[1] || y[i] < rb[2] || y[i] >= rb[3]) {
            free(leaf); free(dup); free(xb); free(yb); oracle_mra_free_tree(t);
            return fail(O_EDOMAIN, "observation outside the root domain");
        }
        if (dup[i]) { t->n_dup++; continue; }
        int64_t k = 0;
        int hit = 0;
        for (int m = 0; m < M; m++) {
            const double *b = t->box + 4 * (t->lvl_start[m] + k);
            if (m + 1 < M) {
                /* knot check against this ancestor (levels above the finest) */
                grid_bars(b[0], b[1], t->nx, offset, xb);
                grid_bars(b[2], b[3], t->ny, offset, yb);
                int hx = 0, hy = 0;
                for (int p = 0; p < t->nx; p++) if (x[i] == xb[p]) hx = 1;
                for (int q = 0; q < t->ny; q++) if (y[i] == yb[q]) hy = 1;
                if (hx && hy) hit = 1;
                k = J * k + child_of(b, J, x[i], y[i]);
            }
        }
        if (hit) { t->n_elim++; continue; }
        leaf[i] = k;
        used++;
    }
    free(xb); free(yb); free(dup);
    t->n_used = used;
    t->x = malloc(sizeof(double) * (used > 0 ? used : 1));
    t->y = malloc(sizeof(double) * (used > 0 ? used : 1));
    t->z = malloc(sizeof(double) * (used > 0 ? used : 1));
    t->orig = malloc(sizeof(int64_t) * (used > 0 ? used : 1));
    /* stable grouping by leaf (counting sort) */
    for (int64_t i = 0; i < n; i++) if (leaf[i] >= 0) t->leaf_off[leaf[i] + 1]++;
    for (int64_t k = 0; k < t->nleaf; k++) t->leaf_off[k + 1] += t->leaf_off[k];
    int64_t *fill = malloc(sizeof(int64_t) * t->nleaf);
    memcpy(fill, t->leaf_off, sizeof(int64_t) * t->nleaf);
    for (int64_t i = 0; i < n; i++) {
        if (leaf[i] < 0) continue;
        int64_t d = fill[leaf[i]]++;
        t->x[d] = x[i]; t->y[d] = y[i]; t->z[d] = z[i]; t->orig[d] = i;
    }
    free(fill); free(leaf);
    *out = t;
    return O_OK;
}

/* Accessors used by the tests. */
int oracle_tree_dims(const otree *t, int64_t *v) {
    v[0] = t->n_in; v[1] = t->n_nan; v[2] = t->n_elim; v[3] = t->n_used;
    v[4] = t->nreg; v[5] = t->nleaf; v[6] = t->rhat; v[7] = t->nx; v[8] = t->ny;
    v[9] = t->n_dup;
    return O_OK;
}
int oracle_tree_arrays(const otree *t, double *x, double *y, double *z, int64_t *orig,
                       int64_t *leaf_off, double *box) {
    if (x) memcpy(x, t->x, sizeof(double) * t->n_used);
    if (y) memcpy(y, t->y, sizeof(double) * t->n_used);
    if (z) memcpy(z, t->z, sizeof(double) * t->n_used);
    if (orig) memcpy(orig, t->orig, sizeof(int64_t) * t->n_used);
    if (leaf_off) memcpy(leaf_off, t->leaf_off, sizeof(int64_t) * (t->nleaf + 1));
    if (box) memcpy(box, t->box, sizeof(double) * 4 * t->nreg);
    return O_OK;
}

/* ------------------------------------------------------------------------ */
/* Covariance.  Exponential (the only family in the paper's code, Sec. 2.2), */
/* Matern nu = 3/2 and 5/2, and Gaussian, as functions of t = distance/range: */
/*   nu = 1/2 : alpha * exp(-t);   nu = 3/2 : alpha * (1 + t) * exp(-t);       */
/*   nu = 5/2 : alpha * (1 + t + t^2/3) * exp(-t);  Gaussian: alpha exp(-t^2). */
/* Euclidean distance in the (x, y) plane; the nugget is not part of C.       */
/* ------------------------------------------------------------------------ */
typedef struct { double alpha, beta, tau; int smooth; } cpar; /* smooth: 0 -> 1/2, 1 -> 3/2, 2 -> 5/2, 3 -> Gaussian */

static double cov(double ax, double ay, double bx, double by, const cpar *c) {
    double dx = ax - bx, dy = ay - by;
    double t = sqrt(dx * dx + dy * dy) / c->beta;
    if (c->smooth == 3) return c->alpha * exp(-t * t);            /* Gaussian */
    if (c->smooth == 2) return c->alpha * (1.0 + t + t * t / 3.0) * exp(-t); /* Matern 5/2 */
    if (c->smooth == 1) return c->alpha * (1.0 + t) * exp(-t);    /* Matern 3/2 */
    return c->alpha * exp(-t);                                    /* exponential, Matern 1/2 */
}

static int make_par(int family, double nu, const double *th, cpar *c) {
    if (!(th[0] > 0.0) || !(th[1] > 0.0) || !(th[2] >= 0.0)) return fail(O_EINVAL, "theta must be positive");
    c->alpha = th[0]; c->beta = th[1]; c->tau = th[2];
    if (family == 0) { c->smooth = 0; return O_OK; }
    if (family == 1 && nu == 0.5) { c->smooth = 0; return O_OK; }
    if (family == 1 && nu == 1.5) { c->smooth = 1; return O_OK; }
    if (family == 1 && nu == 2.5) { c->smooth = 2; return O_OK; }
    if (family == 2) { c->smooth = 3; return O_OK; }
    return fail(O_EINVAL, "unsupported covariance family / nu");
}

/* ------------------------------------------------------------------------ */
/* Small dense kernels (row-major, plain loops)                              */
/* ------------------------------------------------------------------------ */

/* A = L L^T, L kept in the lower triangle.  Returns O_ENOTPD on a
 * non-positive pivot. */
static int chol(double *A, int n) {
    for (int j = 0; j < n; j++) {
        double s = A[(int64_t)j * n + j];
        for (int k = 0; k < j; k++) s -= A[(int64_t)j * n + k] * A[(int64_t)j * n + k];
        if (!(s > 0.0)) return O_ENOTPD;
        double d = sqrt(s);
        A[(int64_t)j * n + j] = d;
        for (int i = j + 1; i < n; i++) {
            double v = A[(int64_t)i * n + j];
            for (int k = 0; k < j; k++) v -= A[(int64_t)i * n + k] * A[(int64_t)j * n + k];
            A[(int64_t)i * n + j] = v / d;
        }
        for (int i = 0; i < j; i++) A[(int64_t)i * n + j] = 0.0;
    }
    return O_OK;
}

/* B (n x m) <- (L L^T)^{-1} B */
static void chol_solve(const double *L, int n, double *B, int m) {
    for (int c = 0; c < m; c++) {
        for (int i = 0; i < n; i++) {
            double v = B[(int64_t)i * m + c];
            for (int k = 0; k < i; k++) v -= L[(int64_t)i * n + k] * B[(int64_t)k * m + c];
            B[(int64_t)i * m + c] = v / L[(int64_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; i--) {
            double v = B[(int64_t)i * m + c];
            for (int k = i + 1; k < n; k++) v -= L[(int64_t)k * n + i] * B[(int64_t)k * m + c];
            B[(int64_t)i * m + c] = v / L[(int64_t)i * n + i];
        }
    }
}

static double logdet_chol(const double *L, int n) {
    double s = 0.0;
    for (int i = 0; i < n; i++) s += log(L[(int64_t)i * n + i]);
    return 2.0 * s;
}

/* ------------------------------------------------------------------------ */
/* The recursion (posterior inference and likelihood, Sec. 1.1 definitions,   */
/* statistics named ATilde in Sec. 4.2 / Appendix B).                          */
/*                                                                            */
/* Prior, for a point set P inside region R at level m (knots of R, or the    */
/* observations of a leaf) and ancestors A_1 .. A_m:                          */
/*   B^l(P) = C(P, Q_{A_l}) - sum_{i<l} B^i(P) K_{A_i} B^i_{A_l}^T ,            */
/*   K_{A_i} = (B^i_{A_i})^{-1}.                                               */
/* B^l(P) = C_l(P, Q_{A_l}), the level-l remainder covariance.                */
/* Leaf R: Sigma_R = C(S,S) - sum_{i<M} B^i K_{A_i} B^i^T + tau I,             */
/*   A^{kl} = B^k^T Sigma^{-1} B^l, w^k = B^k^T Sigma^{-1} z,                  */
/*   d = log det Sigma, u = z^T Sigma^{-1} z.                                  */
/* Region R at level m < M, children c:                                       */
/*   At^{kl} = sum_c A_c^{kl}, wt^k = sum_c w_c^k,                             */
/*   Kt^{-1} = B^m_R + At^{mm},  d = log det Kt^{-1} - log det B^m_R,           */
/*   u = - wt^m^T Kt wt^m,                                                     */
/*   A_R^{kl} = At^{kl} - At^{km} Kt At^{ml},  w_R^k = wt^k - At^{km} Kt wt^m.  */
/* loglik = -1/2 [ n log 2 pi + sum_R (d_R + u_R) ].                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    double *B[O_MAXLEV]; /* B^l_A for l = 1..m of this ancestor (p x p each), 1-based */
    double *L;           /* Cholesky factor of B^m_A */
    double *kx, *ky;     /* knots */
} anc_t;

/* Prediction state, one entry per prediction point (points grouped by leaf):
 * b = [b^1(p) .. b^{M-1}(p)] prior rows, H = [H^1 .. H^{M-1}], mu, v. */
typedef struct {
    int64_t n;
    const double *x, *y;
    const int64_t *leaf_off; /* nleaf + 1 */
    double *b, *H, *mu, *v;
} pred_t;

typedef struct {
    const otree *t;
    cpar c;
    int p;
    anc_t anc[O_MAXLEV + 1]; /* anc[l] = ancestor at level l on the current path */
    double level_sum[O_MAXLEV];
    double level_logdet[O_MAXLEV]; /* the log-determinant terms d alone, per level */
    int status;
    int64_t bad_region;
    pred_t *pred;            /* NULL for the likelihood */
} rctx;

/* B^l(P) for l = 1..Lc, with Z^l = B^l K_{A_l} for l = 1..Lc (Z needed for l < Lc
 * and, for leaves, for Sigma).  When self_last is set the point set is the knot
 * set of A_Lc itself, whose own B^i are the ones being computed. */
static void prior_rows(rctx *ctx, int np, const double *px, const double *py, int Lc,
                       double **B, double **Z) {
    int p = ctx->p;
    for (int l = 1; l <= Lc; l++) {
        anc_t *A = &ctx->anc[l];
        for (int a = 0; a < np; a++)
            for (int b = 0; b < p; b++)
                B[l][(int64_t)a * p + b] = cov(px[a], py[a], A->kx[b], A->ky[b], &ctx->c);
        for (int i = 1; i < l; i++) {
            const double *Bi_Al = A->B[i];
            for (int a = 0; a < np; a++)
                for (int b = 0; b < p; b++) {
                    double s = 0.0;
                    for (int k = 0; k < p; k++) s += Z[i][(int64_t)a * p + k] * Bi_Al[(int64_t)b * p + k];
                    B[l][(int64_t)a * p + b] -= s;
                }
        }
        if (Z[l]) {
            /* Z^l = B^l K_{A_l}  <=>  Z^l^T = K_{A_l} B^l^T */
            double *T = malloc(sizeof(double) * (size_t)p * (np > 0 ? np : 1));
            for (int a = 0; a < np; a++)
                for (int b = 0; b < p; b++) T[(int64_t)b * np + a] = B[l][(int64_t)a * p + b];
            chol_solve(A->L, p, T, np);
            for (int a = 0; a < np; a++)
                for (int b = 0; b < p; b++) Z[l][(int64_t)a * p + b] = T[(int64_t)b * np + a];
            free(T);
        }
    }
}

/* Prior of the knots of non-leaf region k at level m: B^l_R for l = 1..m and
 * the Cholesky factor of B^m_R, stored as ctx->anc[m] (its ancestors must be
 * in ctx->anc[1..m-1]). */
static void prior_region(rctx *ctx, int m, int64_t k) {
    const otree *t = ctx->t;
    int p = ctx->p;
    anc_t *me = &ctx->anc[m];
    const double *bx = t->box + 4 * (t->lvl_start[m - 1] + k);
    me->kx = malloc(sizeof(double) * p);
    me->ky = malloc(sizeof(double) * p);
    oracle_box_knots(bx[0], bx[1], bx[2], bx[3], t->r, t->offset, me->kx, me->ky);
    double *Z[O_MAXLEV + 1] = {0};
    for (int l = 1; l <= m; l++) {
        me->B[l] = malloc(sizeof(double) * p * p);
        Z[l] = (l < m) ? malloc(sizeof(double) * p * p) : NULL;
    }
    /* B^l_R for l < m (ancestors strictly above), then B^m_R from R's own B^i */
    me->L = NULL;
    prior_rows(ctx, p, me->kx, me->ky, m - 1, me->B, Z);
    {
        double *Bm = me->B[m];
        for (int a = 0; a < p; a++)
            for (int b = 0; b < p; b++) {
                double s = cov(me->kx[a], me->ky[a], me->kx[b], me->ky[b], &ctx->c);
                for (int i = 1; i < m; i++)
                    for (int kk = 0; kk < p; kk++) s -= Z[i][(int64_t)a * p + kk] * me->B[i][(int64_t)b * p + kk];
                Bm[(int64_t)a * p + b] = s;
            }
        for (int a = 0; a < p; a++)
            for (int b = 0; b < a; b++) {
                double v = 0.5 * (Bm[(int64_t)a * p + b] + Bm[(int64_t)b * p + a]);
                Bm[(int64_t)a * p + b] = Bm[(int64_t)b * p + a] = v;
            }
        me->L = malloc(sizeof(double) * p * p);
        memcpy(me->L, Bm, sizeof(double) * p * p);
        if (chol(me->L, p)) { ctx->status = O_ENOTPD; ctx->bad_region = t->lvl_start[m - 1] + k; }
    }
    for (int l = 1; l < m; l++) free(Z[l]);
}

static void free_region(rctx *ctx, int m) {
    anc_t *me = &ctx->anc[m];
    for (int l = 1; l <= m; l++) free(me->B[l]);
    free(me->L); free(me->kx); free(me->ky);
    memset(me, 0, sizeof *me);
}

/* Kriging at the finest level (prediction, Sec. 2.2; a point joins the
 * finest-level set of its leaf, so the remainder C_M is used exactly).  For a
 * point p of leaf R with observations S (np of them, Sigma = C_M(S,S) + tau I
 * factored in S_chol, B^l the observations' prior rows):
 *   G = C_M(p, S) = C(p,S) - sum_i b^i(p) K_{A_i} B^i^T,
 *   mu = G Sigma^{-1} z,  H^k = G Sigma^{-1} B^k,
 *   v = C_M(p,p) - G Sigma^{-1} G^T,  C_M(p,p) = C(p,p) - sum_i b^i K_{A_i} b^i^T. */
static void leaf_predict(rctx *ctx, int64_t k, int64_t np, const double *sx, const double *sy, const double *sz,
                         double **B, const double *S_chol) {
    const otree *t = ctx->t;
    pred_t *pr = ctx->pred;
    int p = ctx->p, M = t->M;
    int64_t po = pr->leaf_off[k], pn = pr->leaf_off[k + 1] - po;
    if (pn == 0) return;
    int q = (M - 1) * p;
    const double *qx = pr->x + po, *qy = pr->y + po;
    double *Bp[O_MAXLEV + 1] = {0}, *Zp[O_MAXLEV + 1] = {0};
    for (int l = 1; l < M; l++) {
        Bp[l] = malloc(sizeof(double) * pn * p);
        Zp[l] = malloc(sizeof(double) * pn * p);
    }
    prior_rows(ctx, (int)pn, qx, qy, M - 1, Bp, Zp);
    for (int64_t j = 0; j < pn; j++) {
        double *bj = pr->b + (po + j) * (q > 0 ? q : 1);
        for (int l = 1; l < M; l++)
            for (int c = 0; c < p; c++) bj[(l - 1) * p + c] = Bp[l][j * p + c];
        double cmpp = cov(qx[j], qy[j], qx[j], qy[j], &ctx->c);
        for (int i = 1; i < M; i++)
            for (int c = 0; c < p; c++) cmpp -= Zp[i][j * p + c] * Bp[i][j * p + c];
        pr->mu[po + j] = 0.0;
        pr->v[po + j] = cmpp;
        double *Hj = pr->H + (po + j) * (q > 0 ? q : 1);
        for (int e = 0; e < q; e++) Hj[e] = 0.0;
    }
    if (np > 0) {
        /* Y = Sigma^{-1} G^T  (np x pn) */
        double *G = malloc(sizeof(double) * pn * np);
        double *Y = malloc(sizeof(double) * np * pn);
        for (int64_t j = 0; j < pn; j++)
            for (int64_t a = 0; a < np; a++) {
                double g = cov(qx[j], qy[j], sx[a], sy[a], &ctx->c);
                for (int i = 1; i < M; i++)
                    for (int c = 0; c < p; c++) g -= Zp[i][j * p + c] * B[i][a * p + c];
                G[j * np + a] = g;
                Y[a * pn + j] = g;
            }
        chol_solve(S_chol, (int)np, Y, (int)pn);
        for (int64_t j = 0; j < pn; j++) {
            double mu = 0.0, gy = 0.0;
            for (int64_t a = 0; a < np; a++) {
                mu += Y[a * pn + j] * sz[a];
                gy += G[j * np + a] * Y[a * pn + j];
            }
            pr->mu[po + j] = mu;
            pr->v[po + j] -= gy;
            double *Hj = pr->H + (po + j) * q;
            for (int l = 1; l < M; l++)
                for (int c = 0; c < p; c++) {
                    double h = 0.0;
                    for (int64_t a = 0; a < np; a++) h += Y[a * pn + j] * B[l][a * p + c];
                    Hj[(l - 1) * p + c] = h;
                }
        }
        free(G); free(Y);
    }
    for (int l = 1; l < M; l++) { free(Bp[l]); free(Zp[l]); }
}

/* Fold of the prediction state at region k of level m (after its posterior
 * Kt^{-1} = B^m_R + At^{mm} is factored in Ki): for every prediction point of
 * the subtree, E = b^m(p) - H^m, u = Kt E^T,
 *   mu += u . wt^m,  H^k += u^T At^{m,k} (k < m),  v += E u. */
static void fold_predict(rctx *ctx, int m, int64_t k, const double *Ki, const double *At, const double *wt) {
    const otree *t = ctx->t;
    pred_t *pr = ctx->pred;
    int p = ctx->p, M = t->M;
    int64_t span = 1;
    for (int e = 0; e < M - m; e++) span *= t->J;
    int64_t lo = pr->leaf_off[k * span], hi = pr->leaf_off[(k + 1) * span];
    int q = m * p, qq = (M - 1) * p, o = (m - 1) * p;
    double *E = malloc(sizeof(double) * p);
    for (int64_t j = lo; j < hi; j++) {
        const double *bj = pr->b + j * qq;
        double *Hj = pr->H + j * qq;
        for (int a = 0; a < p; a++) E[a] = bj[(m - 1) * p + a] - Hj[(m - 1) * p + a];
        double *u = malloc(sizeof(double) * p);
        memcpy(u, E, sizeof(double) * p);
        chol_solve(Ki, p, u, 1);
        double dm = 0.0, dv = 0.0;
        for (int a = 0; a < p; a++) { dm += u[a] * wt[o + a]; dv += E[a] * u[a]; }
        pr->mu[j] += dm;
        pr->v[j] += dv;
        for (int kk = 1; kk < m; kk++)
            for (int c = 0; c < p; c++) {
                double h = 0.0;
                for (int a = 0; a < p; a++) h += u[a] * At[(int64_t)(o + a) * q + (kk - 1) * p + c];
                Hj[(kk - 1) * p + c] += h;
            }
        free(u);
    }
    free(E);
}

/* Visit region k at level m (1-based).  On return, A (size (m-1)p square,
 * full), w ((m-1)p) hold the region's statistics for its ancestors 1..m-1, and
 * *du the sum of d+u over the subtree. */
static void visit(rctx *ctx, int m, int64_t k, double *A, double *w, double *du) {
    const otree *t = ctx->t;
    int p = ctx->p, M = t->M;
    *du = 0.0;
    if (ctx->status) return;
    if (m == M) {
        /* leaf */
        int64_t o = t->leaf_off[k], np = t->leaf_off[k + 1] - o;
        int q = (M - 1) * p;
        memset(A, 0, sizeof(double) * (size_t)q * q);
        memset(w, 0, sizeof(double) * (size_t)(q > 0 ? q : 1));
        if (np == 0) {
            if (ctx->pred) leaf_predict(ctx, k, 0, NULL, NULL, NULL, NULL, NULL);
            return;
        }
        const double *px = t->x + o, *py = t->y + o, *pz = t->z + o;
        const int fa = (t->flags & O_FURTHER_APPROX) != 0;
        /* further approximation: the leaf's own knots form level M of the
         * prior, and C_M(S,S) is replaced by B^M K_M B^M^T with
         * B^M = C_M(S, Q_R) */
        if (fa) {
            prior_region(ctx, M, k);
            if (ctx->status) { free_region(ctx, M); return; }
        }
        const int Lc = fa ? M : M - 1;
        double *B[O_MAXLEV + 1] = {0}, *Z[O_MAXLEV + 1] = {0};
        for (int l = 1; l <= Lc; l++) {
            B[l] = malloc(sizeof(double) * np * p);
            Z[l] = malloc(sizeof(double) * np * p);
        }
        prior_rows(ctx, (int)np, px, py, Lc, B, Z);
        double *S = malloc(sizeof(double) * np * np);
        for (int a = 0; a < np; a++)
            for (int b = 0; b < np; b++) {
                double s;
                if (fa) {
                    s = 0.0;
                    for (int kk = 0; kk < p; kk++) s += Z[M][(int64_t)a * p + kk] * B[M][(int64_t)b * p + kk];
                } else {
                    s = cov(px[a], py[a], px[b], py[b], &ctx->c);
                    for (int i = 1; i < M; i++)
                        for (int kk = 0; kk < p; kk++) s -= Z[i][(int64_t)a * p + kk] * B[i][(int64_t)b * p + kk];
                }
                S[(int64_t)a * np + b] = s;
            }
        /* symmetrise the rounding of the two triangles, then add the nugget */
        for (int a = 0; a < np; a++) {
            for (int b = 0; b < a; b++) {
                double v = 0.5 * (S[(int64_t)a * np + b] + S[(int64_t)b * np + a]);
                S[(int64_t)a * np + b] = S[(int64_t)b * np + a] = v;
            }
            S[(int64_t)a * np + a] += ctx->c.tau;
        }
        if (chol(S, (int)np)) { ctx->status = O_ENOTPD; ctx->bad_region = t->lvl_start[M - 1] + k; goto leaf_done; }
        double d = logdet_chol(S, (int)np);
        /* X = Sigma^{-1} [B^1 .. B^{M-1} | z] */
        int wd = q + 1;
        double *X = malloc(sizeof(double) * np * wd);
        for (int a = 0; a < np; a++) {
            for (int l = 1; l < M; l++)
                for (int b = 0; b < p; b++) X[(int64_t)a * wd + (l - 1) * p + b] = B[l][(int64_t)a * p + b];
            X[(int64_t)a * wd + q] = pz[a];
        }
        chol_solve(S, (int)np, X, wd);
        for (int kk = 1; kk < M; kk++)
            for (int ll = 1; ll < M; ll++)
                for (int i = 0; i < p; i++)
                    for (int j = 0; j < p; j++) {
                        double s = 0.0;
                        for (int a = 0; a < np; a++) s += B[kk][(int64_t)a * p + i] * X[(int64_t)a * wd + (ll - 1) * p + j];
                        A[(int64_t)((kk - 1) * p + i) * q + (ll - 1) * p + j] = s;
                    }
        for (int kk = 1; kk < M; kk++)
            for (int i = 0; i < p; i++) {
                double s = 0.0;
                for (int a = 0; a < np; a++) s += B[kk][(int64_t)a * p + i] * X[(int64_t)a * wd + q];
                w[(kk - 1) * p + i] = s;
            }
        double u = 0.0;
        for (int a = 0; a < np; a++) u += pz[a] * X[(int64_t)a * wd + q];
        *du = d + u;
        ctx->level_sum[M - 1] += d + u;
        ctx->level_logdet[M - 1] += d;
        free(X);
        if (ctx->pred) leaf_predict(ctx, k, np, px, py, pz, B, S);
    leaf_done:
        free(S);
        for (int l = 1; l <= Lc; l++) { free(B[l]); free(Z[l]); }
        if (fa) free_region(ctx, M);
        return;
    }

    /* non-leaf region at level m: prior (knots), children, fold */
    anc_t *me = &ctx->anc[m];
    prior_region(ctx, m, k);
    int q = m * p;
    double *At = calloc((size_t)q * q, sizeof(double));
    double *wt = calloc((size_t)q, sizeof(double));
    double *Ac = malloc(sizeof(double) * (size_t)q * q);
    double *wc = malloc(sizeof(double) * (size_t)q);
    double du_sub = 0.0;
    for (int j = 0; j < t->J && !ctx->status; j++) {
        double duc;
        visit(ctx, m + 1, t->J * k + j, Ac, wc, &duc);
        for (int64_t e = 0; e < (int64_t)q * q; e++) At[e] += Ac[e];
        for (int e = 0; e < q; e++) wt[e] += wc[e];
        du_sub += duc;
    }
    free(Ac); free(wc);
    if (!ctx->status) {
        /* Kt^{-1} = B^m_R + At^{mm} */
        int o = (m - 1) * p;
        double *Ki = malloc(sizeof(double) * p * p);
        for (int a = 0; a < p; a++)
            for (int b = 0; b < p; b++)
                Ki[a * p + b] = me->B[m][a * p + b] + At[(int64_t)(o + a) * q + o + b];
        for (int a = 0; a < p; a++)
            for (int b = 0; b < a; b++) {
                double v = 0.5 * (Ki[a * p + b] + Ki[b * p + a]);
                Ki[a * p + b] = Ki[b * p + a] = v;
            }
        if (chol(Ki, p)) {
            ctx->status = O_ENOTPD; ctx->bad_region = t->lvl_start[m - 1] + k;
        } else {
            if (ctx->pred) fold_predict(ctx, m, k, Ki, At, wt);
            double d = logdet_chol(Ki, p) - logdet_chol(me->L, p);
            /* Y = Kt [At^{m,1..m-1} | wt^m]  (p x ((m-1)p + 1)) */
            int qo = (m - 1) * p, wd = qo + 1;
            double *Y = malloc(sizeof(double) * p * wd);
            for (int a = 0; a < p; a++) {
                for (int b = 0; b < qo; b++) Y[a * wd + b] = At[(int64_t)(o + a) * q + b];
                Y[a * wd + qo] = wt[o + a];
            }
            chol_solve(Ki, p, Y, wd);
            double u = 0.0;
            for (int a = 0; a < p; a++) u -= wt[o + a] * Y[a * wd + qo];
            /* children stats for the parent: indices 1..m-1 */
            for (int i = 0; i < qo; i++) {
                for (int j2 = 0; j2 < qo; j2++) {
                    double s = 0.0;
                    for (int a = 0; a < p; a++) s += At[(int64_t)i * q + o + a] * Y[a * wd + j2];
                    A[(int64_t)i * qo + j2] = At[(int64_t)i * q + j2] - s;
                }
                double s = 0.0;
                for (int a = 0; a < p; a++) s += At[(int64_t)i * q + o + a] * Y[a * wd + qo];
                w[i] = wt[i] - s;
            }
            *du = du_sub + d + u;
            ctx->level_sum[m - 1] += d + u;
            ctx->level_logdet[m - 1] += d;
            free(Y);
        }
        free(Ki);
    }
    free(At); free(wt);
    free_region(ctx, m);
}

/* Sum of d + u over the subtree of region k at level `level` for one theta
 * (the ancestors' priors are computed first).  A bounded piece of a full
 * evaluation, used to time the oracle on large workloads. */
int oracle_mra_subtree(const otree *t, int family, double nu, const double *theta, int level, int64_t k,
                       double *du_out) {
    if (level < 1 || level > t->M) return fail(O_EINVAL, "bad level");
    rctx *ctx = calloc(1, sizeof *ctx);
    ctx->t = t;
    ctx->p = t->rhat;
    int rc = make_par(family, nu, theta, &ctx->c);
    if (rc) { free(ctx); return rc; }
    for (int l = 1; l < level; l++) {
        int64_t kl = k;
        for (int e = 0; e < level - l; e++) kl /= t->J;
        prior_region(ctx, l, kl);
    }
    int q = (level - 1) * ctx->p;
    double *A = malloc(sizeof(double) * (size_t)(q > 0 ? q * q : 1));
    double *w = malloc(sizeof(double) * (size_t)(q > 0 ? q : 1));
    double du = 0.0;
    visit(ctx, level, k, A, w, &du);
    for (int l = 1; l < level; l++) free_region(ctx, l);
    free(A); free(w);
    int st = ctx->status;
    free(ctx);
    if (st) return fail(O_ENOTPD, "not positive definite in subtree");
    *du_out = du;
    return O_OK;
}

static const double LOG2PI = 1.8378770664093454835606594728112;

/* Destination of the per-level log-determinant sums while
 * oracle_mra_level_logdets runs (NULL otherwise). */
static double *g_level_logdet = NULL;

/* Log-likelihood of theta[b] = (alpha, beta, tau) for b < B.  level_sums, if
 * given, receives per theta the sum of d + u over each level (M values). */
int oracle_mra_loglik(const otree *t, int family, double nu, const double *theta, int64_t B,
                      double *loglik, double *level_sums) {
    for (int64_t b = 0; b < B; b++) {
        rctx *ctx = calloc(1, sizeof *ctx);
        ctx->t = t;
        ctx->p = t->rhat;
        int rc = make_par(family, nu, theta + 3 * b, &ctx->c);
        if (rc) { free(ctx); return rc; }
        if (!(ctx->c.tau > 0.0) && !((t->flags & O_ALLOW_ZERO_NUGGET) && ctx->c.tau == 0.0)) {
            free(ctx);
            return fail(O_EINVAL, "tau must be positive (zero only with the zero-nugget flag)");
        }
        double dummyA[1], dummyw[1], du = 0.0;
        if (t->M == 1) {
            visit(ctx, 1, 0, dummyA, dummyw, &du);
        } else {
            int q = 0;
            (void)q;
            visit(ctx, 1, 0, dummyA, dummyw, &du);
        }
        if (ctx->status) {
            snprintf(o_err, sizeof o_err, "not positive definite: theta %lld region %lld",
                     (long long)b, (long long)ctx->bad_region);
            free(ctx);
            return O_ENOTPD;
        }
        loglik[b] = -0.5 * ((double)t->n_used * LOG2PI + du);
        if (level_sums)
            for (int m = 0; m < t->M; m++) level_sums[b * t->M + m] = ctx->level_sum[m];
        if (g_level_logdet)
            for (int m = 0; m < t->M; m++) g_level_logdet[b * t->M + m] = ctx->level_logdet[m];
        free(ctx);
    }
    return O_OK;
}

/* Per theta and level m = 1..M, the sum over the level's regions of their
 * log-determinant term d (leaves: log det Sigma_R; folds: log det Kt^{-1} -
 * log det B^m_R); the M values add up to log det(Sigma_MRA + tau I).  out is
 * B x M.  Not thread-safe (it routes the sums through a static pointer). */
int oracle_mra_level_logdets(const otree *t, int family, double nu, const double *theta, int64_t B, double *out) {
    double *ll = malloc(sizeof(double) * (size_t)(B > 0 ? B : 1));
    g_level_logdet = out;
    int rc = oracle_mra_loglik(t, family, nu, theta, B, ll, NULL);
    g_level_logdet = NULL;
    free(ll);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Definitional dense path (Sec. 1.1).                                        */
/*   U = used observations + knots of every region above the finest level.   */
/*   C_1 = C(U, U); for m = 1 .. M-1 and each level-m region R with knots Q:  */
/*     the level-m predictive process contributes C_m(a,Q) C_m(Q,Q)^{-1}      */
/*     C_m(Q,b) to the covariance of observations a, b inside R, and          */
/*     C_{m+1}(a,b) = C_m(a,b) - C_m(a,Q) C_m(Q,Q)^{-1} C_m(Q,b) for points   */
/*     a, b in the same child of R, 0 otherwise.                              */
/*   Finally the leaf remainder C_M(a,b) is added for a, b in the same leaf.  */
/* ------------------------------------------------------------------------ */

/* Leaf of a location by descent from the root (half-open regions). */
static int locate_leaf(const otree *t, double x, double y, int64_t *leaf) {
    const double *rb = t->box;
    if (!(x >= rb[0] && x < rb[1] && y >= rb[2] && y < rb[3])) return O_EDOMAIN;
    int64_t k = 0;
    for (int m = 0; m + 1 < t->M; m++) k = t->J * k + child_of(t->box + 4 * (t->lvl_start[m] + k), t->J, x, y);
    *leaf = k;
    return O_OK;
}

/* Sigma_MRA over the used observations followed by ne extra finest-level
 * points (ex, ey in leaves eleaf): (n + ne) x (n + ne). */
static int dense_sigma_ext(const otree *t, const cpar *c, int64_t ne, const double *ex, const double *ey,
                           const int64_t *eleaf, double *Sig) {
    int64_t n = t->n_used, nn = n + ne;
    int p = t->rhat, M = t->M, J = t->J;
    /* levels with knots: 1..M-1, or 1..M under the further approximation
     * (the observations then sit one level below the finest knots) */
    const int fa = (t->flags & O_FURTHER_APPROX) != 0;
    const int ML = fa ? M : M - 1, RW = M + 2;
    int64_t nk = 0;
    for (int m = 1; m <= ML; m++) nk += ipow(J, m - 1) * p;
    int64_t nU = nn + nk;
    if (nU > 12000) return fail(O_EINVAL, "dense path limited to 12000 points");
    double *ux = malloc(sizeof(double) * nU), *uy = malloc(sizeof(double) * nU);
    int *lev = malloc(sizeof(int) * nU);
    int64_t *reg = malloc(sizeof(int64_t) * nU * RW); /* region index at each level 1..lev */
    double *C = malloc(sizeof(double) * nU * nU);
    if (!ux || !uy || !lev || !reg || !C) {
        free(ux); free(uy); free(lev); free(reg); free(C);
        return fail(O_ENOMEM, "oom");
    }
    /* observations (indices 0..n-1), extra points (n..nn-1), then knots level by level */
    for (int64_t k = 0; k < t->nleaf; k++)
        for (int64_t a = t->leaf_off[k]; a < t->leaf_off[k + 1]; a++) {
            ux[a] = t->x[a]; uy[a] = t->y[a]; lev[a] = ML + 1;
            for (int l = 1; l <= M; l++) reg[a * RW + l] = k / ipow(J, M - l);
            reg[a * RW + M + 1] = -1 - a; /* below the finest knots every observation is alone */
        }
    for (int64_t e = 0; e < ne; e++) {
        int64_t a = n + e;
        ux[a] = ex[e]; uy[a] = ey[e]; lev[a] = ML + 1;
        for (int l = 1; l <= M; l++) reg[a * RW + l] = eleaf[e] / ipow(J, M - l);
        reg[a * RW + M + 1] = -1 - a;
    }
    int64_t u = nn;
    for (int m = 1; m <= ML; m++)
        for (int64_t k = 0; k < ipow(J, m - 1); k++) {
            const double *b = t->box + 4 * (t->lvl_start[m - 1] + k);
            oracle_box_knots(b[0], b[1], b[2], b[3], t->r, t->offset, ux + u, uy + u);
            for (int q = 0; q < p; q++, u++) {
                lev[u] = m;
                for (int l = 1; l <= m; l++) reg[u * RW + l] = k / ipow(J, m - l);
            }
        }
    for (int64_t a = 0; a < nU; a++)
        for (int64_t b = 0; b < nU; b++) C[a * nU + b] = cov(ux[a], uy[a], ux[b], uy[b], c);
    memset(Sig, 0, sizeof(double) * nn * nn);

    int64_t *P = malloc(sizeof(int64_t) * (nU > 0 ? nU : 1));
    int64_t *Qi = malloc(sizeof(int64_t) * p);
    double *G = malloc(sizeof(double) * p * p);
    int status = O_OK;
    int64_t kstart = nn;
    for (int m = 1; m <= ML && !status; m++) {
        int64_t nreg_m = ipow(J, m - 1);
        for (int64_t k = 0; k < nreg_m && !status; k++) {
            for (int q = 0; q < p; q++) Qi[q] = kstart + k * p + q;
            int64_t np = 0;
            for (int64_t a = 0; a < nU; a++)
                if (lev[a] > m && reg[a * RW + m] == k) P[np++] = a;
            for (int i = 0; i < p; i++)
                for (int j = 0; j < p; j++) G[i * p + j] = C[Qi[i] * nU + Qi[j]];
            if (chol(G, p)) { status = O_ENOTPD; break; }
            if (np == 0) continue;
            /* X = C_m(Q,Q)^{-1} C_m(Q, P) */
            double *X = malloc(sizeof(double) * p * np);
            for (int i = 0; i < p; i++)
                for (int64_t b = 0; b < np; b++) X[i * np + b] = C[Qi[i] * nU + P[b]];
            chol_solve(G, p, X, (int)np);
            for (int64_t a = 0; a < np; a++)
                for (int64_t b = 0; b < np; b++) {
                    int64_t ia = P[a], ib = P[b];
                    double s = 0.0;
                    for (int i = 0; i < p; i++) s += C[ia * nU + Qi[i]] * X[i * np + b];
                    if (ia < nn && ib < nn) Sig[ia * nn + ib] += s;
                    if (reg[ia * RW + m + 1] == reg[ib * RW + m + 1])
                        C[ia * nU + ib] -= s; /* becomes C_{m+1} */
                    else
                        C[ia * nU + ib] = 0.0;
                }
            free(X);
        }
        kstart += nreg_m * p;
    }
    /* the finest level kept exact (C_M within each leaf), unless the
     * further approximation represents it by the leaves' knots */
    if (!status && !fa) {
        for (int64_t a = 0; a < nn; a++)
            for (int64_t b = 0; b < nn; b++)
                if (reg[a * RW + M] == reg[b * RW + M]) Sig[a * nn + b] += C[a * nU + b];
    }
    free(P); free(Qi); free(G);
    free(ux); free(uy); free(lev); free(reg); free(C);
    if (status) return fail(status, "dense path: knot covariance not positive definite");
    return O_OK;
}

/* Sigma_MRA over the used observations (n_used x n_used, sorted order). */
int oracle_dense_sigma(const otree *t, int family, double nu, const double *theta, double *Sig) {
    cpar c;
    int rc = make_par(family, nu, theta, &c);
    if (rc) return rc;
    return dense_sigma_ext(t, &c, 0, NULL, NULL, NULL, Sig);
}

/* Gaussian log-density of z under S + tau I (S is n x n, overwritten). */
static int gauss_loglik(double *S, const double *z, int64_t n, double tau, double *out) {
    for (int64_t a = 0; a < n; a++) S[a * n + a] += tau;
    if (chol(S, (int)n)) return fail(O_ENOTPD, "dense covariance not positive definite");
    double *v = malloc(sizeof(double) * (n > 0 ? n : 1));
    memcpy(v, z, sizeof(double) * n);
    /* forward solve only: |L^{-1} z|^2 */
    for (int64_t i = 0; i < n; i++) {
        double s = v[i];
        for (int64_t k = 0; k < i; k++) s -= S[i * n + k] * v[k];
        v[i] = s / S[i * n + i];
    }
    double q = 0.0;
    for (int64_t i = 0; i < n; i++) q += v[i] * v[i];
    *out = -0.5 * ((double)n * LOG2PI + logdet_chol(S, (int)n) + q);
    free(v);
    return O_OK;
}

/* The MRA log-likelihood by the definition: log N(z; 0, Sigma_MRA + tau I). */
int oracle_dense_loglik(const otree *t, int family, double nu, const double *theta, double *out) {
    int64_t n = t->n_used;
    double *S = malloc(sizeof(double) * (n > 0 ? n * n : 1));
    if (!S) return fail(O_ENOMEM, "oom");
    int rc = oracle_dense_sigma(t, family, nu, theta, S);
    if (!rc) rc = gauss_loglik(S, t->z, n, theta[2], out);
    free(S);
    return rc;
}

/* The exact Gaussian-process log-likelihood log N(z; 0, C(S,S) + tau I). */
int oracle_exact_loglik(const otree *t, int family, double nu, const double *theta, double *out) {
    cpar c;
    int rc = make_par(family, nu, theta, &c);
    if (rc) return rc;
    int64_t n = t->n_used;
    double *S = malloc(sizeof(double) * (n > 0 ? n * n : 1));
    if (!S) return fail(O_ENOMEM, "oom");
    for (int64_t a = 0; a < n; a++)
        for (int64_t b = 0; b < n; b++) S[a * n + b] = cov(t->x[a], t->y[a], t->x[b], t->y[b], &c);
    rc = gauss_loglik(S, t->z, n, c.tau, out);
    free(S);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Prediction (kriging) of the latent process X at np locations given the    */
/* data (prediction mode, Sec. 2.2): posterior mean and variance.            */
/* ------------------------------------------------------------------------ */

static int sort_points(const otree *t, const double *px, const double *py, int64_t np, double **sx, double **sy,
                       int64_t **perm, int64_t **off, int64_t **leafs) {
    int64_t *leaf = malloc(sizeof(int64_t) * (np > 0 ? np : 1));
    for (int64_t i = 0; i < np; i++)
        if (locate_leaf(t, px[i], py[i], &leaf[i])) {
            free(leaf);
            return fail(O_EDOMAIN, "prediction location outside the root region");
        }
    int64_t *cnt = calloc(t->nleaf + 1, sizeof(int64_t));
    for (int64_t i = 0; i < np; i++) cnt[leaf[i] + 1]++;
    for (int64_t k = 0; k < t->nleaf; k++) cnt[k + 1] += cnt[k];
    int64_t *fill = malloc(sizeof(int64_t) * (t->nleaf > 0 ? t->nleaf : 1));
    memcpy(fill, cnt, sizeof(int64_t) * t->nleaf);
    *sx = malloc(sizeof(double) * (np > 0 ? np : 1));
    *sy = malloc(sizeof(double) * (np > 0 ? np : 1));
    *perm = malloc(sizeof(int64_t) * (np > 0 ? np : 1));
    for (int64_t i = 0; i < np; i++) {
        int64_t d = fill[leaf[i]]++;
        (*sx)[d] = px[i]; (*sy)[d] = py[i]; (*perm)[d] = i;
    }
    free(fill);
    *off = cnt;
    *leafs = leaf;
    return O_OK;
}

/* The recursion: leaf kriging, then the fold updates of mu, H, v. */
int oracle_mra_predict(const otree *t, int family, double nu, const double *theta, const double *px,
                       const double *py, int64_t np, double *mean, double *var) {
    if (t->flags & O_FURTHER_APPROX) return fail(O_EINVAL, "kriging is not provided for the further approximation");
    cpar c;
    int rc = make_par(family, nu, theta, &c);
    if (rc) return rc;
    if (!(c.tau > 0.0)) return fail(O_EINVAL, "tau must be positive");
    double *sx, *sy;
    int64_t *perm, *off, *leaf;
    rc = sort_points(t, px, py, np, &sx, &sy, &perm, &off, &leaf);
    if (rc) return rc;
    int q = (t->M - 1) * t->rhat;
    pred_t pr = {np, sx, sy, off, NULL, NULL, NULL, NULL};
    size_t w = (size_t)(q > 0 ? q : 1) * (size_t)(np > 0 ? np : 1);
    pr.b = calloc(w, sizeof(double));
    pr.H = calloc(w, sizeof(double));
    pr.mu = calloc(np > 0 ? np : 1, sizeof(double));
    pr.v = calloc(np > 0 ? np : 1, sizeof(double));
    rctx *ctx = calloc(1, sizeof *ctx);
    ctx->t = t;
    ctx->p = t->rhat;
    ctx->c = c;
    ctx->pred = &pr;
    double dA[1], dw[1], du = 0.0;
    visit(ctx, 1, 0, dA, dw, &du);
    rc = ctx->status ? fail(O_ENOTPD, "not positive definite") : O_OK;
    if (!rc)
        for (int64_t d = 0; d < np; d++) {
            mean[perm[d]] = pr.mu[d];
            var[perm[d]] = pr.v[d];
        }
    free(ctx);
    free(pr.b); free(pr.H); free(pr.mu); free(pr.v);
    free(sx); free(sy); free(perm); free(off); free(leaf);
    return rc;
}

/* The definition: with the prediction points joined to the finest level,
 * mean = Sigma(p,S) (Sigma(S,S) + tau I)^{-1} z and
 * var = Sigma(p,p) - Sigma(p,S) (Sigma(S,S) + tau I)^{-1} Sigma(S,p). */
int oracle_dense_predict(const otree *t, int family, double nu, const double *theta, const double *px,
                         const double *py, int64_t np, double *mean, double *var) {
    if (t->flags & O_FURTHER_APPROX) return fail(O_EINVAL, "kriging is not provided for the further approximation");
    cpar c;
    int rc = make_par(family, nu, theta, &c);
    if (rc) return rc;
    int64_t *leaf = malloc(sizeof(int64_t) * (np > 0 ? np : 1));
    for (int64_t i = 0; i < np; i++)
        if (locate_leaf(t, px[i], py[i], &leaf[i])) {
            free(leaf);
            return fail(O_EDOMAIN, "prediction location outside the root region");
        }
    int64_t n = t->n_used, nn = n + np;
    double *S = malloc(sizeof(double) * nn * nn);
    rc = dense_sigma_ext(t, &c, np, px, py, leaf, S);
    if (!rc) {
        /* K = Sigma(S,S) + tau I, factor; solve K X = [Sigma(S,p) | z] */
        double *K = malloc(sizeof(double) * n * n);
        for (int64_t a = 0; a < n; a++)
            for (int64_t b = 0; b < n; b++) K[a * n + b] = S[a * nn + b] + (a == b ? c.tau : 0.0);
        if (chol(K, (int)n)) {
            rc = fail(O_ENOTPD, "dense covariance not positive definite");
        } else {
            int64_t wd = np + 1;
            double *X = malloc(sizeof(double) * n * wd);
            for (int64_t a = 0; a < n; a++) {
                for (int64_t j = 0; j < np; j++) X[a * wd + j] = S[a * nn + n + j];
                X[a * wd + np] = t->z[a];
            }
            chol_solve(K, (int)n, X, (int)wd);
            for (int64_t j = 0; j < np; j++) {
                double mu = 0.0, g = 0.0;
                for (int64_t a = 0; a < n; a++) {
                    mu += S[(n + j) * nn + a] * X[a * wd + np];
                    g += S[(n + j) * nn + a] * X[a * wd + j];
                }
                mean[j] = mu;
                var[j] = S[(n + j) * nn + n + j] - g;
            }
            free(X);
        }
        free(K);
    }
    free(S); free(leaf);
    return rc;
}
