// Device-side building blocks of the MRA hot path on gfx950.
//
// Notation (Sec. 1.1): levels m = 1 (root) .. M (finest); region R at level m
// has ancestors A_1 .. A_m = R, knots Q_R (r_hat grid knots above the finest
// level, the observations at the finest level).  The library works with the
// whitened prior factors
//     V^l(P) = C_l(P, Q_{A_l}) L_{A_l}^{-T},   L_R L_R^T = C_m(Q_R, Q_R),
// for which the remainder recursion reads
//     C_l(P, Q_{A_l}) = C(P, Q_{A_l}) - sum_{i<l} V^i(P) V^i(Q_{A_l})^T ,
// and with factors F = L_S^{-1} [V | z] of the finest-level covariance
//     S = C(S,S) - sum_l V^l V^l^T + tau I .
// Tiles are padded from r_hat to P in {16, 32, 64}: padded knots carry zero
// covariance with everything and an identity block in every factor.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace mra {

constexpr int NT = 256;  // threads per workgroup (4 wavefronts of 64)
constexpr int TB = 64;   // output tile edge of the workgroup GEMM
constexpr int KC = 16;   // K chunk staged through LDS
constexpr int MAXL = 16; // maximum number of levels
constexpr int MAXJ = 4;  // maximum number of children per region (J is 2 or 4)

struct KArgs {
    // tree (device)
    const double* x;
    const double* y;
    const double* z;
    const double* box;
    const int64_t* obs_lo;
    const int64_t* obs_hi;
    const int64_t* vst_off;   // per region: offset of its V store (non-leaf), doubles
    const int64_t* gram_off;  // per region: offset of its Gram matrix or -1
    const int8_t* form;       // per region: FOLD_FACTOR / FOLD_GRAM
    int64_t lvl[MAXL + 1];    // first level-order index of each level (0-based level)
    int J, M, nx, ny, rhat, P, WF, WFs;
    double offset;
    int smooth;               // 0: exp(-t), 1: (1+t) exp(-t)
    // per chunk of theta
    const double* theta;      // ntheta x 3
    int ntheta;
    double* vst;   int64_t vst_stride;
    double* F;     int64_t F_stride;
    double* gram;  int64_t gram_stride;
    double* dval;  int64_t d_stride;
    double* scratch; int64_t scratch_stride;
    int* status;              // per theta: 0, or 1 + global index of the failing region
    // Theta that share alpha and range share the prior (levels 1..M-1 and the
    // observations' whitened rows do not involve the nugget).  rep (per theta
    // of the chunk, or null for no sharing) is the first theta of the chunk
    // with the same alpha and range: the prior kernels run for such
    // representatives only.  leaf_phase, for the finest-level finishers when
    // rep is set: 0 = the other theta, reading [V | z] from their
    // representative's rows; 1 = the representatives, in place.
    const int* rep;
    int leaf_phase;
    // leaf_phase 3 (the leaf finisher only): every theta in one launch.  A
    // representative's task waits until the other theta of its group have
    // read its rows: wait[task * ntheta + rep] counts them up to need[rep]
    // (the group's size less one); need[ntheta] is the number of
    // representatives.  order lists the chunk's theta with the
    // representatives last; the finisher's queue takes a region's
    // representatives after that region's other theta.
    const int* order;
    const int* need;
    int* wait;
    // work queue of the finishers (null: grid-stride): a ticket counter and
    // a count of finished workgroups, zero at launch and set back to zero by
    // the last workgroup; tasks are taken in ticket order
    int* queue;
    // leaf_phase 2 (representatives): C(S, S) - V V^T of every leaf (lower,
    // pitch n rounded up to 4) into S0 at the representative's slot; phases
    // 0, 1 and 3 then start from it (plus the nugget) instead of forming it
    double* S0;
    const int64_t* S0_off;    // per leaf (index within the finest level)
    int64_t S0_stride;        // per theta
    const int* tasks;         // region list of this launch
    int64_t ntasks;           // regions per theta
    int level;                // level (1-based) of this launch
    double* out;              // final: loglik per theta
    double* out_ld;           // final (optional): sum of log-determinants per theta
    double* out_q;            // final (optional): quadratic form per theta
    double* out_lev;          // final (optional): per theta, M sums of log-determinants, one per level
    double n_used;
    int zero_nugget;          // 1: tau = 0 is a valid nugget
    // 1: knots at the finest level too (the further approximation): the
    // observation rows carry one more level, the leaf's own knots, in the P
    // columns before column 0 of a row (rows are WFs apart, F points P
    // columns into the first row), and the finest-level matrix is W W^T +
    // tau I with W those columns
    int fa;
    // prediction (one theta): points grouped by leaf
    const double* px;
    const double* py;
    const int64_t* pred_lo;   // per region: first prediction point of its subtree
    const int64_t* pred_hi;
    const int64_t* pred_leaf; // per point: global index of its leaf
    const int64_t* pred_perm; // per point: index in the caller's order
    double* PV;               // npred x WFs: whitened prior rows of the points
    double* PS;               // npred x WFs: H (columns of the levels) and the mean (last column)
    double* PVAR;             // npred: variance
    int64_t npred;
    double* mean_out;
    double* var_out;
};

}  // namespace mra
