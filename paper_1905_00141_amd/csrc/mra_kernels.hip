// HIP kernels of the MRA log-likelihood for gfx950 (FP64 throughout).
//
// Per chunk of covariance-parameter vectors theta, the host launches, in
// order (all regions of a level and all theta of the chunk in one launch):
//   k_prior   levels 1 .. M-1 : whitened prior factors of every region's knots
//   k_leaf    level M         : finest-level factors F = L_S^{-1} [V | z]
//   k_fold_*  levels M-1 .. 1 : fold of the children's statistics, either in
//                               observation space (factor form) or in knot
//                               space (Gram form)
//   k_final                   : log-likelihood per theta
// The recursion is the remainder-covariance recursion of Sec. 1.1 written in
// whitened form; its posterior statistics are the conditional (co)variances
// the paper keeps per region (ATilde, Sec. 4.2 / Appendix B).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "mra_internal.h"
#include "mra_kernels.h"

namespace mra {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ double cov_t(double t, double alpha, int smooth) {
    const double e = exp(-t);
    return smooth ? alpha * (1.0 + t) * e : alpha * e;
}

__device__ __forceinline__ double cov_pts(double ax, double ay, double bx, double by, double alpha,
                                          double inv_beta, int smooth) {
    const double dx = ax - bx, dy = ay - by;
    return cov_t(sqrt(dx * dx + dy * dy) * inv_beta, alpha, smooth);
}

// Grid bar p of nb bars over [lo, hi) (Sec. 1.2, Appendix A form).
__device__ __forceinline__ double grid_bar(double lo, double hi, int nb, double f, int p) {
    const double L = hi - lo;
    if (nb == 1) return lo + f * L;
    return (lo + f * L) + ((double(p) * L) * (1.0 - 2.0 * f)) / double(nb - 1);
}

// Knots of region g into LDS arrays kx, ky (P entries; padded ones unused).
__device__ void region_knots(const KArgs& a, int64_t g, double* kx, double* ky) {
    const double* b = a.box + 4 * g;
    for (int i = threadIdx.x; i < a.P; i += NT) {
        if (i < a.rhat) {
            const int p = i % a.nx, q = i / a.nx;
            kx[i] = grid_bar(b[0], b[1], a.nx, a.offset, p);
            ky[i] = grid_bar(b[2], b[3], a.ny, a.offset, q);
        } else {
            kx[i] = 0.0;
            ky[i] = 0.0;
        }
    }
}

__device__ __forceinline__ int64_t ipow_d(int64_t b, int e) {
    int64_t v = 1;
    for (int i = 0; i < e; ++i) v *= b;
    return v;
}

// Global index of the level-l ancestor of region k (index within level m).
__device__ __forceinline__ int64_t ancestor(const KArgs& a, int m, int64_t k, int l) {
    return a.lvl[l - 1] + k / ipow_d(a.J, m - l);
}

__device__ void flag_fail(const KArgs& a, int th, int64_t g) {
    if (threadIdx.x == 0) atomicCAS(a.status + th, 0, int(g + 1));
}

// ---------------------------------------------------- workgroup primitives

// C(r,c) +=/-= sum_k A(r,k) B(c,k) for r < R, c < N (c <= r when lower),
// A(r,k) = A[r*sar + k*sak], B(c,k) = B[c*sbc + k*sbk], C row-major (ldc).
// 64x64 output tiles, 4x4 per thread, K staged through LDS in chunks of 16.
template <bool SUB>
__device__ void wg_gemm(double* C, int64_t ldc, int R, int N, int K, const double* A, int64_t sar,
                        int64_t sak, const double* B, int64_t sbc, int64_t sbk, bool lower,
                        double* sm) {
    double* As = sm;
    double* Bs = sm + KC * TB;
    const int tid = threadIdx.x, tr = tid / 16, tc = tid % 16;
    for (int r0 = 0; r0 < R; r0 += TB)
        for (int c0 = 0; c0 < N; c0 += TB) {
            if (lower && c0 > r0 + TB - 1) continue;
            double acc[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
            for (int k0 = 0; k0 < K; k0 += KC) {
                for (int e = tid; e < TB * KC; e += NT) {
                    int r, k;
                    if (sak == 1) { r = e / KC; k = e % KC; } else { k = e / TB; r = e % TB; }
                    double v = 0.0;
                    if (r0 + r < R && k0 + k < K) v = A[int64_t(r0 + r) * sar + int64_t(k0 + k) * sak];
                    As[k * TB + r] = v;
                    int c, kb;
                    if (sbk == 1) { c = e / KC; kb = e % KC; } else { kb = e / TB; c = e % TB; }
                    double w = 0.0;
                    if (c0 + c < N && k0 + kb < K) w = B[int64_t(c0 + c) * sbc + int64_t(k0 + kb) * sbk];
                    Bs[kb * TB + c] = w;
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < KC; ++k) {
                    double av[4], bv[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) { av[i] = As[k * TB + tr * 4 + i]; bv[i] = Bs[k * TB + tc * 4 + i]; }
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
                }
                __syncthreads();
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r = r0 + tr * 4 + i, c = c0 + tc * 4 + j;
                    if (r < R && c < N && (!lower || c <= r)) {
                        double* p = C + int64_t(r) * ldc + c;
                        *p = SUB ? (*p - acc[i][j]) : (*p + acc[i][j]);
                    }
                }
        }
    __syncthreads();
}

// In-place Cholesky of an n x n (n <= 64) lower triangle held in LDS (ld).
// Returns true when a pivot is not positive (the factor is then garbage).
__device__ bool wg_potrf_lds(double* T, int n, int ld, int* flag) {
    const int tid = threadIdx.x;
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        if (tid == 0) {
            double d = T[j * ld + j];
            if (!(d > 0.0)) { *flag = 1; d = 1.0; }
            T[j * ld + j] = sqrt(d);
        }
        __syncthreads();
        const double djj = T[j * ld + j];
        for (int i = j + 1 + tid; i < n; i += NT) T[i * ld + j] /= djj;
        __syncthreads();
        const int m = n - j - 1;
        for (int e = tid; e < m * m; e += NT) {
            const int i = j + 1 + e / m, k = j + 1 + e % m;
            if (k <= i) T[i * ld + k] -= T[i * ld + j] * T[k * ld + j];
        }
        __syncthreads();
    }
    const bool bad = *flag != 0;
    __syncthreads();
    return bad;
}

// Forward substitution L v = w for one vector of length n <= 64 whose entries
// sit at v[i*stride]; L in LDS (lower, ld).  Registers hold the vector.
__device__ __forceinline__ void tri_solve_vec(const double* L, int ld, int n, double* v, int64_t stride) {
    double x[64];
#pragma unroll
    for (int r = 0; r < 64; ++r) {
        if (r < n) {
            double s = v[int64_t(r) * stride];
#pragma unroll
            for (int k = 0; k < r; ++k) s = fma(-L[r * ld + k], x[k], s);
            x[r] = s / L[r * ld + r];
            v[int64_t(r) * stride] = x[r];
        }
    }
}

// X (R x n, row-major ldx) <- X L^{-T}, L (n x n, n <= 64) in LDS.
__device__ void wg_trsm_rlt(double* X, int64_t ldx, int R, const double* L, int ld, int n) {
    for (int a = threadIdx.x; a < R; a += NT) tri_solve_vec(L, ld, n, X + int64_t(a) * ldx, 1);
    __syncthreads();
}

// Load an n x n lower triangle (global, ldg) into LDS (ld), zero above.
__device__ void load_tile(double* T, int ld, const double* G, int64_t ldg, int n) {
    for (int e = threadIdx.x; e < n * n; e += NT) {
        const int i = e / n, j = e % n;
        T[i * ld + j] = (j <= i) ? G[int64_t(i) * ldg + j] : 0.0;
    }
    __syncthreads();
}

__device__ void store_tile(double* G, int64_t ldg, const double* T, int ld, int n) {
    for (int e = threadIdx.x; e < n * n; e += NT) {
        const int i = e / n, j = e % n;
        G[int64_t(i) * ldg + j] = (j <= i) ? T[i * ld + j] : 0.0;
    }
    __syncthreads();
}

// Blocked right-looking Cholesky of an n x n lower triangle in global memory.
// Accumulates sum(log diag) into *logdet (thread 0's copy).  Returns failure.
__device__ bool wg_potrf_global(double* A, int64_t lda, int n, double* Ls, double* sm, int* flag,
                                double* logdet) {
    double ld_acc = 0.0;
    for (int j0 = 0; j0 < n; j0 += TB) {
        const int jb = min(TB, n - j0);
        double* Ajj = A + int64_t(j0) * lda + j0;
        load_tile(Ls, TB + 1, Ajj, lda, jb);
        if (wg_potrf_lds(Ls, jb, TB + 1, flag)) return true;
        store_tile(Ajj, lda, Ls, TB + 1, jb);
        if (threadIdx.x == 0)
            for (int i = 0; i < jb; ++i) ld_acc += log(Ls[i * (TB + 1) + i]);
        const int rest = n - j0 - jb;
        if (rest > 0) {
            double* Aij = A + int64_t(j0 + jb) * lda + j0;
            wg_trsm_rlt(Aij, lda, rest, Ls, TB + 1, jb);
            wg_gemm<true>(A + int64_t(j0 + jb) * lda + j0 + jb, lda, rest, rest, jb, Aij, lda, 1, Aij,
                          lda, 1, true, sm);
        }
    }
    if (threadIdx.x == 0) *logdet = ld_acc;
    return false;
}

// X (n x W, ldx) <- L^{-1} X with L (n x n lower, global, ldl).
__device__ void wg_trsm_lln(const double* L, int64_t ldl, int n, double* X, int64_t ldx, int W,
                            double* Ls, double* sm) {
    for (int i0 = 0; i0 < n; i0 += TB) {
        const int ib = min(TB, n - i0);
        load_tile(Ls, TB + 1, L + int64_t(i0) * ldl + i0, ldl, ib);
        for (int c = threadIdx.x; c < W; c += NT) tri_solve_vec(Ls, TB + 1, ib, X + int64_t(i0) * ldx + c, ldx);
        __syncthreads();
        const int rest = n - i0 - ib;
        if (rest > 0)
            wg_gemm<true>(X + int64_t(i0 + ib) * ldx, ldx, rest, W, ib, L + int64_t(i0 + ib) * ldl + i0, ldl,
                          1, X + int64_t(i0) * ldx, 1, ldx, false, sm);
    }
}

// Whitened prior factors of R point rows (coordinates px/py; rows >= nreal
// are padding) for ancestor levels 1..L (global indices anc[1..L], knots in
// akx/aky, P per ancestor).  Block l of row a is written at
//     dst0 + (l-1)*bstride + a*ldd  (P consecutive doubles).
__device__ void chain(const KArgs& a, const double* th, int R, int nreal, const double* px,
                      const double* py, int L, const int64_t* anc, const double* akx, const double* aky,
                      const double* vst, double* dst0, int64_t bstride, int64_t ldd, double* Ls,
                      double* sm) {
    const int P = a.P;
    const double alpha = th[0], inv_beta = 1.0 / th[1];
    for (int l = 1; l <= L; ++l) {
        double* dl = dst0 + int64_t(l - 1) * bstride;
        const double* kx = akx + (l - 1) * P;
        const double* ky = aky + (l - 1) * P;
        for (int e = threadIdx.x; e < R * P; e += NT) {
            const int r = e / P, b = e % P;
            double v = 0.0;
            if (r < nreal && b < a.rhat) v = cov_pts(px[r], py[r], kx[b], ky[b], alpha, inv_beta, a.smooth);
            dl[int64_t(r) * ldd + b] = v;
        }
        __syncthreads();
        const double* Vanc = vst + a.vst_off[anc[l]];
        for (int i = 1; i < l; ++i)
            wg_gemm<true>(dl, ldd, R, P, P, dst0 + int64_t(i - 1) * bstride, ldd, 1,
                          Vanc + int64_t(i - 1) * P * P, P, 1, false, sm);
        load_tile(Ls, TB + 1, Vanc + int64_t(l - 1) * P * P, P, P);
        wg_trsm_rlt(dl, ldd, R, Ls, TB + 1, P);
    }
}

// ------------------------------------------------------------------ kernels

struct Smem {
    double gemm[2 * KC * TB];
    double L[TB * (TB + 1)];
    double akx[MAXL * TB], aky[MAXL * TB];
    double kx[TB], ky[TB];
    double red[NT];
    int flag;
};

// Prior of every region at `level` (< M) for every theta of the chunk.
__global__ void __launch_bounds__(NT) k_prior(KArgs a) {
    __shared__ Smem s;
    const int64_t total = a.ntasks * a.ntheta;
    const int m = a.level, P = a.P;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        const int th = int(t / a.ntasks);
        const int64_t g = a.tasks[t % a.ntasks];
        const int64_t k = g - a.lvl[m - 1];  // index within level
        const double* thp = a.theta + 3 * th;
        const double* vst = a.vst + th * a.vst_stride;
        int64_t anc[MAXL + 1];
        for (int l = 1; l <= m; ++l) anc[l] = ancestor(a, m, k, l);
        for (int l = 1; l < m; ++l) region_knots(a, anc[l], s.akx + (l - 1) * P, s.aky + (l - 1) * P);
        region_knots(a, g, s.kx, s.ky);
        __syncthreads();
        double* mine = a.vst + th * a.vst_stride + a.vst_off[g];
        chain(a, thp, P, a.rhat, s.kx, s.ky, m - 1, anc, s.akx, s.aky, vst, mine, int64_t(P) * P, P, s.L, s.gemm);
        // C_m(Q_R, Q_R) = C(Q_R, Q_R) - sum_{i<m} V^i V^i^T, padded with an identity block
        double* W = mine + int64_t(m - 1) * P * P;
        const double alpha = thp[0], inv_beta = 1.0 / thp[1];
        for (int e = threadIdx.x; e < P * P; e += NT) {
            const int i = e / P, j = e % P;
            double v;
            if (i < a.rhat && j < a.rhat) v = cov_pts(s.kx[i], s.ky[i], s.kx[j], s.ky[j], alpha, inv_beta, a.smooth);
            else v = (i == j) ? 1.0 : 0.0;
            W[e] = v;
        }
        __syncthreads();
        for (int i = 1; i < m; ++i)
            wg_gemm<true>(W, P, P, P, P, mine + int64_t(i - 1) * P * P, P, 1, mine + int64_t(i - 1) * P * P, P, 1,
                          true, s.gemm);
        load_tile(s.L, TB + 1, W, P, P);
        if (wg_potrf_lds(s.L, P, TB + 1, &s.flag)) flag_fail(a, th, g);
        store_tile(W, P, s.L, TB + 1, P);
    }
}

// Finest-level regions: factors F = L_S^{-1} [V^{M-1} .. V^1 | z] in place in
// the F buffer rows of the leaf, and d = log det S.
__global__ void __launch_bounds__(NT) k_leaf(KArgs a) {
    __shared__ Smem s;
    const int64_t total = a.ntasks * a.ntheta;
    const int M = a.M, P = a.P;
    double* S = a.scratch + blockIdx.x * a.scratch_stride;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        const int th = int(t / a.ntasks);
        const int64_t g = a.tasks[t % a.ntasks];
        const int64_t k = g - a.lvl[M - 1];
        const int64_t lo = a.obs_lo[g];
        const int n = int(a.obs_hi[g] - lo);
        const double* thp = a.theta + 3 * th;
        const double* vst = a.vst + th * a.vst_stride;
        double* Frows = a.F + th * a.F_stride + lo * a.WFs;
        int64_t anc[MAXL + 1];
        for (int l = 1; l < M; ++l) anc[l] = ancestor(a, M, k, l);
        for (int l = 1; l < M; ++l) region_knots(a, anc[l], s.akx + (l - 1) * P, s.aky + (l - 1) * P);
        for (int r = threadIdx.x; r < n; r += NT) Frows[int64_t(r) * a.WFs + (a.WF - 1)] = a.z[lo + r];
        __syncthreads();
        if (M > 1)
            chain(a, thp, n, n, a.x + lo, a.y + lo, M - 1, anc, s.akx, s.aky, vst, Frows + int64_t(M - 2) * P,
                  -int64_t(P), a.WFs, s.L, s.gemm);
        // S = C(S,S) - sum_l V^l V^l^T + tau I  (lower)
        const double alpha = thp[0], inv_beta = 1.0 / thp[1], tau = thp[2];
        const double* px = a.x + lo;
        const double* py = a.y + lo;
        for (int64_t e = threadIdx.x; e < int64_t(n) * n; e += NT) {
            const int i = int(e / n), j = int(e % n);
            if (j <= i) {
                double v = cov_pts(px[i], py[i], px[j], py[j], alpha, inv_beta, a.smooth);
                if (i == j) v += tau;
                S[e] = v;
            }
        }
        __syncthreads();
        for (int l = 1; l < M; ++l) {
            const double* Vl = Frows + int64_t(M - 1 - l) * P;
            wg_gemm<true>(S, n, n, n, P, Vl, a.WFs, 1, Vl, a.WFs, 1, true, s.gemm);
        }
        double logdet = 0.0;
        if (wg_potrf_global(S, n, n, s.L, s.gemm, &s.flag, &logdet)) {
            flag_fail(a, th, g);
            continue;
        }
        if (threadIdx.x == 0) a.dval[th * a.d_stride + g] = 2.0 * logdet;
        wg_trsm_lln(S, n, n, Frows, a.WFs, a.WF, s.L, s.gemm);
    }
}

// Fold in observation space for regions at `level` whose subtree holds few
// observations: G = I + F_m F_m^T over the region's rows (F_m: the columns of
// this region's own knots), d = log det G, and F_rest <- L_G^{-1} F_rest.
__global__ void __launch_bounds__(NT) k_fold_factor(KArgs a) {
    __shared__ Smem s;
    const int64_t total = a.ntasks * a.ntheta;
    const int m = a.level, P = a.P;
    const int cm = (a.M - 1 - m) * P;
    double* G = a.scratch + blockIdx.x * a.scratch_stride;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        const int th = int(t / a.ntasks);
        const int64_t g = a.tasks[t % a.ntasks];
        const int64_t lo = a.obs_lo[g];
        const int n = int(a.obs_hi[g] - lo);
        double* Frows = a.F + th * a.F_stride + lo * a.WFs;
        for (int64_t e = threadIdx.x; e < int64_t(n) * n; e += NT) {
            const int i = int(e / n), j = int(e % n);
            if (j <= i) G[e] = (i == j) ? 1.0 : 0.0;
        }
        __syncthreads();
        wg_gemm<false>(G, n, n, n, P, Frows + cm, a.WFs, 1, Frows + cm, a.WFs, 1, true, s.gemm);
        double logdet = 0.0;
        if (wg_potrf_global(G, n, n, s.L, s.gemm, &s.flag, &logdet)) {
            flag_fail(a, th, g);
            continue;
        }
        if (threadIdx.x == 0) a.dval[th * a.d_stride + g] = 2.0 * logdet;
        wg_trsm_lln(G, n, n, Frows + cm + P, a.WFs, a.WF - cm - P, s.L, s.gemm);
    }
}

// Fold in knot space: Gram matrix of the live columns over the children
// (factor-form children contribute F^T F over their rows, Gram-form children
// the trailing part of their own Gram matrix), then one block step of
// Cholesky on I + G_mm and the Schur update of the trailing part.
__global__ void __launch_bounds__(NT) k_fold_gram(KArgs a) {
    __shared__ Smem s;
    const int64_t total = a.ntasks * a.ntheta;
    const int m = a.level, P = a.P, M = a.M;
    const int cm = (M - 1 - m) * P;
    const int D = m * P + 1;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        const int th = int(t / a.ntasks);
        const int64_t g = a.tasks[t % a.ntasks];
        const int64_t k = g - a.lvl[m - 1];
        double* G = a.gram + th * a.gram_stride + a.gram_off[g];
        const double* Fth = a.F + th * a.F_stride;
        for (int64_t e = threadIdx.x; e < int64_t(D) * D; e += NT) G[e] = 0.0;
        __syncthreads();
        for (int j = 0; j < a.J; ++j) {
            const int64_t gc = a.lvl[m] + a.J * k + j;
            if (m + 1 == M || a.form[gc] == FOLD_FACTOR) {
                const int64_t lo = a.obs_lo[gc];
                const int nc = int(a.obs_hi[gc] - lo);
                if (nc == 0) continue;
                const double* Fc = Fth + lo * a.WFs + cm;
                wg_gemm<false>(G, D, D, D, nc, Fc, 1, a.WFs, Fc, 1, a.WFs, true, s.gemm);
            } else {
                const double* Gc = a.gram + th * a.gram_stride + a.gram_off[gc];
                const int Dc = D + P;
                for (int64_t e = threadIdx.x; e < int64_t(D) * D; e += NT) {
                    const int i = int(e / D), jj = int(e % D);
                    if (jj <= i) G[e] += Gc[int64_t(P + i) * Dc + P + jj];
                }
                __syncthreads();
            }
        }
        // I + G_mm -> Cholesky in LDS
        for (int e = threadIdx.x; e < P * P; e += NT) {
            const int i = e / P, j = e % P;
            s.L[i * (TB + 1) + j] = (j <= i) ? G[int64_t(i) * D + j] + (i == j ? 1.0 : 0.0) : 0.0;
        }
        __syncthreads();
        if (wg_potrf_lds(s.L, P, TB + 1, &s.flag)) {
            flag_fail(a, th, g);
            continue;
        }
        if (threadIdx.x == 0) {
            double ld = 0.0;
            for (int i = 0; i < P; ++i) ld += log(s.L[i * (TB + 1) + i]);
            a.dval[th * a.d_stride + g] = 2.0 * ld;
        }
        // Z = G[P:D, 0:P] <- Z L^{-T};  G[P:D, P:D] -= Z Z^T
        double* Z = G + int64_t(P) * D;
        wg_trsm_rlt(Z, D, D - P, s.L, TB + 1, P);
        wg_gemm<true>(Z + P, D, D - P, D - P, P, Z, D, 1, Z, D, 1, true, s.gemm);
    }
}

// log-likelihood per theta: -1/2 [ n log 2 pi + sum of log-determinants + q ],
// q the quadratic form left in the root's statistics.  Fixed-order sums.
__global__ void __launch_bounds__(NT) k_final(KArgs a, int64_t nreg, int root_gram) {
    __shared__ double red[NT];
    const int th = blockIdx.x;
    const double* d = a.dval + th * a.d_stride;
    double sd = 0.0;
    for (int64_t g = threadIdx.x; g < nreg; g += NT) sd += d[g];
    red[threadIdx.x] = sd;
    __syncthreads();
    for (int w = NT / 2; w > 0; w /= 2) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double dsum = red[0];
    __syncthreads();
    double q = 0.0;
    if (root_gram) {
        const int D = a.P + 1;
        q = a.gram[th * a.gram_stride + a.gram_off[0] + int64_t(a.P) * D + a.P];
    } else {
        const double* F = a.F + th * a.F_stride;
        const int64_t n = int64_t(a.n_used);
        double sq = 0.0;
        for (int64_t r = threadIdx.x; r < n; r += NT) {
            const double y = F[r * a.WFs + (a.WF - 1)];
            sq = fma(y, y, sq);
        }
        red[threadIdx.x] = sq;
        __syncthreads();
        for (int w = NT / 2; w > 0; w /= 2) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        q = red[0];
    }
    if (threadIdx.x == 0) {
        const double LOG2PI = 1.8378770664093454835606594728112;
        double ll = -0.5 * (a.n_used * LOG2PI + dsum + q);
        if (a.status[th] != 0) ll = __builtin_nan("");
        a.out[th] = ll;
    }
}

__global__ void k_fill(double* p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_int(int* p, int64_t n, int v) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

// ------------------------------------------------------- host-side launchers

hipError_t launch_prior(const KArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_prior, dim3(grid), dim3(NT), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_leaf(const KArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_leaf, dim3(grid), dim3(NT), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_fold_factor(const KArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_fold_factor, dim3(grid), dim3(NT), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_fold_gram(const KArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_fold_gram, dim3(grid), dim3(NT), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_final(const KArgs& a, int64_t nreg, int root_gram, hipStream_t st) {
    hipLaunchKernelGGL(k_final, dim3(a.ntheta), dim3(NT), 0, st, a, nreg, root_gram);
    return hipGetLastError();
}
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill, dim3(unsigned(blocks < 4096 ? blocks : 4096)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_int(int* p, int64_t n, int v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_int, dim3(unsigned(blocks < 4096 ? blocks : 4096)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace mra
