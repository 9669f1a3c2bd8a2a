// Finishers: the prior factor of every region, the finest-level factors and
// the observation-space folds.
#include "mra_device.h"

namespace mra {

// Level-m regions, one wave per region: W = C(Q_R, Q_R) - sum_{i<m} V^i V^i^T
// (lower 16x16 tiles on the matrix cores, padded with an identity block), its
// Cholesky factor and inverse; the inverse is stored as the last block of the
// region's V store.
template <int P>
__global__ void __launch_bounds__(NT) k_prior_finish_w(KArgs a) {
    constexpr int NM = P / 16, NT2 = NM * (NM + 1) / 2;
    constexpr int LDT = P + 1;
    __shared__ double T[4][P * LDT];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 15, lg = lane >> 4;
    const int64_t total = a.ntasks * a.ntheta;
    const int m = a.level;
    double* Tw = T[w];
    for (int64_t t = int64_t(blockIdx.x) * 4 + w; t < total; t += int64_t(gridDim.x) * 4) {
        const int th = int(t / a.ntasks);
        const int64_t g = a.tasks[t % a.ntasks];
        const double* thp = a.theta + 3 * th;
        const double alpha = thp[0], inv_beta = 1.0 / thp[1];
        double* V = a.vst + th * a.vst_stride + a.vst_off[g];
        const int64_t ld = int64_t(m) * P;
        v4d acc[NT2];
#pragma unroll
        for (int e = 0; e < NT2; ++e) acc[e] = v4d{0.0, 0.0, 0.0, 0.0};
        const int K = (m - 1) * P;
        // two k-steps of 16 per batch, their loads issued together (K is a
        // multiple of 16)
        for (int kb = 0; kb < K; kb += 32) {
            v4d fr[2][NM];
#pragma unroll
            for (int d = 0; d < 2; ++d)
#pragma unroll
                for (int rt = 0; rt < NM; ++rt) {
                    fr[d][rt] = v4d{0.0, 0.0, 0.0, 0.0};
                    if (kb + 16 * d < K)
                        fr[d][rt] = *reinterpret_cast<const v4d*>(V + int64_t(16 * rt + lr) * ld + kb + 16 * d + 4 * lg);
                }
#pragma unroll
            for (int d = 0; d < 2; ++d)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    int e = 0;
#pragma unroll
                    for (int rt = 0; rt < NM; ++rt)
#pragma unroll
                        for (int ct = 0; ct <= rt; ++ct) acc[e] = mfma(fr[d][rt][j], fr[d][ct][j], acc[e]), ++e;
                }
        }
        // W = C - acc into LDS (lower), identity in the padding
        double kx_r[4], ky_r[4];
        {
            int e = 0;
#pragma unroll
            for (int rt = 0; rt < NM; ++rt)
#pragma unroll
                for (int ct = 0; ct <= rt; ++ct) {
                    const int c = 16 * ct + lr;
                    double cx = 0.0, cy = 0.0;
                    if (c < a.rhat) knot_xy(a, g, c, cx, cy);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int r = 16 * rt + lg + 4 * i;
                        double v;
                        if (r < a.rhat && c < a.rhat) {
                            knot_xy(a, g, r, kx_r[i], ky_r[i]);
                            v = cov_pts(kx_r[i], ky_r[i], cx, cy, alpha, inv_beta, a.smooth) - acc[e][i];
                        } else {
                            v = (r == c) ? 1.0 : 0.0;
                        }
                        if (c <= r) Tw[r * LDT + c] = v;
                    }
                    ++e;
                }
        }
        wsync();
        // factor in LDS; the inverse goes straight to its place in the V store
        if (wave_potrf_inv<P>(Tw, LDT, V + (m - 1) * P, ld, P) && lane == 0) atomicCAS(a.status + th, 0, int(g + 1));
    }
}

// Small dense finisher, one wave per region of n <= NMAX rows (NMAX 16, 32 or
// 64), on the matrix cores without workgroup barriers:
//   FIN_LEAF (finest-level region): S = C(S,S) + tau I - V V^T with V the
//     region's F rows, columns [0, (M-1)P); F <- L_S^{-1} [V | z] (all WF
//     columns, z copied into the last one first); d = log det S.
//   FIN_FOLD (observation-space fold at a.level): G = I + F_m F_m^T with F_m
//     the columns of the region's own knots; F_rest <- L_G^{-1} F_rest;
//     d = log det G.
// The n x n matrix is padded to NMAX with an identity block; its inverse
// factor replaces it in the wave's LDS tile.
enum { FIN_LEAF = 0, FIN_FOLD = 1 };

template <int NMAX, int MODE>
__global__ void __launch_bounds__(NT, (NMAX <= 32 ? 2 : 1)) k_small(KArgs a) {
    constexpr int LDT = NMAX + 1;
    constexpr int NR = NMAX / 16;
    __shared__ double T[4][NMAX * LDT];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 15, lg = lane >> 4;
    const int64_t total = a.ntasks * a.ntheta;
    const int M = a.M, P = a.P;
    double* Tw = T[w];
    double* Tiw = T[w];
    const int kc0 = MODE == FIN_LEAF ? 0 : (M - 1 - a.level) * P;  // first column of the product
    const int K = MODE == FIN_LEAF ? (M - 1) * P : P;
    const int tc0 = MODE == FIN_LEAF ? 0 : kc0 + P;                  // first column of the solve
    for (int64_t t = int64_t(blockIdx.x) * 4 + w; t < total; t += int64_t(gridDim.x) * 4) {
        const int th = int(t / a.ntasks);
        const int64_t g = a.tasks[t % a.ntasks];
        const int64_t lo = a.obs_lo[g];
        const int n = int(a.obs_hi[g] - lo);
        const double* thp = a.theta + 3 * th;
        const double alpha = thp[0], inv_beta = 1.0 / thp[1], tau = thp[2];
        double* Fr = a.F + th * a.F_stride + lo * a.WFs;
        // product over K columns: 16x16 lower tiles (rt >= ct)
        v4d acc[NR * (NR + 1) / 2];
#pragma unroll
        for (int e = 0; e < NR * (NR + 1) / 2; ++e) acc[e] = v4d{0.0, 0.0, 0.0, 0.0};
        // KD k-steps of 16 per batch: their loads are issued together (K is a
        // multiple of 16)
        constexpr int KD = NR <= 2 ? 4 : 2;
        for (int kb = 0; kb < K; kb += 16 * KD) {
            v4d fr[KD][NR];
#pragma unroll
            for (int d = 0; d < KD; ++d)
#pragma unroll
                for (int rt = 0; rt < NR; ++rt) {
                    const int row = 16 * rt + lr;
                    fr[d][rt] = v4d{0.0, 0.0, 0.0, 0.0};
                    if (row < n && kb + 16 * d < K)
                        fr[d][rt] = *reinterpret_cast<const v4d*>(Fr + int64_t(row) * a.WFs + kc0 + kb + 16 * d + 4 * lg);
                }
#pragma unroll
            for (int d = 0; d < KD; ++d)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    int e = 0;
#pragma unroll
                    for (int rt = 0; rt < NR; ++rt)
#pragma unroll
                        for (int ct = 0; ct <= rt; ++ct) acc[e] = mfma(fr[d][rt][j], fr[d][ct][j], acc[e]), ++e;
                }
        }
        // matrix into LDS (lower), identity beyond n
        {
            int e = 0;
#pragma unroll
            for (int rt = 0; rt < NR; ++rt)
#pragma unroll
                for (int ct = 0; ct <= rt; ++ct) {
                    const int c = 16 * ct + lr;
                    double cx = 0.0, cy = 0.0;
                    if (MODE == FIN_LEAF && c < n) { cx = a.x[lo + c]; cy = a.y[lo + c]; }
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int r = 16 * rt + lg + 4 * i;
                        double v;
                        if (r < n && c < n) {
                            if (MODE == FIN_LEAF) {
                                v = cov_pts(a.x[lo + r], a.y[lo + r], cx, cy, alpha, inv_beta, a.smooth) - acc[e][i];
                                if (r == c) v += tau;
                            } else {
                                v = acc[e][i] + (r == c ? 1.0 : 0.0);
                            }
                        } else {
                            v = (r == c) ? 1.0 : 0.0;
                        }
                        if (c <= r) Tw[r * LDT + c] = v;
                    }
                    ++e;
                }
        }
        wsync();
        const bool bad = wave_potrf_inv<NMAX>(Tw, LDT, Tiw, LDT, NMAX);
        if (bad && lane == 0) atomicCAS(a.status + th, 0, int(g + 1));
        // the tile now holds L^{-1}: log det = -2 sum log diag(L^{-1})
        double ldv = (lane < n) ? -log(Tw[lane * LDT + lane]) : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) ldv += __shfl_xor(ldv, off);
        if (lane == 0) a.dval[th * a.d_stride + g] = 2.0 * ldv;
        if (MODE == FIN_LEAF) {
            if (lane < n) Fr[int64_t(lane) * a.WFs + (a.WF - 1)] = a.z[lo + lane];
            wsync();
        }
        // solve: columns [tc0, WF) in 16-column tiles, CD tiles per batch (their
        // loads issued together), Li (NMAX x NMAX) on the left
        constexpr int CD = NMAX <= 32 ? 2 : 1;
        for (int c0 = tc0; c0 < a.WF; c0 += 16 * CD) {
            double bv[CD][NMAX / 4];
#pragma unroll
            for (int d = 0; d < CD; ++d)
#pragma unroll
                for (int ks = 0; ks < NMAX / 4; ++ks) {
                    const int kk = 4 * ks + lg, c = c0 + 16 * d + lr;
                    bv[d][ks] = ldg0(Fr, int64_t(kk) * a.WFs + c, kk < n && c < a.WF);
                }
#pragma unroll
            for (int d = 0; d < CD; ++d) {
                const int c = c0 + 16 * d + lr;
                v4d o[NR];
#pragma unroll
                for (int rt = 0; rt < NR; ++rt) o[rt] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int ks = 0; ks < NMAX / 4; ++ks) {
                    const int kk = 4 * ks + lg;
#pragma unroll
                    for (int rt = 0; rt < NR; ++rt) o[rt] = mfma(Tiw[(16 * rt + lr) * LDT + kk], bv[d][ks], o[rt]);
                }
                wsync();
#pragma unroll
                for (int rt = 0; rt < NR; ++rt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int r = 16 * rt + lg + 4 * i;
                        if (r < n && c < a.WF) Fr[int64_t(r) * a.WFs + c] = o[rt][i];
                    }
            }
        }
        wsync();
    }
}

// Finest-level regions: S = C(S,S) - sum_l V^l V^l^T + tau I, its Cholesky
// factor, d = log det S, and F <- L_S^{-1} [V^{M-1} .. V^1 | z] in place.
// S lives in the workgroup's global scratch slot (n^2 doubles).
__global__ void __launch_bounds__(NT) k_leaf_finish(KArgs a) {
    __shared__ Smem s;
    const int64_t total = a.ntasks * a.ntheta;
    const int M = a.M;
    double* Sg = a.scratch + blockIdx.x * a.scratch_stride;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        const int th = int(t / a.ntasks);
        const int64_t g = a.tasks[t % a.ntasks];
        const int64_t lo = a.obs_lo[g];
        const int n = int(a.obs_hi[g] - lo);
        const double* thp = a.theta + 3 * th;
        const double alpha = thp[0], inv_beta = 1.0 / thp[1], tau = thp[2];
        double* Frows = a.F + th * a.F_stride + lo * a.WFs;
        const double* px = a.x + lo;
        const double* py = a.y + lo;
        double* S = Sg;
        const int64_t lds = n;
        for (int r = threadIdx.x; r < n; r += NT) Frows[int64_t(r) * a.WFs + (a.WF - 1)] = a.z[lo + r];
        for (int64_t e0 = 0; e0 < int64_t(n) * n; e0 += 4 * NT) {
            double xi[4], yi[4], xj[4], yj[4];
#pragma unroll
            for (int j2 = 0; j2 < 4; ++j2) {
                const int64_t e = e0 + threadIdx.x + j2 * NT;
                const bool ok = e < int64_t(n) * n;
                const int i = ok ? int(e / n) : 0, j = ok ? int(e % n) : 0;
                xi[j2] = px[i]; yi[j2] = py[i]; xj[j2] = px[j]; yj[j2] = py[j];
            }
#pragma unroll
            for (int j2 = 0; j2 < 4; ++j2) {
                const int64_t e = e0 + threadIdx.x + j2 * NT;
                const int i = int(e / n), j = int(e % n);
                if (e < int64_t(n) * n && j <= i) {
                    double v = cov_pts(xi[j2], yi[j2], xj[j2], yj[j2], alpha, inv_beta, a.smooth);
                    if (i == j) v += tau;
                    S[i * lds + j] = v;
                }
            }
        }
        __syncthreads();
        if (M > 1) wg_mm<MM_SUB>(S, lds, n, n, (M - 1) * a.P, Frows, a.WFs, 1, Frows, a.WFs, 1, true, s.mm);
        double logdet = 0.0;
        double* Lst = S + int64_t(n) * n;  // inverses of the diagonal blocks
        if (wg_potrf(S, lds, n, s.L, s.Li, s.mm, &s.flag, &logdet, Lst)) {
            flag_fail(a, th, g);
            continue;
        }
        if (threadIdx.x == 0) a.dval[th * a.d_stride + g] = 2.0 * logdet;
        wg_trsm_lln(S, lds, n, Frows, a.WFs, a.WF, s.L, s.Li, s.mm, &s.flag, true, Lst);
    }
}

// Fold in observation space for regions at `level` whose subtree holds few
// observations: G = I + F_m F_m^T over the region's rows (F_m: the columns of
// this region's own knots), d = log det G, and F_rest <- L_G^{-1} F_rest.
__global__ void __launch_bounds__(NT, 2) k_fold_factor(KArgs a) {
    __shared__ Smem s;
    const int64_t total = a.ntasks * a.ntheta;
    const int m = a.level, P = a.P;
    const int cm = (a.M - 1 - m) * P;
    double* Gg = a.scratch + blockIdx.x * a.scratch_stride;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        const int th = int(t / a.ntasks);
        const int64_t g = a.tasks[t % a.ntasks];
        const int64_t lo = a.obs_lo[g];
        const int n = int(a.obs_hi[g] - lo);
        double* Frows = a.F + th * a.F_stride + lo * a.WFs;
        double* G = Gg;
        const int64_t ldg = n;
        for (int64_t e = threadIdx.x; e < int64_t(n) * n; e += NT) {
            const int i = int(e / n), j = int(e % n);
            if (j <= i) G[i * ldg + j] = (i == j) ? 1.0 : 0.0;
        }
        __syncthreads();
        wg_mm<MM_ADD>(G, ldg, n, n, P, Frows + cm, a.WFs, 1, Frows + cm, a.WFs, 1, true, s.mm);
        double logdet = 0.0;
        double* Lst = G + int64_t(n) * n;  // inverses of the diagonal blocks
        if (wg_potrf(G, ldg, n, s.L, s.Li, s.mm, &s.flag, &logdet, Lst)) {
            flag_fail(a, th, g);
            continue;
        }
        if (threadIdx.x == 0) a.dval[th * a.d_stride + g] = 2.0 * logdet;
        wg_trsm_lln(G, ldg, n, Frows + cm + P, a.WFs, a.WF - cm - P, s.L, s.Li, s.mm, &s.flag, true, Lst);
    }
}

// ---- host-side launchers

hipError_t launch_prior_finish(const KArgs& a, int grid, hipStream_t st) {
    const int g4 = (grid + 3) / 4;
    switch (a.P) {
        case 16: hipLaunchKernelGGL((k_prior_finish_w<16>), dim3(g4), dim3(NT), 0, st, a); break;
        case 32: hipLaunchKernelGGL((k_prior_finish_w<32>), dim3(g4), dim3(NT), 0, st, a); break;
        case 64: hipLaunchKernelGGL((k_prior_finish_w<64>), dim3(g4), dim3(NT), 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
// nmax: 16, 32 or 64; mode: FIN_LEAF or FIN_FOLD
hipError_t launch_small(const KArgs& a, int nmax, int mode, int grid, hipStream_t st) {
    const dim3 g((grid + 3) / 4);
    if (nmax == 16 && mode == FIN_LEAF) hipLaunchKernelGGL((k_small<16, FIN_LEAF>), g, dim3(NT), 0, st, a);
    else if (nmax == 32 && mode == FIN_LEAF) hipLaunchKernelGGL((k_small<32, FIN_LEAF>), g, dim3(NT), 0, st, a);
    else if (nmax == 64 && mode == FIN_LEAF) hipLaunchKernelGGL((k_small<64, FIN_LEAF>), g, dim3(NT), 0, st, a);
    else if (nmax == 16 && mode == FIN_FOLD) hipLaunchKernelGGL((k_small<16, FIN_FOLD>), g, dim3(NT), 0, st, a);
    else if (nmax == 32 && mode == FIN_FOLD) hipLaunchKernelGGL((k_small<32, FIN_FOLD>), g, dim3(NT), 0, st, a);
    else if (nmax == 64 && mode == FIN_FOLD) hipLaunchKernelGGL((k_small<64, FIN_FOLD>), g, dim3(NT), 0, st, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}
hipError_t launch_leaf(const KArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_leaf_finish, dim3(grid), dim3(NT), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_fold_factor(const KArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_fold_factor, dim3(grid), dim3(NT), 0, st, a);
    return hipGetLastError();
}

}  // namespace mra
