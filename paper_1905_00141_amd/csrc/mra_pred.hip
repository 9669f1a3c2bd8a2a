// Kriging kernels.
#include "mra_device.h"

namespace mra {

// ---------------------------------------------------------- prediction
// Kriging of the latent process at prediction points (one theta).  A point p
// joins the finest-level set of its leaf R; with V(p) its whitened prior rows,
// g = L_S^{-1} C_M(S, p) and the leaf factors F = L_S^{-1} V(S), y = L_S^{-1} z:
//   mean_0 = g^T y,  H = g^T F (whitened),  v_0 = C(p,p) - |V(p)|^2 - |g|^2.
// Every fold above (knot space, L^{-1} and Y of the region kept) then adds,
// with e = L^{-1} (V^m(p) - H^m):  v += |e|^2,  [H_rest | mean] += Y^T e.

// Leaves holding prediction points (run before the leaf finishers overwrite
// the observations' rows).  Scratch per slot: n^2 + n (WFs + k).
__global__ void __launch_bounds__(NT) k_pred_leaf(KArgs a) {
    __shared__ Smem s;
    const int M = a.M, P = a.P, K = (M - 1) * P;
    const double alpha = a.theta[0], inv_beta = 1.0 / a.theta[1], tau = a.theta[2];
    for (int64_t t = blockIdx.x; t < a.ntasks; t += gridDim.x) {
        const int64_t g = a.tasks[t];
        const int64_t lo = a.obs_lo[g], plo = a.pred_lo[g];
        const int n = int(a.obs_hi[g] - lo), k = int(a.pred_hi[g] - plo);
        const double* Fr = a.F + lo * a.WFs;
        double* PVr = a.PV + plo * a.WFs;
        double* PSr = a.PS + plo * a.WFs;
        if (n > 0) {
            double* S = a.scratch + blockIdx.x * a.scratch_stride;
            const int64_t ldx = a.WFs + k;
            double* X = S + int64_t(n) * n;
            for (int64_t e = threadIdx.x; e < int64_t(n) * n; e += NT) {
                const int i = int(e / n), j = int(e % n);
                if (j <= i) {
                    double v = cov_pts(a.x[lo + i], a.y[lo + i], a.x[lo + j], a.y[lo + j], alpha, inv_beta, a.smooth);
                    S[e] = (i == j) ? v + tau : v;
                }
            }
            // X = [V(S) | z | pad | C(S, p_j)]
            for (int64_t e = threadIdx.x; e < int64_t(n) * ldx; e += NT) {
                const int i = int(e / ldx), c = int(e % ldx);
                double v;
                if (c < a.WF - 1) v = Fr[int64_t(i) * a.WFs + c];
                else if (c == a.WF - 1) v = a.z[lo + i];
                else if (c < a.WFs) v = 0.0;
                else {
                    const int j = c - a.WFs;
                    v = cov_pts(a.x[lo + i], a.y[lo + i], a.px[plo + j], a.py[plo + j], alpha, inv_beta, a.smooth);
                }
                X[e] = v;
            }
            __syncthreads();
            if (K > 0) {
                wg_mm<MM_SUB>(S, n, n, n, K, Fr, a.WFs, 1, Fr, a.WFs, 1, true, s.mm);
                wg_mm<MM_SUB>(X + a.WFs, ldx, n, k, K, Fr, a.WFs, 1, PVr, a.WFs, 1, false, s.mm);
            }
            double logdet = 0.0;
            if (wg_potrf(S, n, n, s.L, s.Li, s.mm, &s.flag, &logdet)) {
                flag_fail(a, 0, g);
                continue;
            }
            wg_trsm_lln(S, n, n, X, ldx, int(ldx), s.L, s.Li, s.mm, &s.flag, true);
            // [H | mean] of point j = g_j^T [F | y]
            wg_mm<MM_SET>(PSr, a.WFs, k, a.WF, n, X + a.WFs, 1, ldx, X, 1, ldx, false, s.mm);
            for (int j = threadIdx.x; j < k; j += NT) {
                double v = alpha;
                for (int c = 0; c < K; ++c) v = fma(-PVr[int64_t(j) * a.WFs + c], PVr[int64_t(j) * a.WFs + c], v);
                for (int i = 0; i < n; ++i) v = fma(-X[int64_t(i) * ldx + a.WFs + j], X[int64_t(i) * ldx + a.WFs + j], v);
                a.PVAR[plo + j] = v;
            }
            __syncthreads();
        } else {
            for (int64_t e = threadIdx.x; e < int64_t(k) * a.WF; e += NT) PSr[(e / a.WF) * a.WFs + (e % a.WF)] = 0.0;
            for (int j = threadIdx.x; j < k; j += NT) {
                double v = alpha;
                for (int c = 0; c < K; ++c) v = fma(-PVr[int64_t(j) * a.WFs + c], PVr[int64_t(j) * a.WFs + c], v);
                a.PVAR[plo + j] = v;
            }
            __syncthreads();
        }
    }
}

// Fold of the prediction state at level a.level, one wave per point.
__global__ void __launch_bounds__(NT) k_pred_fold(KArgs a) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = a.level, P = a.P, M = a.M;
    const int D = m * P + 1, cm = (M - 1 - m) * P;
    for (int64_t j = int64_t(blockIdx.x) * 4 + w; j < a.npred; j += int64_t(gridDim.x) * 4) {
        const int64_t kl = a.pred_leaf[j] - a.lvl[M - 1];
        const int64_t R = a.lvl[m - 1] + kl / ipow_d(a.J, M - m);
        const int64_t goff = a.gram_off[R];
        double* PSr = a.PS + j * a.WFs;
        const double* PVr = a.PV + j * a.WFs;
        const double E = (lane < P) ? PVr[cm + lane] - PSr[cm + lane] : 0.0;
        double e = E;
        const double* G = a.gram + (goff >= 0 ? goff : 0);
        if (goff >= 0) {
            e = 0.0;
            for (int b = 0; b < P; ++b) {
                const double Eb = __shfl(E, b);
                if (lane < P && b <= lane) e = fma(G[int64_t(lane) * D + b], Eb, e);
            }
        }
        double e2 = e * e;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) e2 += __shfl_xor(e2, off);
        if (lane == 0) a.PVAR[j] += e2;
        if (goff >= 0) {
            for (int r0 = 0; r0 < D - P; r0 += 64) {
                const int r = r0 + lane;
                double acc = 0.0;
                for (int b = 0; b < P; ++b) {
                    const double eb = __shfl(e, b);
                    if (r < D - P) acc = fma(G[int64_t(P + r) * D + b], eb, acc);
                }
                if (r < D - P) PSr[cm + P + r] += acc;
            }
        }
    }
}

// Posterior mean and variance back to the caller's order.
__global__ void k_pred_out(KArgs a) {
    for (int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; j < a.npred; j += int64_t(gridDim.x) * blockDim.x) {
        a.mean_out[a.pred_perm[j]] = a.PS[j * a.WFs + (a.WF - 1)];
        a.var_out[a.pred_perm[j]] = a.PVAR[j];
    }
}

// ---- host-side launchers

hipError_t launch_pred_leaf(const KArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_pred_leaf, dim3(grid), dim3(NT), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_pred_fold(const KArgs& a, hipStream_t st) {
    const int64_t g = (a.npred + 3) / 4;
    hipLaunchKernelGGL(k_pred_fold, dim3(unsigned(g < 65536 ? g : 65536)), dim3(NT), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_pred_out(const KArgs& a, hipStream_t st) {
    const int64_t g = (a.npred + 255) / 256;
    hipLaunchKernelGGL(k_pred_out, dim3(unsigned(g < 4096 ? (g > 0 ? g : 1) : 4096)), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace mra
