// Finishers: the prior factor of every region, the finest-level factors and
// the observation-space folds.
#include "mra_device.h"

namespace mra {

// Level-m regions, one wave per region: W = C(Q_R, Q_R) - sum_{i<m} V^i V^i^T
// (lower 16x16 tiles on the matrix cores, padded with an identity block), its
// Cholesky factor and inverse (the one-wave blocked factorization); the
// inverse is stored as the last block of the region's V store.
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
        if (a.rep && a.rep[th] != th) continue;  // shares its representative's prior
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
        // factor and inverse in LDS, then the inverse to its place in the V store
        double ldv;
        if (wave_chol_inv<NM>(Tw, LDT, P, &ldv) && lane == 0) atomicCAS(a.status + th, 0, int(g + 1));
        double* Li = V + (m - 1) * P;
        for (int e = lane; e < P * P; e += 64) Li[int64_t(e / P) * ld + (e % P)] = Tw[(e / P) * LDT + (e % P)];
        wsync();  // the wave's next task rewrites its tile
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
__global__ void __launch_bounds__(NT, (NMAX <= 32 ? 3 : 1)) k_small(KArgs a) {
    constexpr int LDT = NMAX + 1;
    constexpr int NR = NMAX / 16;
    __shared__ double T[4][NMAX * LDT];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 15, lg = lane >> 4;
    const int64_t total = a.ntasks * a.ntheta;
    const int M = a.M, P = a.P;
    double* Tw = T[w];
    double* Tiw = T[w];
    // first column of the product and its width (the further approximation:
    // the leaf's own-knot columns W before column 0, the matrix W W^T + tau I)
    const int kc0 = MODE == FIN_LEAF ? (a.fa ? -P : 0) : (M - 1 - a.level) * P;
    const int K = MODE == FIN_LEAF ? (a.fa ? P : (M - 1) * P) : P;
    const int tc0 = MODE == FIN_LEAF ? 0 : kc0 + P;                  // first column of the solve
    for (int64_t t = int64_t(blockIdx.x) * 4 + w; t < total; t += int64_t(gridDim.x) * 4) {
        const int th = int(t / a.ntasks);
        if (MODE == FIN_LEAF && a.rep && (a.leaf_phase == 0) == (a.rep[th] == th)) continue;
        const int64_t g = a.tasks[t % a.ntasks];
        const int64_t lo = a.obs_lo[g];
        const int n = int(a.obs_hi[g] - lo);
        const double* thp = a.theta + 3 * th;
        const double alpha = thp[0], inv_beta = 1.0 / thp[1], tau = thp[2];
        double* Fr = a.F + th * a.F_stride + lo * a.WFs;
        // rows read: [V | z] of the representative for a theta that shares it
        const double* Fs = (MODE == FIN_LEAF && a.rep && a.leaf_phase == 0) ? a.F + a.rep[th] * a.F_stride + lo * a.WFs : Fr;
        // a shared prior: C - V V^T (pitch n rounded up to 4), formed once per
        // representative (phase 2) and taken from there by its group
        const bool s0_build = MODE == FIN_LEAF && a.S0 && a.leaf_phase == 2;
        const bool s0_use = MODE == FIN_LEAF && a.S0 && a.leaf_phase != 2;
        double* S0p = (MODE == FIN_LEAF && a.S0) ? a.S0 + a.rep[th] * a.S0_stride + a.S0_off[g - a.lvl[M - 1]] : nullptr;
        const int lds = (n + 3) & ~3;
        if (s0_use) {
            for (int e = lane; e < NMAX * NMAX; e += 64) {
                const int r = e / NMAX, c = e % NMAX;
                if (c <= r)
                    Tw[r * LDT + c] = (r < n && c < n) ? S0p[r * lds + c] + (r == c ? tau : 0.0) : (r == c ? 1.0 : 0.0);
            }
        } else {
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
                        fr[d][rt] = *reinterpret_cast<const v4d*>(Fs + int64_t(row) * a.WFs + kc0 + kb + 16 * d + 4 * lg);
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
                    if (MODE == FIN_LEAF && !a.fa && c < n) { cx = a.x[lo + c]; cy = a.y[lo + c]; }
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int r = 16 * rt + lg + 4 * i;
                        double v;
                        if (r < n && c < n) {
                            if (MODE == FIN_LEAF) {
                                v = a.fa ? acc[e][i]
                                         : cov_pts(a.x[lo + r], a.y[lo + r], cx, cy, alpha, inv_beta, a.smooth) - acc[e][i];
                                if (r == c && !s0_build) v += tau;
                            } else {
                                v = acc[e][i] + (r == c ? 1.0 : 0.0);
                            }
                        } else {
                            v = (r == c) ? 1.0 : 0.0;
                        }
                        if (s0_build) {
                            if (c <= r && r < n) S0p[r * lds + c] = v;
                        } else if (c <= r) {
                            Tw[r * LDT + c] = v;
                        }
                    }
                    ++e;
                }
        }
        }
        if (s0_build) continue;  // phase 2 forms the matrix only
        wsync();
        // the tile is replaced by L^{-1}
        double ldv = 0.0;
        const bool bad = wave_chol_inv<NR>(Tw, LDT, n, &ldv);
        if (bad && lane == 0) atomicCAS(a.status + th, 0, int(g + 1));
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
                    bv[d][ks] = ldg0(Fs, int64_t(kk) * a.WFs + c, kk < n && c < a.WF);
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

// Workgroup finisher for regions of more than 64 rows (one workgroup per
// region and theta, grid-stride over tasks):
//   FIN_LEAF (finest level): A = C(S,S) + tau I - V V^T, V the rows' F
//     columns [0, (M-1)P); right-hand sides X = all WF columns (z copied into
//     the last one first).
//   FIN_FOLD (observation-space fold at a.level): A = I + F_m F_m^T, F_m the
//     columns of the region's own knots; X = the columns after them.
// Then A = L L^T, d = log det A and X <- L^{-1} X in place.  A (n x n lower,
// row pitch n rounded up to 4) lives in the workgroup's global scratch slot.
// Blocked right-looking Cholesky with 64-wide block columns: the diagonal
// block is factored and inverted by one wave in LDS (wave_chol_inv64); the
// right-hand sides of the block rows are solved with that inverse (each wave
// a 16-column slice at a time, the slice in registers); the panel below is
// formed 64 rows at a time as A_ik L_kk^{-T} in LDS, then the trailing
// triangle and the right-hand sides of those rows are updated with it.  Every
// matrix product runs on the matrix cores; the k index of a 16-wide step is
// permuted the same way on both operands (lane group g holds k = 4g .. 4g+3),
// so that F rows are loaded four consecutive doubles at a time.
constexpr int FPD = 66;  // LDS pitch of the 64-column tiles (matrix-core operand reads hit each bank twice)

template <int MODE>
__device__ __forceinline__ void fin_body(const KArgs& a, double* Tt, double* Pn, double* red, int* flag, int* tick) {
    const int tid = threadIdx.x, lane = tid & 63, lr = lane & 15, lg = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index, uniform
    const int64_t total = a.ntasks * a.ntheta;
    const int M = a.M, P = a.P;
    // first product column and product columns (the further approximation:
    // the leaf's own-knot columns W before column 0, the matrix W W^T + tau I)
    const int cm = MODE == FIN_LEAF ? (a.fa ? -P : 0) : (M - 1 - a.level) * P;
    const int K = MODE == FIN_LEAF ? (a.fa ? P : (M - 1) * P) : P;
    const int xc0 = MODE == FIN_LEAF ? 0 : cm + P;                 // first right-hand-side column
    const int W = a.WF - xc0;                                      // right-hand-side columns
    const int nsl = (W + 15) / 16;                                 // 16-column slices
    double* Ag = a.scratch + int64_t(blockIdx.x) * a.scratch_stride;
    // tasks theta-minor: all theta of the first region, then of the next
    // (regions come largest first, so that the longest tasks start first).
    // One launch for groups sharing a prior: the others' tasks of region i,
    // then the representatives' tasks of region i - LAG (so that a
    // representative rarely has to wait for the others' first block step),
    // and at the end the representatives of the last LAG regions.
    const bool merged = MODE == FIN_LEAF && a.rep && a.leaf_phase == 3;
    constexpr int64_t LAG = 64;
    for (int64_t t = next_task(a, -1, tick); t < total; t = next_task(a, t, tick)) {
        int64_t ti;
        int th;
        if (!merged) {
            ti = t / a.ntheta;
            th = int(t - ti * a.ntheta);
        } else {
            const int nr = a.need[a.ntheta], nn = a.ntheta - nr;  // representatives, others
            const int64_t L = a.ntasks < LAG ? a.ntasks : LAG;
            int64_t q;
            bool rslot;
            if (nn == 0) {
                ti = t / nr, q = t - ti * nr, rslot = true;
            } else if (t < L * nn) {
                ti = t / nn, q = t - ti * nn, rslot = false;
            } else {
                const int64_t t1 = t - L * nn, per = nn + nr, mid = (a.ntasks - L) * per;
                if (t1 < mid) {
                    const int64_t i = L + t1 / per, off = t1 - (i - L) * per;
                    rslot = off >= nn;
                    ti = rslot ? i - L : i;
                    q = rslot ? off - nn : off;
                } else {
                    const int64_t t2 = t1 - mid;
                    ti = a.ntasks - L + t2 / nr, q = t2 % nr, rslot = true;
                }
            }
            th = __builtin_amdgcn_readfirstlane(a.order[rslot ? nn + q : q]);
        }
        const bool is_rep = MODE == FIN_LEAF && a.rep && a.rep[th] == th;
        if (MODE == FIN_LEAF && a.rep && !merged && (a.leaf_phase == 0) == is_rep) continue;  // uniform
        const int64_t g = a.tasks[ti];
        const int64_t lo = a.obs_lo[g];
        const int n = int(a.obs_hi[g] - lo);
        const int lda = (n + 3) & ~3;
        const double* thp = a.theta + 3 * th;
        const double alpha = thp[0], inv_beta = 1.0 / thp[1], tau = thp[2];
        double* Fr = a.F + th * a.F_stride + lo * a.WFs;
        // rows read at their first touch (the matrix, and every row in the
        // first block step): [V | z] of the representative for a theta that
        // shares it, else the theta's own
        const double* Fs = (MODE == FIN_LEAF && a.rep && !is_rep) ? a.F + a.rep[th] * a.F_stride + lo * a.WFs : Fr;
        const double* px = a.x + lo;
        const double* py = a.y + lo;
        // a shared prior: C - V V^T of the leaf, formed once per representative
        // (phase 2) and taken from there by every theta of its group
        const bool s0_build = MODE == FIN_LEAF && a.S0 && a.leaf_phase == 2;
        const bool s0_use = MODE == FIN_LEAF && a.S0 && a.leaf_phase != 2;
        double* S0p = (MODE == FIN_LEAF && a.S0) ? a.S0 + a.rep[th] * a.S0_stride + a.S0_off[g - a.lvl[M - 1]] : nullptr;
        // (a representative's own rows already hold z: its chain wrote them)
        if (MODE == FIN_LEAF && !s0_build && !(merged && is_rep))
            for (int r = tid; r < n; r += NT) Fr[int64_t(r) * a.WFs + (a.WF - 1)] = a.z[lo + r];
        // one launch for the whole group: a theta reading its representative's
        // rows counts itself done once past the first block step (or on
        // failure); the representative's task, taken from the queue after
        // all of them (so each is running or finished), waits for that count
        // before it writes its rows
        bool released = !(merged && !is_rep);
        auto release = [&]() {
            if (released) return;
            released = true;
            __syncthreads();  // every read of the representative's rows is done
            if (tid == 0)
                __hip_atomic_fetch_add(a.wait + ti * a.ntheta + a.rep[th], 1, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
        };
        // ---- 1. the matrix: 16-row strips (round robin over the waves),
        // 64 columns (four 16 x 16 tiles) at a time, lower triangle
        double* Sd = s0_build ? S0p : Ag;
        const int ns = s0_use ? 0 : (n + 15) / 16;
        // (with a shared prior the first block step reads the group's
        // C - V V^T, plus this theta's nugget on the diagonal, in place of the
        // matrix, and writes its results to the scratch slot as usual)
        for (int st = ns - 1 - w; st >= 0; st -= 4) {
            const int r = 16 * st + lr;
            const bool rok = r < n;
            const double* ra = Fs + (rok ? int64_t(r) * a.WFs : 0) + cm;
            for (int cg = 0; cg <= st; cg += 4) {
                v4d acc[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
                const double* cb[4];
                bool cok[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int cc = 16 * (cg + c) + lr;
                    cok[c] = cg + c <= st && cc < n;
                    cb[c] = Fs + (cok[c] ? int64_t(cc) * a.WFs : 0) + cm;
                }
                for (int k0 = 0; k0 < K; k0 += 32) {
                    v4d av[2], bv[2][4];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int kk = k0 + 16 * h + 4 * lg;
                        av[h] = (rok && kk < K) ? *reinterpret_cast<const v4d*>(ra + kk) : v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            bv[h][c] = (cok[c] && kk < K) ? *reinterpret_cast<const v4d*>(cb[c] + kk)
                                                          : v4d{0.0, 0.0, 0.0, 0.0};
                    }
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
#pragma unroll
                            for (int c = 0; c < 4; ++c) acc[c] = mfma(av[h][j], bv[h][c][j], acc[c]);
                }
                // epilogue: lane holds column 16 (cg + c) + lr of rows 16 st + lg + 4 i
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int cc = 16 * (cg + c) + lr;
                    if (cg + c > st || cc >= n) continue;
                    double cx = 0.0, cy = 0.0;
                    if (MODE == FIN_LEAF && !a.fa) { cx = px[cc]; cy = py[cc]; }
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int rr = 16 * st + lg + 4 * i;
                        if (rr < n && cc <= rr) {
                            double v;
                            if (MODE == FIN_LEAF) {
                                v = a.fa ? acc[c][i] : cov_pts(px[rr], py[rr], cx, cy, alpha, inv_beta, a.smooth) - acc[c][i];
                                if (rr == cc && !s0_build) v += tau;
                            } else {
                                v = acc[c][i] + (rr == cc ? 1.0 : 0.0);
                            }
                            Sd[int64_t(rr) * lda + cc] = v;
                        }
                    }
                }
            }
        }
        if (merged && is_rep) {
            if (tid == 0) {
                const int need = a.need[th];
                const int* c = a.wait + ti * a.ntheta + th;
                int it = 0;
                while (__hip_atomic_load(c, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need && ++it < (1 << 22))
                    __builtin_amdgcn_s_sleep(8);
                *flag = it >= (1 << 22) ? 1 : 0;
                if (*flag)  // (bounded wait ran out) the group's results are void
                    for (int i = 0; i < a.ntheta; ++i)
                        if (a.rep[i] == th) atomicCAS(a.status + i, 0, STATUS_WAIT);
            }
            __syncthreads();
            if (*flag) continue;  // uniform
        }
        __syncthreads();
        if (s0_build) continue;  // uniform: phase 2 forms the matrix only
        // ---- 2. blocked factorization and solve
        double logdet = 0.0;
        bool failed = false;
        for (int j0 = 0; j0 < n; j0 += 64) {
            const int jb = min(64, n - j0);
            // the matrix as this step reads it: the shared C - V V^T (+ tau on
            // the diagonal) in the first step of a theta that shares a prior
            const bool from_s0 = s0_use && j0 == 0;
            const double* As = from_s0 ? S0p : Ag;
            const double dtau = from_s0 ? tau : 0.0;
            // a. the diagonal block into LDS (lower part)
            for (int e = tid; e < 64 * 64; e += NT) {
                const int i = e >> 6, j = e & 63;
                Tt[i * FPD + j] = (i < jb && j <= i) ? As[int64_t(j0 + i) * lda + j0 + j] + (i == j ? dtau : 0.0) : 0.0;
            }
            __syncthreads();
            // b. one wave: factor and inverse
            if (w == 0) {
                double ldv = 0.0;
                const bool bad = wave_chol_inv64(Tt, FPD, jb, &ldv);
                if (lane == 0) { *flag = bad ? 1 : 0; red[0] = ldv; }
            }
            __syncthreads();
            if (*flag) { failed = true; break; }
            logdet += red[0];
            // the panel below, 64 rows (a chunk) at a time:
            //   P = A[r0 .., j0 ..] L_kk^{-T} into LDS (wave w forms rows
            //   r0 + 16 w .. + 15) and into the scratch slot
            auto panel = [&](int r0) {
                const int r = r0 + 16 * w + lr;
                const bool rok = r < n;
                const double* ra = As + (rok ? int64_t(r) * lda : 0) + j0;
                v4d acc[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int k = 16 * kk + 4 * lg;
                    double av[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) av[j] = (rok && k + j < jb) ? ra[k + j] : 0.0;
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int c = 0; c < 4; ++c) acc[c] = mfma(av[j], Tt[(16 * c + lr) * FPD + k + j], acc[c]);
                }
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int rr = 16 * w + lg + 4 * i, cc = 16 * c + lr;
                        Pn[rr * FPD + cc] = acc[c][i];
                        if (r0 + rr < n) Ag[int64_t(r0 + rr) * lda + j0 + cc] = acc[c][i];
                    }
            };
            //   trailing triangle of the chunk's rows: A[r][c] -= P_r . P_c for
            //   j0 + 64 <= c <= r (P_c from LDS for this chunk, from the
            //   scratch slot for earlier chunks)
            auto syrk = [&](int r0) {
                const int R = r0 + 16 * w;
                if (R >= n) return;
#pragma unroll 1
                for (int cb0 = j0 + 64; cb0 <= r0; cb0 += 64) {
                    const bool here = cb0 == r0;
                    v4d acc[4];
                    bool tok[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const int c0 = cb0 + 16 * c;
                        tok[c] = c0 < n && c0 <= R + 15;
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int rr = R + lg + 4 * i, cc = c0 + lr;
                            const bool ok = tok[c] && rr < n && cc < n && cc <= rr;
                            acc[c][i] = ldg0(As, int64_t(rr) * lda + cc, ok) + (ok && rr == cc ? dtau : 0.0);
                        }
                    }
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        const int k = 16 * kk + 4 * lg;
                        double av[4], bv[4][4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) av[j] = Pn[(16 * w + lr) * FPD + k + j];
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            const int cr = 16 * c + lr;  // row of P within its chunk
                            if (here) {
#pragma unroll
                                for (int j = 0; j < 4; ++j) bv[c][j] = Pn[cr * FPD + k + j];
                            } else {
                                const bool ok = tok[c] && cb0 + cr < n;
                                const v4d v = *reinterpret_cast<const v4d*>(Ag + (ok ? int64_t(cb0 + cr) * lda + j0 + k : 0));
#pragma unroll
                                for (int j = 0; j < 4; ++j) bv[c][j] = ok ? v[j] : 0.0;
                            }
                        }
#pragma unroll
                        for (int j = 0; j < 4; ++j)
#pragma unroll
                            for (int c = 0; c < 4; ++c) acc[c] = mfma(-av[j], bv[c][j], acc[c]);
                    }
#pragma unroll
                    for (int c = 0; c < 4; ++c)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int rr = R + lg + 4 * i, cc = cb0 + 16 * c + lr;
                            if (tok[c] && rr < n && cc < n && cc <= rr) Ag[int64_t(rr) * lda + cc] = acc[c][i];
                        }
                }
            };
            // c. the first chunk's panel and trailing triangle
            const int r1 = j0 + 64;
            const bool chunk1 = r1 < n;
            if (chunk1) {
                panel(r1);
                __syncthreads();
                syrk(r1);
            }
            // d. right-hand sides: X_k <- L_kk^{-1} X_k, then (fused) the first
            // chunk's rows X_r -= P_r X_k with the solved tiles as the second
            // operand; each wave a 16-column slice at a time, the next slice's
            // rows loaded while the current one is computed
            {
                // row r of a slice: base + (r - lg) * WFs with a per-lane base
                // and a uniform offset (no per-row address kept live); a
                // masked lane reads the region's first element instead (the
                // base itself may lie past the region's last row)
                const int64_t s4 = int64_t(4) * a.WFs;
                const double* Fx = j0 == 0 ? Fs : Fr;  // rows not yet written by this task
                auto load_k = [&](int sl, v4d (&v)[4]) {
                    const int c = xc0 + 16 * sl + lr;
                    const bool cok = sl < nsl && c < a.WF;
                    const double* b = Fx + int64_t(j0 + lg) * a.WFs + c;
#pragma unroll
                    for (int t2 = 0; t2 < 4; ++t2)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const bool ok = cok && 16 * t2 + lg + 4 * i < jb;
                            const double vv = *(ok ? b + (4 * t2 + i) * s4 : Fx);
                            v[t2][i] = ok ? vv : 0.0;
                        }
                };
                v4d xv[4];
                load_k(w, xv);
#pragma unroll 1
                for (int sl = w; sl < nsl; sl += 4) {
                    const int c = xc0 + 16 * sl + lr;
                    const bool cok = c < a.WF;
                    v4d xr[4];
                    double* bk = Fr + int64_t(j0 + lg) * a.WFs + c;  // rows of block k (stores only when valid)
                    double* b1 = Fr + int64_t(r1 + lg) * a.WFs + c;  // rows of the first chunk
                    if (chunk1) {
                        const double* b1x = Fx + int64_t(r1 + lg) * a.WFs + c;
#pragma unroll
                        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                const bool ok = cok && r1 + 16 * rt + lg + 4 * i < n;
                                const double vv = *(ok ? b1x + (4 * rt + i) * s4 : Fx);
                                xr[rt][i] = ok ? vv : 0.0;
                            }
                    }
                    v4d xn[4];
                    load_k(sl + 4, xn);
                    v4d o[4];
#pragma unroll
                    for (int t2 = 0; t2 < 4; ++t2) {
                        o[t2] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                        for (int k2 = 0; k2 <= t2; ++k2)
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                o[t2] = mfma(Tt[(16 * t2 + lr) * FPD + 16 * k2 + 4 * q + lg], xv[k2][q], o[t2]);
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            if (cok && 16 * t2 + lg + 4 * i < jb) bk[(4 * t2 + i) * s4] = o[t2][i];
                    }
                    if (chunk1) {
#pragma unroll
                        for (int rt = 0; rt < 4; ++rt) {
#pragma unroll
                            for (int t2 = 0; t2 < 4; ++t2)
#pragma unroll
                                for (int q = 0; q < 4; ++q)
                                    xr[rt] = mfma(-Pn[(16 * rt + lr) * FPD + 16 * t2 + 4 * q + lg], o[t2][q], xr[rt]);
#pragma unroll
                            for (int i = 0; i < 4; ++i)
                                if (cok && r1 + 16 * rt + lg + 4 * i < n) b1[(4 * rt + i) * s4] = xr[rt][i];
                        }
                    }
#pragma unroll
                    for (int t2 = 0; t2 < 4; ++t2) xv[t2] = xn[t2];
                }
            }
            __syncthreads();
            // e. further chunks: panel, trailing triangle, right-hand sides
            // (X_k read back from memory)
#pragma unroll 1
            for (int r0 = r1 + 64; r0 < n; r0 += 64) {
                panel(r0);
                __syncthreads();
                syrk(r0);
#pragma unroll 1
                for (int sl = w; sl < nsl; sl += 4) {
                    const int c = xc0 + 16 * sl + lr;
                    const bool cok = c < a.WF;
                    double xb[4][4];  // X_k[16 t2 + 4 q + lg][c]
#pragma unroll
                    for (int t2 = 0; t2 < 4; ++t2)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            xb[t2][q] = ldg0(Fr, int64_t(j0 + 16 * t2 + 4 * q + lg) * a.WFs + c, cok);
#pragma unroll
                    for (int rt = 0; rt < 4; ++rt) {
                        if (r0 + 16 * rt >= n) break;
                        v4d o;
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int rr = r0 + 16 * rt + lg + 4 * i;
                            o[i] = ldg0(j0 == 0 ? Fs : Fr, int64_t(rr) * a.WFs + c, cok && rr < n);
                        }
#pragma unroll
                        for (int t2 = 0; t2 < 4; ++t2)
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                o = mfma(-Pn[(16 * rt + lr) * FPD + 16 * t2 + 4 * q + lg], xb[t2][q], o);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int rr = r0 + 16 * rt + lg + 4 * i;
                            if (cok && rr < n) Fr[int64_t(rr) * a.WFs + c] = o[i];
                        }
                    }
                }
                __syncthreads();
            }
            if (j0 == 0) release();
        }
        release();  // (a failed first block step)
        if (failed) {
            flag_fail(a, th, g);
            __syncthreads();
            continue;
        }
        if (tid == 0) a.dval[th * a.d_stride + g] = 2.0 * logdet;
        __syncthreads();
    }
    queue_done(a);
}

__global__ void __launch_bounds__(NT, 2) k_leaf_finish(KArgs a) {
    __shared__ double Tt[64 * FPD];
    __shared__ double Pn[64 * FPD];
    __shared__ double red[4];
    __shared__ int flag, tick;
    fin_body<FIN_LEAF>(a, Tt, Pn, red, &flag, &tick);
}

__global__ void __launch_bounds__(NT, 2) k_fold_factor(KArgs a) {
    __shared__ double Tt[64 * FPD];
    __shared__ double Pn[64 * FPD];
    __shared__ double red[4];
    __shared__ int flag, tick;
    fin_body<FIN_FOLD>(a, Tt, Pn, red, &flag, &tick);
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
