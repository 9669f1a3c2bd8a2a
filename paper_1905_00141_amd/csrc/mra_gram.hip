// Knot-space folds, the final log-likelihood sum and fills.
#include "mra_device.h"

namespace mra {

// Knot-space fold in two launches.  With D = mP + 1 and the columns of a
// level-m region (its own knots, then the ancestors' knots, then the data):
//   G = sum over the children of F_c^T F_c (observation-space children, F rows)
//       or of their Schur blocks (knot-space children);
//   L L^T = I + G[0:P, 0:P];  Z = G[P:D, 0:P] L^{-T};  S = G[P:D, P:D] - Z Z^T.
// The parent reads S (lower triangle); prediction reads L^{-1} and Z.
//
// k_gram_panel (one workgroup per region): the first block column of G and
// its last row, the factor and inverse of I + G[0:P, 0:P], Z, and the last
// row of S (the data row, computed with the vector units).
// k_gram_tile (one wave per 64 x 64 block of S below the data row): the block
// is accumulated over all children in registers and written once.

// the children of region g (level m) as runs of consecutive observation-space
// children (one row range each) and knot-space children (one block each)
__device__ __forceinline__ bool child_is_rows(const KArgs& a, int m, int64_t gc) {
    return m + 1 == a.M || a.form[gc] == FOLD_FACTOR;
}

// The first block column of the Gram sum over one run of observation rows,
// with its data row: for the rows' F columns f_0 .. f_{D-1} (f_{D-1} = z),
//   G[r][c] (=|+=) sum_k f_r(k) f_c(k)   for r < D - 1, c < P   (matrix cores)
//   G[D-1][r] (=|+=) sum_k z(k) f_r(k)   for r < D - 1          (vector units)
//   G[D-1][D-1] (=|+=) sum_k z(k)^2
// Each wave takes 64-row blocks round robin and, while its matrix products
// run, multiplies the A fragments it has loaded by z (four more loads per
// 16 k), so the data row costs no pass of its own.  F(k, c) = F[k ld + c].
// Ends with a workgroup barrier.
template <int MODE>
__device__ __forceinline__ void panel_gather(double* G, int D, int P, int K, const double* F, int64_t ld) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 15, lg = lane >> 4;
    const int R = D - 1, nbr = (R + TB - 1) / TB;
    const double* zc = F + (D - 1);
    double* grow = G + int64_t(D - 1) * D;
    for (int br = w; br < nbr; br += NT / 64) {
        const int r0 = br * TB;
        v4d acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
        double yp[4] = {0.0, 0.0, 0.0, 0.0}, zz = 0.0;
        bool rok[4], cok[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            rok[t] = r0 + 16 * t + lr < R;
            cok[t] = 16 * t + lr < P;
        }
        for (int k0 = 0; k0 < K; k0 += 16) {
            double fa[4][4], fb[4][4], zv[4];  // [tile][k-step]
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = k0 + 4 * q + lg;
                const bool kok = k < K;
                const double* row = F + (kok ? int64_t(k) * ld : 0);
                zv[q] = kok ? zc[row - F] : 0.0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const double va = row[rok[t] ? r0 + 16 * t + lr : 0];
                    const double vb = row[cok[t] ? 16 * t + lr : 0];
                    fa[t][q] = (rok[t] && kok) ? va : 0.0;
                    fb[t][q] = (cok[t] && kok) ? vb : 0.0;
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = mfma(fa[i][q], fb[j][q], acc[i][j]);
#pragma unroll
                for (int t = 0; t < 4; ++t) yp[t] = fma(zv[q], fa[t][q], yp[t]);
                if (br == 0) zz = fma(zv[q], zv[q], zz);
            }
        }
        // the data row: sum over the four lane groups (k = 4q + lg)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            yp[t] += __shfl_xor(yp[t], 16);
            yp[t] += __shfl_xor(yp[t], 32);
            const int r = r0 + 16 * t + lr;
            if (lg == 0 && r < R) grow[r] = MODE == MM_ADD ? grow[r] + yp[t] : yp[t];
        }
        if (br == 0) {
            zz += __shfl_xor(zz, 16);
            zz += __shfl_xor(zz, 32);
            if (lane == 0) grow[D - 1] = MODE == MM_ADD ? grow[D - 1] + zz : zz;
        }
        // the block: one 16-row strip at a time, reads of G batched before writes
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double cold[4][4];
            if (MODE == MM_ADD) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int r = r0 + 16 * i + lg + 4 * e, c = 16 * j + lr;
                        cold[j][e] = ldg0(G, int64_t(r) * D + c, r < R && c < P);
                    }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = r0 + 16 * i + lg + 4 * e, c = 16 * j + lr;
                    if (r < R && c < P) G[int64_t(r) * D + c] = MODE == MM_ADD ? cold[j][e] + acc[i][j][e] : acc[i][j][e];
                }
        }
    }
    __syncthreads();
}

__global__ void __launch_bounds__(NT, 2) k_gram_panel(KArgs a) {
    __shared__ Smem s;
    const int64_t total = a.ntasks * a.ntheta;
    const int m = a.level, P = a.P, M = a.M;
    const int cm = (M - 1 - m) * P;
    const int D = m * P + 1, Dt = D - P;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        const int th = int(t / a.ntasks);
        const int64_t g = a.tasks[t % a.ntasks];
        const int64_t k = g - a.lvl[m - 1];
        double* G = a.gram + th * a.gram_stride + a.gram_off[g];
        const double* Fth = a.F + th * a.F_stride;
        double* yrow = G + int64_t(D - 1) * D + P;  // last row of S: columns P .. D-1
        bool first = true;
        // knot-space children: their blocks are added after the runs of
        // observation rows, all in one pass (up to J independent loads per
        // element instead of one pass per child)
        const double* kcs[MAXJ];
        bool anyk = false;
#pragma unroll
        for (int j = 0; j < MAXJ; ++j) {
            kcs[j] = nullptr;
            if (j < a.J) {
                const int64_t gc = a.lvl[m] + a.J * k + j;
                if (!child_is_rows(a, m, gc)) kcs[j] = a.gram + th * a.gram_stride + a.gram_off[gc], anyk = true;
            }
        }
        for (int j = 0; j < a.J;) {
            const int64_t gc = a.lvl[m] + a.J * k + j;
            if (child_is_rows(a, m, gc)) {
                // a run of consecutive observation-space children: one row range
                int j2 = j + 1;
                while (j2 < a.J && child_is_rows(a, m, a.lvl[m] + a.J * k + j2)) ++j2;
                const int64_t lo = a.obs_lo[gc], hi = a.obs_hi[a.lvl[m] + a.J * k + j2 - 1];
                j = j2;
                const int nc = int(hi - lo);
                if (nc == 0) continue;
                const double* Fc = Fth + lo * a.WFs + cm;
                if (first) panel_gather<MM_SET>(G, D, P, nc, Fc, a.WFs);
                else panel_gather<MM_ADD>(G, D, P, nc, Fc, a.WFs);
                first = false;
            } else {
                ++j;
            }
        }
        if (anyk) {
            // G[i][c] for i < D, c < P (lower part of the top block only), a
            // row per wave step and a column per lane (P <= 64), and the data
            // row of the Schur complement; child blocks have D + P columns
            const int Dc = D + P, lane = threadIdx.x & 63;
            for (int i = threadIdx.x >> 6; i < D; i += NT / 64)
                if (lane < P && lane <= i) {
                    const int64_t off = int64_t(P + i) * Dc + P + lane;
                    double v = 0.0;
#pragma unroll
                    for (int q = 0; q < MAXJ; ++q)
                        if (kcs[q]) v += kcs[q][off];
                    double* gp = G + int64_t(i) * D + lane;
                    *gp = first ? v : *gp + v;
                }
            for (int c = threadIdx.x; c < Dt; c += NT) {
                const int64_t off = int64_t(P + D - 1) * Dc + P + P + c;
                double v = 0.0;
#pragma unroll
                for (int q = 0; q < MAXJ; ++q)
                    if (kcs[q]) v += kcs[q][off];
                yrow[c] = first ? v : yrow[c] + v;
            }
            __syncthreads();
        }
        // I + G[0:P, 0:P] -> Cholesky factor and inverse in LDS
        for (int e = threadIdx.x; e < TB * TB; e += NT) {
            const int i = e / TB, j = e % TB;
            s.L[i * MLD + j] = (i < P && j <= i) ? G[int64_t(i) * D + j] + (i == j ? 1.0 : 0.0) : 0.0;
        }
        __syncthreads();
        // one wave: the factor's inverse replaces the tile
        if ((threadIdx.x >> 6) == 0) {
            double ldv = 0.0;
            const bool bad = wave_chol_inv<4, 0>(s.L, MLD, P, &ldv);
            if (threadIdx.x == 0) { s.flag = bad ? 1 : 0; s.Li[0] = ldv; }
        }
        __syncthreads();
        const bool bad = s.flag != 0;
        const double ldv = s.Li[0];
        __syncthreads();
        if (bad) {
            flag_fail(a, th, g);
            continue;
        }
        if (threadIdx.x == 0) a.dval[th * a.d_stride + g] = 2.0 * ldv;
#pragma unroll 4
        for (int i = threadIdx.x >> 6; i < P; i += NT / 64) {
            const int j = threadIdx.x & 63;
            if (j < P) G[int64_t(i) * D + j] = (j <= i) ? s.L[i * MLD + j] : 0.0;
        }
        // Z = G[P:D, 0:P] L^{-T} in place: the data row (Z's last) by the
        // last wave, one column per lane, before its share of the blocks of
        // the other rows on the matrix cores
        double* Z = G + int64_t(P) * D;
        if ((threadIdx.x >> 6) == NT / 64 - 1) {
            // the row is read once (one value per lane) and broadcast lane by lane
            const int lane = threadIdx.x & 63;
            double* zl = Z + int64_t(Dt - 1) * D;
            const double zr = ldg0(zl, lane, lane < P);
            const int zlo = __double2loint(zr), zhi = __double2hiint(zr);
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < 64; ++k) {
                const double zk = __hiloint2double(__builtin_amdgcn_readlane(zhi, k), __builtin_amdgcn_readlane(zlo, k));
                v = fma(zk, (k < P && lane < P) ? s.L[lane * MLD + k] : 0.0, v);
            }
            if (lane < P) zl[lane] = v;
        }
        wg_mm<MM_SET>(Z, D, Dt - 1, P, P, Z, D, 1, s.L, MLD, 1, false, s.mm);
        // last row of S: yrow[c] -= Z[Dt-1] . Z[c].  A wave step takes 8 rows
        // c, two per 16-lane group; each lane multiplies four consecutive k
        // (a row is read as one contiguous 512-byte run) and the group sums
        // its lanes by shuffles in a fixed order
        {
            const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, rs = lane >> 4, kq = lane & 15;
            const double* zl = Z + int64_t(Dt - 1) * D;
            double zk[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) zk[i] = ldg0(zl, 4 * kq + i, 4 * kq + i < P);
            for (int c0 = 8 * w; c0 < Dt; c0 += 32) {
                double v[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int c = c0 + 4 * h + rs;
                    double zc[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) zc[i] = ldg0(Z, int64_t(c) * D + 4 * kq + i, c < Dt && 4 * kq + i < P);
                    v[h] = fma(zk[0], zc[0], zk[1] * zc[1]) + fma(zk[2], zc[2], zk[3] * zc[3]);
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
#pragma unroll
                    for (int off = 8; off > 0; off >>= 1) v[h] += __shfl_xor(v[h], off);
                    const int c = c0 + 4 * h + rs;
                    if (kq == 0 && c < Dt) yrow[c] -= v[h];
                }
            }
        }
        __syncthreads();
    }
}

// One wave per 64 x 64 block (bi >= bj) of S[0:Ds, 0:Ds], Ds = (m-1)P (rows
// and columns counted from P in G; the data row is done by k_gram_panel).
// Knot-space children initialise the accumulators, observation-space runs
// add F_c^T F_c on the matrix cores, Z Z^T is subtracted, and the lower part
// of the block is written once.
__global__ void __launch_bounds__(NT, 2) k_gram_tile(KArgs a) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 15, lg = lane >> 4;
    const int m = a.level, P = a.P, M = a.M;
    const int cm = (M - 1 - m) * P;
    const int D = m * P + 1, Ds = (m - 1) * P;
    const int nb = (Ds + TB - 1) / TB;
    const int64_t ntile = int64_t(nb) * (nb + 1) / 2;
    const int64_t total = a.ntasks * a.ntheta * ntile;
    for (int64_t wt = int64_t(blockIdx.x) * 4 + w; wt < total; wt += int64_t(gridDim.x) * 4) {
        const int64_t rt = wt / ntile;
        int64_t tix = wt % ntile;
        int bi = 0;
        while (tix > bi) { tix -= bi + 1; ++bi; }
        const int bj = int(tix);
        const int th = int(rt / a.ntasks);
        const int64_t g = a.tasks[rt % a.ntasks];
        const int64_t k = g - a.lvl[m - 1];
        double* G = a.gram + th * a.gram_stride + a.gram_off[g];
        const double* Fth = a.F + th * a.F_stride;
        const int r0 = bi * TB, c0 = bj * TB;  // within S
        bool rv[4], cv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            rv[t] = r0 + 16 * t + lr < Ds;
            cv[t] = c0 + 16 * t + lr < Ds;
        }
        v4d acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
        for (int j = 0; j < a.J;) {
            const int64_t gc = a.lvl[m] + a.J * k + j;
            if (child_is_rows(a, m, gc)) {
                int j2 = j + 1;
                while (j2 < a.J && child_is_rows(a, m, a.lvl[m] + a.J * k + j2)) ++j2;
                const int64_t lo = a.obs_lo[gc], hi = a.obs_hi[a.lvl[m] + a.J * k + j2 - 1];
                j = j2;
                const int nc = int(hi - lo);
                if (nc == 0) continue;
                // S column x is F column cm + P + x
                const double* Fa = Fth + lo * a.WFs + cm + P + r0;
                const double* Fb = Fth + lo * a.WFs + cm + P + c0;
                for (int k0 = 0; k0 < nc; k0 += 16) {
                    double fa[4][4], fb[4][4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int kk = k0 + 4 * q + lg;
                        const bool kok = kk < nc;
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const int64_t o = int64_t(kk) * a.WFs + 16 * t + lr;
                            fa[t][q] = ldg0(Fa, o, kok && rv[t]);
                            fb[t][q] = ldg0(Fb, o, kok && cv[t]);
                        }
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
#pragma unroll
                            for (int jj = 0; jj < 4; ++jj)
                                if (bi > bj || jj <= i) acc[i][jj] = mfma(fa[i][q], fb[jj][q], acc[i][jj]);
                }
            } else {
                ++j;  // knot-space child: added in the epilogue
            }
        }
        // - Z Z^T over the P columns of Z (row P + x of G holds Z row x)
        const double* Za = G + int64_t(P + r0) * D;
        const double* Zb = G + int64_t(P + c0) * D;
        for (int k0 = 0; k0 < P; k0 += 16) {
            double fa[4][4], fb[4][4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int kk = k0 + 4 * q + lg;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    fa[t][q] = ldg0(Za, int64_t(16 * t + lr) * D + kk, rv[t]);
                    fb[t][q] = ldg0(Zb, int64_t(16 * t + lr) * D + kk, cv[t]);
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj)
                        if (bi > bj || jj <= i) acc[i][jj] = mfma(-fa[i][q], fb[jj][q], acc[i][jj]);
        }
        // the lower part of the block, written once (row P + r, column P + c of
        // G), with the knot-space children's Schur blocks (their rows and
        // columns P + P + (r, c)) added one 16-row strip at a time
        const int Dc = D + P;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double add[4][4];
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                for (int e = 0; e < 4; ++e) add[jj][e] = 0.0;
            for (int j = 0; j < a.J; ++j) {
                const int64_t gc = a.lvl[m] + a.J * k + j;
                if (child_is_rows(a, m, gc)) continue;
                const double* Gc = a.gram + th * a.gram_stride + a.gram_off[gc];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int r = r0 + 16 * i + lg + 4 * e, c = c0 + 16 * jj + lr;
                        add[jj][e] += ldg0(Gc, int64_t(2 * P + r) * Dc + 2 * P + c, r < Ds && c < Ds && c <= r);
                    }
            }
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = r0 + 16 * i + lg + 4 * e, c = c0 + 16 * jj + lr;
                    if (r < Ds && c < Ds && c <= r) G[int64_t(P + r) * D + P + c] = acc[i][jj][e] + add[jj][e];
                }
        }
    }
}

// The same blocks of S, one workgroup per 128 x 128 super-block (bi >= bj):
// the observation-space rows are staged through LDS 16 at a time, each wave
// computing one 64 x 64 quarter from the shared copy, so every F row segment
// is read from memory once per super-block instead of once per 64 x 64 block.
// The next chunk is loaded into registers while the current one is used.
constexpr int SB = 128;       // super-block edge
constexpr int KCH = 16;       // rows per staged chunk
constexpr int SPAD = SB + 8;  // LDS pitch: the four 16-lane groups of a read fall on different banks

__global__ void __launch_bounds__(NT, 2) k_gram_tile2(KArgs a) {
    __shared__ double As[KCH * SPAD];
    __shared__ double Bs[KCH * SPAD];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 15, lg = lane >> 4;
    const int m = a.level, P = a.P, M = a.M;
    const int cm = (M - 1 - m) * P;
    const int D = m * P + 1, Ds = (m - 1) * P;
    const int nsb = (Ds + SB - 1) / SB;
    const int64_t nst = int64_t(nsb) * (nsb + 1) / 2;
    const int64_t total = a.ntasks * a.ntheta * nst;
    const int wr = w >> 1, wc = w & 1;
    // XCD-aware order: workgroups are dealt round robin over the 8 XCDs, so
    // workgroup b runs on XCD b % 8; each XCD gets a contiguous range of
    // tasks instead, and the super-blocks of one region and theta (adjacent
    // tasks, reading the same child rows) share that XCD's L2
    const int64_t G = gridDim.x, G8 = G - G % 8, b = blockIdx.x;
    const int64_t t0 = b < G8 ? (b % 8) * (G8 / 8) + b / 8 : b;
    for (int64_t t = t0; t < total; t += G) {
        const int64_t rt = t / nst;
        int64_t tix = t % nst;
        int BI = 0;
        while (tix > BI) { tix -= BI + 1; ++BI; }
        const int BJ = int(tix);
        const int th = int(rt / a.ntasks);
        const int64_t g = a.tasks[rt % a.ntasks];
        const int64_t k = g - a.lvl[m - 1];
        double* G = a.gram + th * a.gram_stride + a.gram_off[g];
        const double* Fth = a.F + th * a.F_stride;
        const int R0 = BI * SB, C0 = BJ * SB;
        const int r0 = R0 + 64 * wr, c0 = C0 + 64 * wc;  // this wave's quarter (within S)
        // quarters above the diagonal or past the last row or column (the
        // half-filled last super-block row when Ds is not a multiple of SB)
        // are skipped; their waves still stage operands for the others
        const bool active = !(BI == BJ && wc > wr) && r0 < Ds && c0 < Ds;
        const bool diagq = (BI == BJ && wc == wr);
        v4d acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
        for (int j = 0; j < a.J;) {
            const int64_t gc = a.lvl[m] + a.J * k + j;
            if (!child_is_rows(a, m, gc)) { ++j; continue; }
            int j2 = j + 1;
            while (j2 < a.J && child_is_rows(a, m, a.lvl[m] + a.J * k + j2)) ++j2;
            const int64_t lo = a.obs_lo[gc], hi = a.obs_hi[a.lvl[m] + a.J * k + j2 - 1];
            j = j2;
            const int nc = int(hi - lo);
            if (nc == 0) continue;
            const double* base = Fth + lo * a.WFs + cm + P;  // S column x is base[x]
            // chunk staging: 16 rows x 128 columns per operand, 4 double2 per thread each
            double2 pa[4], pb[4];
            auto load_chunk = [&](int k0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int idx = threadIdx.x + NT * q;
                    const int kr = idx >> 6, c2 = (idx & 63) * 2;
                    const bool kok = k0 + kr < nc;
                    const bool aok = kok && R0 + c2 < Ds, bok = kok && C0 + c2 < Ds;
                    const double* pra = base + int64_t(k0 + kr) * a.WFs + R0 + c2;
                    const double* prb = base + int64_t(k0 + kr) * a.WFs + C0 + c2;
                    const double2 va = *reinterpret_cast<const double2*>(aok ? pra : base);
                    const double2 vb = *reinterpret_cast<const double2*>(bok ? prb : base);
                    pa[q] = aok ? va : double2{0.0, 0.0};
                    pb[q] = bok ? vb : double2{0.0, 0.0};
                }
            };
            load_chunk(0);
            for (int k0 = 0; k0 < nc; k0 += KCH) {
                __syncthreads();
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int idx = threadIdx.x + NT * q;
                    const int kr = idx >> 6, c2 = (idx & 63) * 2;
                    *reinterpret_cast<double2*>(As + kr * SPAD + c2) = pa[q];
                    *reinterpret_cast<double2*>(Bs + kr * SPAD + c2) = pb[q];
                }
                __syncthreads();
                if (k0 + KCH < nc) load_chunk(k0 + KCH);
                if (active) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int kk = 4 * q + lg;
                        double fa[4], fb[4];
#pragma unroll
                        for (int tt = 0; tt < 4; ++tt) {
                            fa[tt] = As[kk * SPAD + 64 * wr + 16 * tt + lr];
                            fb[tt] = Bs[kk * SPAD + 64 * wc + 16 * tt + lr];
                        }
#pragma unroll
                        for (int i = 0; i < 4; ++i)
#pragma unroll
                            for (int jj = 0; jj < 4; ++jj)
                                if (!diagq || jj <= i) acc[i][jj] = mfma(fa[i], fb[jj], acc[i][jj]);
                    }
                }
            }
        }
        if (active) {
            bool rv[4], cv[4];
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) {
                rv[tt] = r0 + 16 * tt + lr < Ds;
                cv[tt] = c0 + 16 * tt + lr < Ds;
            }
            // - Z Z^T over the P columns of Z (row P + x of G holds Z row x)
            const double* Za = G + int64_t(P + r0) * D;
            const double* Zb = G + int64_t(P + c0) * D;
            for (int k0 = 0; k0 < P; k0 += 16) {
                double fa[4][4], fb[4][4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int kk = k0 + 4 * q + lg;
#pragma unroll
                    for (int tt = 0; tt < 4; ++tt) {
                        fa[tt][q] = ldg0(Za, int64_t(16 * tt + lr) * D + kk, rv[tt]);
                        fb[tt][q] = ldg0(Zb, int64_t(16 * tt + lr) * D + kk, cv[tt]);
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj)
                            if (!diagq || jj <= i) acc[i][jj] = mfma(-fa[i][q], fb[jj][q], acc[i][jj]);
            }
            // the lower part of the quarter, written once, knot-space children added
            const int Dc = D + P;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                double add[4][4];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                    for (int e = 0; e < 4; ++e) add[jj][e] = 0.0;
                for (int j = 0; j < a.J; ++j) {
                    const int64_t gc = a.lvl[m] + a.J * k + j;
                    if (child_is_rows(a, m, gc)) continue;
                    const double* Gc = a.gram + th * a.gram_stride + a.gram_off[gc];
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int r = r0 + 16 * i + lg + 4 * e, c = c0 + 16 * jj + lr;
                            add[jj][e] += ldg0(Gc, int64_t(2 * P + r) * Dc + 2 * P + c, r < Ds && c < Ds && c <= r);
                        }
                }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int r = r0 + 16 * i + lg + 4 * e, c = c0 + 16 * jj + lr;
                        if (r < Ds && c < Ds && c <= r) G[int64_t(P + r) * D + P + c] = acc[i][jj][e] + add[jj][e];
                    }
            }
        }
        __syncthreads();
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
    // optional per-level sums (same fixed order within each level)
    if (a.out_lev) {
        for (int m = 1; m <= a.M; ++m) {
            double sl = 0.0;
            for (int64_t g = a.lvl[m - 1] + threadIdx.x; g < a.lvl[m]; g += NT) sl += d[g];
            red[threadIdx.x] = sl;
            __syncthreads();
            for (int w = NT / 2; w > 0; w /= 2) {
                if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
                __syncthreads();
            }
            if (threadIdx.x == 0) a.out_lev[int64_t(th) * a.M + (m - 1)] = (a.status[th] != 0) ? __builtin_nan("") : red[0];
            __syncthreads();
        }
    }
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
        const double* thp = a.theta + 3 * th;
        const bool ok = thp[0] > 0.0 && thp[1] > 0.0 && (thp[2] > 0.0 || (a.zero_nugget && thp[2] == 0.0)) &&
                        thp[0] < 1.0 / 0.0 && thp[1] < 1.0 / 0.0 && thp[2] < 1.0 / 0.0;
        const bool bad = a.status[th] != 0 || !ok;
        if (bad) ll = __builtin_nan("");
        a.out[th] = ll;
        if (a.out_ld) a.out_ld[th] = bad ? __builtin_nan("") : dsum;
        if (a.out_q) a.out_q[th] = bad ? __builtin_nan("") : q;
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

// Representatives of a chunk's theta: rep[i] = the first j <= i with the same
// alpha and range (the prior does not involve the nugget).  Also, in
// rep[nb ..], the theta in the order the leaf finisher takes them (the others
// first, then the representatives) and in rep[2 nb ..], per representative,
// the number of other theta in its group, and in rep[3 nb] the number of
// representatives.  One workgroup.
__global__ void k_rep(const double* theta, int nb, int* rep) {
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        int r = i;
        for (int j = 0; j < i; ++j)
            if (theta[3 * j] == theta[3 * i] && theta[3 * j + 1] == theta[3 * i + 1]) {
                r = j;
                break;
            }
        rep[i] = r;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        int c = 0;
        if (rep[i] == i)
            for (int j = i + 1; j < nb; ++j) c += rep[j] == i ? 1 : 0;
        rep[2 * nb + i] = c;
    }
    if (threadIdx.x == 0) {
        int k = 0;
        for (int i = 0; i < nb; ++i)
            if (rep[i] != i) rep[nb + k++] = i;
        int nr = 0;
        for (int i = 0; i < nb; ++i)
            if (rep[i] == i) rep[nb + k++] = i, ++nr;
        rep[3 * nb] = nr;
    }
}

// A failed prior factor of a representative fails the theta that share it.
__global__ void k_rep_status(const int* rep, int nb, int* status) {
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
        if (rep[i] != i && status[i] == 0) status[i] = status[rep[i]];
}

// ---- host-side launchers

hipError_t launch_rep(const double* theta, int nb, int* rep, hipStream_t st) {
    hipLaunchKernelGGL(k_rep, dim3(1), dim3(64), 0, st, theta, nb, rep);
    return hipGetLastError();
}
hipError_t launch_rep_status(const int* rep, int nb, int* status, hipStream_t st) {
    hipLaunchKernelGGL(k_rep_status, dim3(1), dim3(64), 0, st, rep, nb, status);
    return hipGetLastError();
}

hipError_t launch_gram_panel(const KArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_gram_panel, dim3(grid), dim3(NT), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_gram_tile2(const KArgs& a, hipStream_t st) {
    const int Ds = (a.level - 1) * a.P;
    const int64_t nsb = (Ds + SB - 1) / SB;
    const int64_t blocks = std::min<int64_t>(a.ntasks * a.ntheta * nsb * (nsb + 1) / 2, int64_t(1) << 20);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gram_tile2, dim3(unsigned(blocks)), dim3(NT), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_gram_tile(const KArgs& a, hipStream_t st) {
    const int Ds = (a.level - 1) * a.P;
    const int64_t nb = (Ds + TB - 1) / TB;
    const int64_t waves = a.ntasks * a.ntheta * nb * (nb + 1) / 2;
    if (waves == 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((waves + 3) / 4, int64_t(1) << 20);
    hipLaunchKernelGGL(k_gram_tile, dim3(unsigned(blocks)), dim3(NT), 0, st, a);
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
