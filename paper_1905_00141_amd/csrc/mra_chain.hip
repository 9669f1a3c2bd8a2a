// Whitened prior rows of knots and observations (the prior recursion).
#include "mra_device.h"

namespace mra {

// Whitened prior rows.  mode 0: the r_hat knots of every level-m region
// (a.level = m) for ancestors 1..m-1, written into the region's V store
// (row-major P x mP, block i-1 = V^i).  mode 1: every observation under a
// level-(M-1) region for ancestors 1..M-1, written into the F buffer (block of
// level l at columns (M-1-l)P, the observation's value in the last column).
// For ancestor level l, with C the covariance:
//     V^l = ( C(rows, Q_{A_l}) - sum_{i<l} V^i V^i(Q_{A_l})^T ) L_{A_l}^{-T}.
// Each wave owns 16 rows.  Ancestor levels are taken in groups of GS = 128/P:
// one pending accumulator per level of the group (MFMA destinations, knots x
// rows) receives the covariance, the contributions of all earlier groups (their
// V rows read back from memory) and, right-looking, those of the group's own
// earlier levels.  A V^i in accumulator layout serves directly as the B
// operand: the summation index is permuted consistently on the A operand,
// which is staged in LDS one P x P block at a time.
// Staging of a P x P block (row-major, ld; rows 16-byte aligned) into LDS,
// row-major with pitch P + 2: blk[r * (P + 2) + c] = src[r][c].  A matrix-core
// operand read (lane (l, g) of a 16-lane group reads row r0 + l, column
// c0 + g) then touches every one of the 64 four-byte banks exactly twice (the
// minimum for 64 lanes of 8 bytes), and the staging stores of consecutive
// lanes are consecutive.  Split in two for software pipelining: the loads of the
// next block (into registers) are issued before the current block is used, so
// their latency overlaps the matrix-core work; the stores into LDS follow.
template <int P>
struct StageRegs {
    double2 v[(P * P / 2 + NT - 1) / NT];
};
template <int P>
__device__ __forceinline__ void stage_load(StageRegs<P>& rg, const double* src, int64_t ld) {
    constexpr int E2 = P * P / 2;
    constexpr int PER = (E2 + NT - 1) / NT;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int e = threadIdx.x + j * NT;
        const int r = (2 * e) / P, c = (2 * e) % P;
        const bool ok = e < E2;
        rg.v[j] = *reinterpret_cast<const double2*>(src + (ok ? int64_t(r) * ld + c : 0));
    }
}
template <int P>
__device__ __forceinline__ void stage_store(double* blk, const StageRegs<P>& rg) {
    constexpr int E2 = P * P / 2;
    constexpr int PER = (E2 + NT - 1) / NT;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int e = threadIdx.x + j * NT;
        if (e < E2) {
            const int r = (2 * e) / P, c = (2 * e) % P;
            blk[r * (P + 2) + c] = rg.v[j].x;
            blk[r * (P + 2) + c + 1] = rg.v[j].y;
        }
    }
}

template <int P, int mode>
__global__ void __launch_bounds__(NT, 2) k_chain(KArgs a) {
    constexpr int NM = P / 16;
    constexpr int GS = 128 / P;  // accumulator budget for two workgroups per CU
    // two staging buffers: block s is written while block s - 1 may still be
    // read, so one barrier per block suffices
    __shared__ __align__(16) double blk2[2][P * (P + 2)];
    // the ancestors' knot bars (a knot is a pair of bars, r_hat <= 64 gives <= 8 each)
    __shared__ double kbx[MAXL * 8], kby[MAXL * 8];
    __shared__ int kq[P];  // knot q -> its bars: (q % nx) + 8 (q / nx), or -1 beyond r_hat
    __shared__ int64_t voff[MAXL];
    // the staged blocks of one row tile, in the order the loops below use them:
    // offset into the theta's V stores and row stride
    __shared__ int64_t soff[MAXL * (MAXL + 1) / 2];
    __shared__ int sld[MAXL * (MAXL + 1) / 2];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, lr = lane & 15, lg = lane >> 4;
    const int64_t total = a.ntasks * a.ntheta;
    // level of the task region and ancestor levels of the rows; observation
    // rows of the further approximation are tasked per leaf and include the
    // leaf's own knots (its level-M block lands at column -P)
    const int m = mode == 0 ? a.level : a.M - 1 + a.fa;
    const int L = mode == 0 ? m - 1 : a.M - 1 + a.fa;
    int ph = 0;  // staging buffer parity, continued across tiles and tasks
    for (int q = threadIdx.x; q < P; q += NT) kq[q] = q < a.rhat ? (q % a.nx) + 8 * (q / a.nx) : -1;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        const int th = int(t / a.ntasks);
        if (a.rep && a.rep[th] != th) continue;  // shares its representative's prior
        const int64_t g = a.tasks[t % a.ntasks];
        const int64_t k = g - a.lvl[m - 1];
        const double* thp = a.theta + 3 * th;
        const double alpha = thp[0], inv_beta = 1.0 / thp[1];
        const double* vst = a.vst + th * a.vst_stride;
        if (tid < L) voff[tid] = a.vst_off[ancestor(a, m, k, tid + 1)];
        if (tid < 8 * L) {
            const int l = tid >> 3, pb = tid & 7;
            const double* bx = a.box + 4 * ancestor(a, m, k, l + 1);
            kbx[tid] = pb < a.nx ? grid_bar(bx[0], bx[1], a.nx, a.offset, pb) : 0.0;
            kby[tid] = pb < a.ny ? grid_bar(bx[2], bx[3], a.ny, a.offset, pb) : 0.0;
        }
        __syncthreads();
        int nsteps = 0;
        if (tid == 0) {
            // same order as the compute loops: earlier groups, then the group's
            // diagonal blocks each followed by its right-looking updates
            for (int g0 = 0; g0 < L; g0 += GS) {
                for (int i = 0; i < g0; ++i)
                    for (int l = 0; l < GS; ++l)
                        if (g0 + l < L) { soff[nsteps] = voff[g0 + l] + int64_t(i) * P; sld[nsteps] = (g0 + l + 1) * P; ++nsteps; }
                for (int i = 0; i < GS; ++i) {
                    if (g0 + i >= L) continue;
                    const int li = g0 + i;
                    soff[nsteps] = voff[li] + int64_t(li) * P; sld[nsteps] = (li + 1) * P; ++nsteps;
                    for (int l = i + 1; l < GS; ++l)
                        if (g0 + l < L) { soff[nsteps] = voff[g0 + l] + int64_t(li) * P; sld[nsteps] = (g0 + l + 1) * P; ++nsteps; }
                }
            }
        }
        nsteps = L * (L + 1) / 2;
        __syncthreads();
        StageRegs<P> pf;
        if (nsteps > 0) stage_load<P>(pf, vst + soff[0], sld[0]);
        int step = 0;
        // stage block `step` (held in pf) into the next LDS buffer, start
        // loading the one after, and return the staged copy
        auto advance = [&]() -> const double* {
            double* blk = blk2[ph & 1];
            ++ph;
            stage_store<P>(blk, pf);
            __syncthreads();
            const int nx = (step + 1 < nsteps) ? step + 1 : 0;
            stage_load<P>(pf, vst + soff[nx], sld[nx]);
            ++step;
            return blk;
        };
        int nrows;
        int64_t lo = 0, ldd;
        double* dst;
        if (mode == 0) {
            nrows = P;
            ldd = int64_t(m) * P;
            dst = a.vst + th * a.vst_stride + a.vst_off[g];
        } else {
            lo = a.obs_lo[g];
            nrows = int(a.obs_hi[g] - lo);
            ldd = a.WFs;
            dst = a.F + th * a.F_stride + lo * a.WFs;
        }
        for (int r0 = 0; r0 < nrows; r0 += 64) {
            step = 0;
            const int rr = r0 + 16 * w + lr;
            const bool valid = rr < nrows && (mode == 1 || rr < a.rhat);
            // a wave whose 16 rows all lie past the region's last observation
            // (the ragged last tile) still stages blocks and meets every
            // barrier, but leaves the matrix core to the other workgroup
            const bool act = mode == 0 || __builtin_amdgcn_readfirstlane(r0 + 16 * w) < nrows;
            const bool store = mode == 0 ? (rr < P) : (rr < nrows);
            double px = 0.0, py = 0.0;
            if (valid) {
                if (mode == 1) { px = a.x[lo + rr]; py = a.y[lo + rr]; }
                else knot_xy(a, g, rr, px, py);
            }
            double* drow = dst + int64_t(rr) * ldd;
            if (mode == 1 && store) drow[a.WF - 1] = a.z[lo + rr];  // the data column of [V | z]
            auto colof = [&](int i) -> int64_t { return mode == 0 ? int64_t(i) * P : int64_t(a.M - 2 - i) * P; };
            for (int g0 = 0; g0 < L; g0 += GS) {
                v4d acc[GS][NM];
#pragma unroll
                for (int l = 0; l < GS; ++l)
#pragma unroll
                    for (int mt = 0; mt < NM; ++mt)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int q = 16 * mt + lg + 4 * i;
                            const int la = g0 + l;
                            const int kk = kq[q];
                            const bool ok = la < L && valid && kk >= 0;
                            acc[l][mt][i] = ok ? cov_pts(kbx[la * 8 + (kk & 7)], kby[la * 8 + (kk >> 3)], px, py, alpha,
                                                         inv_beta, a.smooth)
                                               : 0.0;
                        }
                // earlier groups: acc_l -= V^{i+1}(Q_{A_l}) V^{i+1}
                for (int i = 0; i < g0; ++i) {
                    v4d vi[NM];
                    // base: the task's first row (always inside the buffer); masked
                    // lanes read that row's first element instead of their own
                    const int64_t roff = int64_t(rr) * ldd + colof(i);
#pragma unroll
                    for (int mt = 0; mt < NM; ++mt)
#pragma unroll
                        for (int q = 0; q < 4; ++q) vi[mt][q] = ldg0(dst, roff + 16 * mt + lg + 4 * q, valid);
#pragma unroll
                    for (int l = 0; l < GS; ++l) {
                        if (g0 + l < L) {
                            const double* blk = advance();
                            if (!act) continue;
#pragma unroll
                            for (int mt2 = 0; mt2 < NM; ++mt2)
#pragma unroll
                                for (int q = 0; q < 4; ++q) {
                                    const double bv = vi[mt2][q];
#pragma unroll
                                    for (int mt = 0; mt < NM; ++mt)
                                        acc[l][mt] = mfma(-blk[(16 * mt + lr) * (P + 2) + 16 * mt2 + lg + 4 * q], bv, acc[l][mt]);
                                }
                        }
                    }
                }
                // this group, right-looking
#pragma unroll
                for (int i = 0; i < GS; ++i) {
                    if (g0 + i < L) {
                        const int li = g0 + i;
                        const double* blk = advance();
                        v4d vi[NM];
                        if (act) {
#pragma unroll
                            for (int mt = 0; mt < NM; ++mt) {
                                v4d vn = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                                for (int mt2 = 0; mt2 <= mt; ++mt2)
#pragma unroll
                                    for (int q = 0; q < 4; ++q)
                                        vn = mfma(blk[(16 * mt + lr) * (P + 2) + 16 * mt2 + lg + 4 * q], acc[i][mt2][q], vn);
                                vi[mt] = vn;
                            }
                            if (store) {
                                double* d = drow + colof(li);
#pragma unroll
                                for (int mt = 0; mt < NM; ++mt)
#pragma unroll
                                    for (int q = 0; q < 4; ++q) d[16 * mt + lg + 4 * q] = vi[mt][q];
                            }
                        }
#pragma unroll
                        for (int l = i + 1; l < GS; ++l) {
                            if (g0 + l < L) {
                                const double* blk = advance();
                                if (!act) continue;
#pragma unroll
                                for (int mt2 = 0; mt2 < NM; ++mt2)
#pragma unroll
                                    for (int q = 0; q < 4; ++q) {
                                        const double bv = vi[mt2][q];
#pragma unroll
                                        for (int mt = 0; mt < NM; ++mt)
                                            acc[l][mt] = mfma(-blk[(16 * mt + lr) * (P + 2) + 16 * mt2 + lg + 4 * q], bv, acc[l][mt]);
                                    }
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
}

// ---- host-side launchers

int chain_lmax(int P) { (void)P; return MAXL - 1; }

// mode 0: knots of the regions of a.level; mode 1: observations of the
// level-(M-1) regions (a distinct kernel symbol, so that profilers report the
// two separately)
hipError_t launch_chain(const KArgs& a, int mode, int grid, hipStream_t st) {
    const int key = a.P * 2 + mode;
    switch (key) {
        case 32: hipLaunchKernelGGL((k_chain<16, 0>), dim3(grid), dim3(NT), 0, st, a); break;
        case 33: hipLaunchKernelGGL((k_chain<16, 1>), dim3(grid), dim3(NT), 0, st, a); break;
        case 64: hipLaunchKernelGGL((k_chain<32, 0>), dim3(grid), dim3(NT), 0, st, a); break;
        case 65: hipLaunchKernelGGL((k_chain<32, 1>), dim3(grid), dim3(NT), 0, st, a); break;
        case 128: hipLaunchKernelGGL((k_chain<64, 0>), dim3(grid), dim3(NT), 0, st, a); break;
        case 129: hipLaunchKernelGGL((k_chain<64, 1>), dim3(grid), dim3(NT), 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mra
