// HIP kernels of the MRA log-likelihood for gfx950 (FP64 throughout).
//
// Per chunk of covariance-parameter vectors theta, the host launches, in
// order (all regions of a level and all theta of the chunk in one launch):
//   level m = 1 .. M-1:
//     k_chain (knots)  : whitened prior rows of every level-m region's knots
//     k_prior_finish   : C_m(Q_R, Q_R), its Cholesky factor and that factor's
//                        inverse (the only thing descendants need of R)
//   k_chain (obs)      : whitened prior rows of every observation, one task
//                        per level-(M-1) region (its leaves share the path)
//   k_leaf_finish      : finest-level factors F = L_S^{-1} [V | z], d = log det S
//   level m = M-1 .. 1 : k_fold_factor / k_gram_panel + k_gram_tile (observation-space or
//                        knot-space fold of the children's statistics)
//   k_final            : log-likelihood per theta
// The recursion is the remainder-covariance recursion of Sec. 1.1 written in
// whitened form; its posterior statistics are the conditional (co)variances
// the paper keeps per region (ATilde, Sec. 4.2 / Appendix B).
//
// Dense contractions run on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and B[l/16][l%16]
// and holds D[l/16 + 4i][l%16], i = 0..3, of the 16x16 result).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "mra_internal.h"
#include "mra_kernels.h"

namespace mra {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

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

__device__ __forceinline__ void knot_xy(const KArgs& a, int64_t g, int i, double& kx, double& ky) {
    const double* b = a.box + 4 * g;
    kx = grid_bar(b[0], b[1], a.nx, a.offset, i % a.nx);
    ky = grid_bar(b[2], b[3], a.ny, a.offset, i / a.nx);
}

// Knots of region g into LDS arrays kx, ky (P entries; padded ones zero).
__device__ __forceinline__ void region_knots(const KArgs& a, int64_t g, double* kx, double* ky) {
    for (int i = threadIdx.x; i < a.P; i += NT) {
        double x = 0.0, y = 0.0;
        if (i < a.rhat) knot_xy(a, g, i, x, y);
        kx[i] = x;
        ky[i] = y;
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

__device__ __forceinline__ void flag_fail(const KArgs& a, int th, int64_t g) {
    if (threadIdx.x == 0) atomicCAS(a.status + th, 0, int(g + 1));
}

// ---------------------------------------------------- workgroup primitives

enum { MM_ADD = 0, MM_SUB = 1, MM_SET = 2 };
constexpr int MK = 32;       // K chunk of the workgroup GEMM
constexpr int MLD = TB + 1;  // LDS row pitch of the staged operands

// Branch-free guarded load: reads p[off] when ok, else p[0], and returns 0 for
// !ok.  Keeps masked loads unconditional so that batches of them are issued
// back to back instead of one round trip at a time.  p itself must always be
// a valid address (the start of the operand), never a per-lane pointer.
__device__ __forceinline__ double ldg0(const double* p, int64_t off, bool ok) {
    const double v = p[ok ? off : 0];
    return ok ? v : 0.0;
}

// C(r,c) (+= | -= | =) sum_k A(r,k) B(c,k) over r < R, c < N (c <= r when
// lower), A(r,k) = A[r*sar + k*sak], B(c,k) = B[c*sbc + k*sbk] (generic
// pointers: global or LDS), C row-major (ldc).  The output is cut into 64x64
// blocks dealt round-robin to the workgroup's waves; a wave computes its block
// with sixteen 16x16 MFMA accumulators, loading its A and B fragments straight
// from memory (L1/L2; no LDS staging and no barrier inside), 16 values of k
// per batch so that the loads of a batch are in flight together.  With MM_SET
// an output block may alias the operand columns it is computed from (each
// wave reads all of K for its block before writing it).  Ends with a
// workgroup barrier.
template <int MODE>
__device__ __forceinline__ void wg_mm(double* C, int64_t ldc, int R, int N, int K, const double* A, int64_t sar,
                                      int64_t sak, const double* B, int64_t sbc, int64_t sbk, bool lower,
                                      double* sm) {
    (void)sm;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 15, lg = lane >> 4;
    const int nbr = (R + TB - 1) / TB, nbc = (N + TB - 1) / TB;
    for (int b = w; b < nbr * nbc; b += NT / 64) {
        const int br = b / nbc, bc = b % nbc;
        const int r0 = br * TB, c0 = bc * TB;
        if (lower && c0 > r0 + TB - 1) continue;
        v4d acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
        // per-lane row / column of each 16-row tile
        bool rok[4], cok[4];
        const double* pa[4];
        const double* pb[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int r = r0 + 16 * t + lr, c = c0 + 16 * t + lr;
            rok[t] = r < R;
            cok[t] = c < N;
            pa[t] = A + (rok[t] ? int64_t(r) * sar : 0);
            pb[t] = B + (cok[t] ? int64_t(c) * sbc : 0);
        }
        for (int k0 = 0; k0 < K; k0 += 16) {
            double fa[4][4], fb[4][4];  // [tile][k-step]
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = k0 + 4 * q + lg;
                const bool kok = k < K;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const double va = *(rok[t] && kok ? pa[t] + int64_t(k) * sak : A);
                    const double vb = *(cok[t] && kok ? pb[t] + int64_t(k) * sbk : B);
                    fa[t][q] = (rok[t] && kok) ? va : 0.0;
                    fb[t][q] = (cok[t] && kok) ? vb : 0.0;
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (!lower || c0 + 16 * j <= r0 + 16 * i + 15) acc[i][j] = mfma(fa[i][q], fb[j][q], acc[i][j]);
        }
        // epilogue, one 16-row strip at a time: reads of C batched before writes
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double cold[4][4];
            if (MODE != MM_SET) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int r = r0 + 16 * i + lg + 4 * e, c = c0 + 16 * j + lr;
                        cold[j][e] = ldg0(C, int64_t(r) * ldc + c, r < R && c < N && (!lower || c <= r));
                    }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = r0 + 16 * i + lg + 4 * e, c = c0 + 16 * j + lr;
                    if (r < R && c < N && (!lower || c <= r)) {
                        double v = acc[i][j][e];
                        if (MODE == MM_ADD) v = cold[j][e] + v;
                        else if (MODE == MM_SUB) v = cold[j][e] - v;
                        C[int64_t(r) * ldc + c] = v;
                    }
                }
        }
    }
    __syncthreads();
}

// ------------------------------------------------- wave-level primitives
// A wavefront executes in lockstep and its LDS accesses complete in order;
// wsync() only keeps the compiler from moving LDS accesses across it.
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Value of v held by lane `src` (a compile-time constant after unrolling),
// broadcast to the whole wave through two scalar reads.
__device__ __forceinline__ double bcast(double v, int src) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(int(x), src);
    const int hi = __builtin_amdgcn_readlane(int(x >> 32), src);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// L^{-1} of an existing n x n (n <= NMAX) lower-triangular factor L in LDS,
// by one wave (lane j computes column j; rows of L broadcast from LDS).  Li
// may be L itself (the inverse then replaces the factor).
template <int NMAX>
__device__ __forceinline__ void trinv_rows(const double* L, int ld, double* Li, int64_t ld2, int n) {
    const int lane = threadIdx.x & 63;
    double x[NMAX];
#pragma unroll
    for (int q = 0; q < NMAX; ++q) {
        if (q < n) {
            double acc = (q == lane) ? 1.0 : 0.0;
#pragma unroll
            for (int k = 0; k < q; ++k) acc = fma(-L[q * ld + k], x[k], acc);
            x[q] = (q >= lane) ? acc / L[q * ld + q] : 0.0;
        } else {
            x[q] = 0.0;
        }
    }
    wsync();  // every read of L precedes the writes: Li may overwrite L
    if (lane < n) {
#pragma unroll
        for (int q = 0; q < NMAX; ++q)
            if (q < n) Li[int64_t(q) * ld2 + lane] = x[q];
    }
    wsync();
}

// Cholesky factor L of the n x n (n <= NMAX <= 64) lower triangle T (LDS, ld)
// and, if Li is given, L^{-1} (generic pointer, ld2), by one wave.  Lane i
// keeps row i in registers; column j of the factor is broadcast with scalar
// lane reads, so the right-looking update makes no LDS round trips.  L
// overwrites T (zero above the diagonal); Li receives the n x n lower
// triangle and zeros above it.  Returns true (uniformly) on a non-positive
// pivot.
template <int NMAX>
__device__ __forceinline__ bool wave_potrf_inv(double* T, int ld, double* Li, int64_t ld2, int n) {
    const int lane = threadIdx.x & 63;
    const int row = lane < NMAX ? lane : 0;
    double r[NMAX];
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
        const double v = T[row * ld + k];
        r[k] = (lane < n && k <= lane) ? v : 0.0;
    }
    bool bad = false;
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
        if (j < n) {
            const double piv = bcast(r[j], j);
            bad = bad || !(piv > 0.0);
            const double d = sqrt(piv > 0.0 ? piv : 1.0);
            const double lij = (lane > j) ? r[j] / d : (lane == j ? d : 0.0);
            r[j] = lij;
#pragma unroll
            for (int k = j + 1; k < NMAX; ++k)
                if (k < n) r[k] = fma(-lij, bcast(lij, k), r[k]);
        }
    }
    if (lane < n) {
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
            if (k < n) T[lane * ld + k] = (k <= lane) ? r[k] : 0.0;
    }
    wsync();
    // column `lane` of L^{-1}, rows of L read back from LDS (broadcast)
    if (Li) trinv_rows<NMAX>(T, ld, Li, ld2, n);
    wsync();
    return bad;
}

// Cholesky factor (in place) and inverse of an n x n (n <= 64) lower triangle
// held in LDS, by wave 0 while the others wait.  Li (LDS, 64 x 64 tile)
// receives L^{-1} padded with zeros.  Returns true in every thread when a
// pivot is not positive (the factor is then garbage).
__device__ __forceinline__ bool wg_potrf_inv_lds(double* T, int n, int ld, double* Li, int ld2, int* flag) {
    for (int e = threadIdx.x; e < TB * TB; e += NT) Li[(e / TB) * ld2 + (e % TB)] = 0.0;
    __syncthreads();
    if ((threadIdx.x >> 6) == 0) {
        const bool bad = wave_potrf_inv<TB>(T, ld, Li, ld2, n);
        if (threadIdx.x == 0) *flag = bad ? 1 : 0;
    }
    __syncthreads();
    const bool bad = *flag != 0;
    __syncthreads();
    return bad;
}

// Load an n x n lower triangle (generic pointer, ldg) into LDS (ld), zero
// elsewhere in the 64 x 64 tile.  All loads of a thread are issued first.
__device__ __forceinline__ void load_tile(double* T, int ld, const double* G, int64_t ldg, int n) {
    constexpr int PER = TB * TB / NT;
    double v[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int e = threadIdx.x + j * NT, i = e / TB, c = e % TB;
        v[j] = ldg0(G, int64_t(i) * ldg + c, i < n && c <= i);
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int e = threadIdx.x + j * NT;
        T[(e / TB) * ld + (e % TB)] = v[j];
    }
    __syncthreads();
}

__device__ __forceinline__ void store_tile(double* G, int64_t ldg, const double* T, int ld, int n) {
    for (int e = threadIdx.x; e < n * n; e += NT) {
        const int i = e / n, j = e % n;
        G[int64_t(i) * ldg + j] = (j <= i) ? T[i * ld + j] : 0.0;
    }
    __syncthreads();
}

// Blocked right-looking Cholesky of an n x n lower triangle (generic pointer,
// lda).  Diagonal blocks are factored and inverted in LDS; panels are solved
// as products with the inverted block.  *logdet (all threads) = sum log diag.
// For n <= 64, Li holds L^{-1} on return.
__device__ __forceinline__ bool wg_potrf(double* A, int64_t lda, int n, double* Ls, double* Li, double* sm,
                                         int* flag, double* logdet, double* Lst = nullptr) {
    double acc = 0.0;
    for (int j0 = 0; j0 < n; j0 += TB) {
        const int jb = min(TB, n - j0);
        double* Ajj = A + int64_t(j0) * lda + j0;
        load_tile(Ls, MLD, Ajj, lda, jb);
        if (wg_potrf_inv_lds(Ls, jb, MLD, Li, MLD, flag)) return true;
        // keep the block's inverse for a later triangular solve
        if (Lst)
            for (int e = threadIdx.x; e < TB * TB; e += NT) Lst[int64_t(j0 / TB) * TB * TB + e] = Li[(e / TB) * MLD + (e % TB)];
        store_tile(Ajj, lda, Ls, MLD, jb);
        for (int i = 0; i < jb; ++i) acc += log(Ls[i * MLD + i]);
        const int rest = n - j0 - jb;
        if (rest > 0) {
            double* Aij = A + int64_t(j0 + jb) * lda + j0;
            // panel: A_ij <- A_ij L_jj^{-T}
            wg_mm<MM_SET>(Aij, lda, rest, jb, jb, Aij, lda, 1, Li, MLD, 1, false, sm);
            // trailing update (lower)
            wg_mm<MM_SUB>(A + int64_t(j0 + jb) * lda + j0 + jb, lda, rest, rest, jb, Aij, lda, 1, Aij, lda, 1,
                          true, sm);
        }
    }
    *logdet = acc;
    return false;
}

// X (n x W, ldx) <- L^{-1} X with L (n x n lower, generic pointer, ldl).
// Diagonal blocks are inverted in LDS and applied as products; with n <= 64
// and have_inv the inverse already in Li is used.
__device__ __forceinline__ void wg_trsm_lln(const double* L, int64_t ldl, int n, double* X, int64_t ldx, int W,
                                            double* Ls, double* Li, double* sm, int* flag, bool have_inv,
                                            const double* Lst = nullptr) {
    for (int i0 = 0; i0 < n; i0 += TB) {
        const int ib = min(TB, n - i0);
        if (Lst && n > TB) {
            // the diagonal blocks' inverses kept by wg_potrf
            for (int e = threadIdx.x; e < TB * TB; e += NT) Li[(e / TB) * MLD + (e % TB)] = Lst[int64_t(i0 / TB) * TB * TB + e];
            __syncthreads();
        } else if (!(have_inv && n <= TB)) {
            load_tile(Ls, MLD, L + int64_t(i0) * ldl + i0, ldl, ib);
            // the block is already a factor: its Cholesky factor is itself up to
            // rounding of the diagonal; take the inverse of the stored factor
            for (int e = threadIdx.x; e < TB * TB; e += NT) Li[(e / TB) * MLD + (e % TB)] = 0.0;
            __syncthreads();
            if ((threadIdx.x >> 6) == 0) trinv_rows<TB>(Ls, MLD, Li, MLD, ib);
            __syncthreads();
        }
        double* Xi = X + int64_t(i0) * ldx;
        // X_i <- Li X_i : C(r, c) = sum_k Li(r, k) X_i(k, c)
        wg_mm<MM_SET>(Xi, ldx, ib, W, ib, Li, MLD, 1, Xi, 1, ldx, false, sm);
        const int rest = n - i0 - ib;
        if (rest > 0)
            wg_mm<MM_SUB>(X + int64_t(i0 + ib) * ldx, ldx, rest, W, ib, L + int64_t(i0 + ib) * ldl + i0, ldl, 1,
                          Xi, 1, ldx, false, sm);
    }
    (void)flag;
}

// ------------------------------------------------------------------ kernels

struct Smem {
    double mm[NT];  // reduction scratch (wg_rowvec)
    double L[TB * MLD];
    double Li[TB * MLD];
    double kx[TB], ky[TB];
    int flag;
};

// Whitened prior rows.  mode 0: the r_hat knots of every level-m region
// (a.level = m) for ancestors 1..m-1, written into the region's V store
// (row-major P x mP, block i-1 = V^i).  mode 1: every observation under a
// level-(M-1) region for ancestors 1..M-1, written into the F buffer (block of
// level l at columns (M-1-l)P).  For ancestor level l, with C the covariance:
//     V^l = ( C(rows, Q_{A_l}) - sum_{i<l} V^i V^i(Q_{A_l})^T ) L_{A_l}^{-T}.
// Each wave owns 16 rows.  Ancestor levels are taken in groups of GS = 128/P:
// one pending accumulator per level of the group (MFMA destinations, knots x
// rows) receives the covariance, the contributions of all earlier groups (their
// V rows read back from memory) and, right-looking, those of the group's own
// earlier levels.  A V^i in accumulator layout serves directly as the B
// operand: the summation index is permuted consistently on the A operand,
// which is staged in LDS one P x P block at a time.
// Staging of a P x P block (row-major, ld; rows 16-byte aligned) into LDS,
// transposed with an odd pitch: blk[c * (P + 1) + r] = src[r][c], so that the
// 16 lanes of a group, which read 16 consecutive rows r of one column c, hit
// 16 different banks.  Split in two for software pipelining: the loads of the
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
            blk[c * (P + 1) + r] = rg.v[j].x;
            blk[(c + 1) * (P + 1) + r] = rg.v[j].y;
        }
    }
}

template <int P, int mode>
__global__ void __launch_bounds__(NT, 2) k_chain(KArgs a) {
    constexpr int NM = P / 16;
    constexpr int GS = 128 / P;  // accumulator budget for two workgroups per CU
    // two staging buffers: block s is written while block s - 1 may still be
    // read, so one barrier per block suffices
    __shared__ double blk2[2][P * (P + 1)];
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
    const int m = mode == 0 ? a.level : a.M - 1;  // level of the task region
    const int L = mode == 0 ? m - 1 : a.M - 1;    // ancestor levels of the rows
    int ph = 0;  // staging buffer parity, continued across tiles and tasks
    for (int q = threadIdx.x; q < P; q += NT) kq[q] = q < a.rhat ? (q % a.nx) + 8 * (q / a.nx) : -1;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        const int th = int(t / a.ntasks);
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
                                        acc[l][mt] = mfma(-blk[(16 * mt2 + lg + 4 * q) * (P + 1) + 16 * mt + lr], bv, acc[l][mt]);
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
                                        vn = mfma(blk[(16 * mt2 + lg + 4 * q) * (P + 1) + 16 * mt + lr], acc[i][mt2][q], vn);
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
                                            acc[l][mt] = mfma(-blk[(16 * mt2 + lg + 4 * q) * (P + 1) + 16 * mt + lr], bv, acc[l][mt]);
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

// y[c] (=|+=) sum_k u(k) v(k, c) for c < N, u(k) = U[k su], v(k, c) = V[k sv + c].
// Lanes take 64 consecutive columns; the four waves take interleaved slices
// of 8 rows, each lane keeping 8 independent partial sums so that 16 loads
// are in flight; the partials are combined in a fixed order (deterministic).
// red: 4 x 64 doubles of LDS.
template <bool ADD>
__device__ __forceinline__ void wg_rowvec(double* y, int N, int K, const double* U, int64_t su, const double* V,
                                          int64_t sv, double* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int c0 = 0; c0 < N; c0 += 64) {
        const int c = c0 + lane;
        const bool ok = c < N;
        double p[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) p[u] = 0.0;
        for (int k = 8 * w; k < K; k += 32) {
            double uv[8], vv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool kok = k + u < K;
                uv[u] = ldg0(U, int64_t(k + u) * su, kok);
                vv[u] = ldg0(V, int64_t(k + u) * sv + c, kok && ok);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) p[u] = fma(uv[u], vv[u], p[u]);
        }
        red[w * 64 + lane] = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
        __syncthreads();
        if (w == 0 && ok) {
            const double v = (red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane]);
            y[c] = ADD ? y[c] + v : v;
        }
        __syncthreads();
    }
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
                if (first) {
                    wg_mm<MM_SET>(G, D, D, P, nc, Fc, 1, a.WFs, Fc, 1, a.WFs, false, s.mm);
                    wg_rowvec<false>(yrow, Dt, nc, Fc + (D - 1), a.WFs, Fc + P, a.WFs, s.mm);
                } else {
                    wg_mm<MM_ADD>(G, D, D, P, nc, Fc, 1, a.WFs, Fc, 1, a.WFs, false, s.mm);
                    wg_rowvec<true>(yrow, Dt, nc, Fc + (D - 1), a.WFs, Fc + P, a.WFs, s.mm);
                }
                first = false;
            } else {
                ++j;
                const double* Gc = a.gram + th * a.gram_stride + a.gram_off[gc];
                const int Dc = D + P;
                // panel: G[i][c] for i < D, c < P (lower part of the top block only)
                for (int64_t e = threadIdx.x; e < int64_t(D) * P; e += NT) {
                    const int i = int(e / P), c = int(e % P);
                    if (c <= i) {
                        const double v = Gc[int64_t(P + i) * Dc + P + c];
                        G[int64_t(i) * D + c] = first ? v : G[int64_t(i) * D + c] + v;
                    }
                }
                for (int c = threadIdx.x; c < Dt; c += NT) {
                    const double v = Gc[int64_t(P + D - 1) * Dc + P + P + c];
                    yrow[c] = first ? v : yrow[c] + v;
                }
                __syncthreads();
                first = false;
            }
        }
        // I + G[0:P, 0:P] -> Cholesky factor and inverse in LDS
        for (int e = threadIdx.x; e < TB * TB; e += NT) {
            const int i = e / TB, j = e % TB;
            s.L[i * MLD + j] = (i < P && j <= i) ? G[int64_t(i) * D + j] + (i == j ? 1.0 : 0.0) : 0.0;
        }
        __syncthreads();
        if (wg_potrf_inv_lds(s.L, P, MLD, s.Li, MLD, &s.flag)) {
            flag_fail(a, th, g);
            continue;
        }
        if (threadIdx.x == 0) {
            double ld = 0.0;
            for (int i = 0; i < P; ++i) ld += log(s.L[i * MLD + i]);
            a.dval[th * a.d_stride + g] = 2.0 * ld;
        }
        for (int e = threadIdx.x; e < P * P; e += NT) {
            const int i = e / P, j = e % P;
            G[int64_t(i) * D + j] = (j <= i) ? s.Li[i * MLD + j] : 0.0;
        }
        // Z = G[P:D, 0:P] L^{-T} in place
        double* Z = G + int64_t(P) * D;
        wg_mm<MM_SET>(Z, D, Dt, P, P, Z, D, 1, s.Li, MLD, 1, false, s.mm);
        // last row of S: yrow[c] -= Z[Dt-1] . Z[c]; lanes over the P columns
        // of Z (coalesced rows), one row c per wave step, butterfly sum
        {
            const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
            const double zy = lane < P ? Z[int64_t(Dt - 1) * D + lane] : 0.0;
            for (int c = w; c < Dt; c += NT / 64) {
                double v = lane < P ? zy * Z[int64_t(c) * D + lane] : 0.0;
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
                if (lane == 0) yrow[c] -= v;
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
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
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
        const bool active = !(BI == BJ && wc > wr);      // quarters above the diagonal are skipped
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

// ------------------------------------------------------- host-side launchers

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
