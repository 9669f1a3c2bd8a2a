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
// Device helpers shared by the kernel translation units of the MRA library
// (inline; included by mra_chain.hip, mra_finish.hip, mra_gram.hip,
// mra_pred.hip).
#pragma once
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

// The covariance at scaled distance t = |a - b| / range:
//   smooth 0: alpha e^{-t}                    (exponential, Matern 1/2)
//   smooth 1: alpha (1 + t) e^{-t}            (Matern 3/2)
//   smooth 2: alpha (1 + t + t^2 / 3) e^{-t}  (Matern 5/2)
//   smooth 3: alpha e^{-t^2}                  (Gaussian)
__device__ __forceinline__ double cov_t(double t, double alpha, int smooth) {
    if (smooth == 3) return alpha * exp(-t * t);
    const double e = exp(-t);
    if (smooth == 0) return alpha * e;
    if (smooth == 1) return alpha * (1.0 + t) * e;
    return alpha * ((1.0 + t) + (t * t) / 3.0) * e;
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

// ------------------------------------------------ finisher work queue

// The workgroup's next task: with a queue, the next ticket (every thread gets
// the same value; *tick is one int of LDS), else grid-stride from blockIdx.x.
// The barrier before the ticket keeps a fast thread from overwriting *tick
// while a slow one still reads the previous value.
__device__ __forceinline__ int64_t next_task(const KArgs& a, int64_t t, int* tick) {
    if (!a.queue) return t < 0 ? int64_t(blockIdx.x) : t + gridDim.x;
    __syncthreads();
    if (threadIdx.x == 0) *tick = __hip_atomic_fetch_add(a.queue, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(*tick);
}

// End of a queued launch: the last workgroup to finish sets both counters
// back to zero for the next launch on the stream.
__device__ __forceinline__ void queue_done(const KArgs& a) {
    if (!a.queue || threadIdx.x != 0) return;
    if (__hip_atomic_fetch_add(a.queue + 1, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == int(gridDim.x) - 1) {
        __hip_atomic_store(a.queue, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(a.queue + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Status of a theta whose representative's task gave up waiting (a bounded
// wait; not expected to happen, see the leaf finisher).
constexpr int STATUS_WAIT = -1;

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

// 1/sqrt(x) and sqrt(x) for x > 0: the hardware reciprocal-square-root
// estimate refined by two Newton steps (y <- y + y (1 - x y^2) / 2), then one
// Newton step for the square root (s <- s + (x - s^2) y / 2).
__device__ __forceinline__ void rsqrt_sqrt(double x, double& rs, double& sd) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    double s = x * y;
    s = fma(0.5 * y, fma(-s, s, x), s);
    rs = y;
    sd = s;
}

// Cholesky factor and its inverse of an n x n (n <= 16 NB) lower triangle held
// in a 16 NB x 16 NB LDS tile T (pitch ld > 16 NB), by one wave, with no
// workgroup barrier: on return T holds L^{-1} (lower, zeros above the
// diagonal, identity beyond n) where L L^T is the input, and *logdet = sum
// log diag L.  Returns true (uniformly) when a pivot is not positive.  Entries
// of T above the diagonal are neither read as data nor preserved; column
// 16 NB (the padding) is scratch.
// The tile is processed in 16 x 16 blocks, right-looking.  A diagonal block is
// factored in registers, lane r of every 16-lane group holding row r, each
// column of the factor broadcast by lane reads.  Entries right of the
// diagonal in a lane's row are carried along but never used (no per-lane
// conditions: they would be kept as lane masks).  The block is inverted by forward
// substitution, lane c solving for column c, with the reciprocal square roots
// of the pivots as the diagonal of the inverse.  The panel below is
// multiplied by that inverse and the trailing blocks are updated on the
// matrix cores.  The off-diagonal blocks of L^{-1} then follow block row by
// block row: X_ij = -D_i^{-1} sum_{k=j}^{i-1} L_ik X_kj with D_i^{-1} the
// diagonal inverses.  The pivots' product is kept as a mantissa and a binary
// exponent, so that one logarithm serves the whole tile.  PD bounds how many
// rows ahead the inverse's LDS reads may be issued (0: no bound; a caller
// whose registers allow it and whose LDS latency is high under load wants 0).
template <int NB, int PD = 2>
__device__ __forceinline__ bool wave_chol_inv(double* T, int ld, int n, double* logdet) {
    constexpr int NT16 = 16 * NB;
    const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    // identity beyond n (rows and columns), so that padding factors to itself
    for (int e = lane; e < NT16 * NT16; e += 64) {
        const int i = e / NT16, j = e % NT16;
        if ((i >= n || j >= n) && j <= i) T[i * ld + j] = (i == j) ? 1.0 : 0.0;
    }
    wsync();
    bool bad = false;
    double pp = 1.0;  // product of the pivots: mantissa pp, binary exponent pe
    int pe = 0;
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) {
        double* Dg = T + 16 * kb * ld + 16 * kb;
        // (1) factor the 16 x 16 diagonal block
        double d[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) d[k] = Dg[lr * ld + k];
        wsync();
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const double piv = bcast(d[j], j);
            bad = bad || !(piv > 0.0);
            const double pv = piv > 0.0 ? piv : 1.0;
            pp *= pv;
            if ((j & 3) == 3) {
                pe += __builtin_amdgcn_frexp_exp(pp);
                pp = __builtin_amdgcn_frexp_mant(pp);
            }
            double rs, sd;
            rsqrt_sqrt(pv, rs, sd);
            (void)sd;
            T[(16 * kb + j) * ld + 16 * NB] = rs;  // for the inverse
            // column j of the factor; on lane j the pivot times its reciprocal
            // square root, i.e. the diagonal entry
            const double lij = d[j] * rs;
            d[j] = lij;
#pragma unroll
            for (int k = j + 1; k < 16; ++k) d[k] = fma(-lij, bcast(lij, k), d[k]);
        }
        wsync();
#pragma unroll
        for (int k = 0; k < 16; ++k) Dg[lr * ld + k] = d[k];
        wsync();
        // (2) its inverse: entries above the diagonal come out zero, since
        // their right-hand side and every earlier entry of the column are
        double x[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            double acc = (q == lr) ? 1.0 : 0.0;
            // with PD > 0, row q is read once x[q - PD] exists: its offset
            // depends on x[q - PD] (one element further on for a NaN, which
            // only a failed factor produces; still inside row q), so that the
            // compiler does not load every row up front where registers are
            // short (they would spill)
            int off = q * ld;
            if (PD > 0 && q >= PD) off += (x[q - PD] != x[q - PD]) ? 1 : 0;
#pragma unroll
            for (int k = 0; k < q; ++k) acc = fma(-Dg[off + k], x[k], acc);
            x[q] = acc * T[(16 * kb + q) * ld + 16 * NB];
        }
        wsync();
        if (lg == 0) {
#pragma unroll
            for (int q = 0; q < 16; ++q) Dg[q * ld + lr] = x[q];
        }
        wsync();
        // (3) panel: L_ib = A_ib D^{-T} for the blocks below
#pragma unroll
        for (int ib = kb + 1; ib < NB; ++ib) {
            v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc = mfma(T[(16 * ib + lr) * ld + 16 * kb + 4 * q + lg], Dg[lr * ld + 4 * q + lg], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) T[(16 * ib + lg + 4 * i) * ld + 16 * kb + lr] = acc[i];
        }
        wsync();
        // (4) trailing blocks: A_ij -= L_ik L_jk^T
#pragma unroll
        for (int jb = kb + 1; jb < NB; ++jb)
#pragma unroll
            for (int ib = jb; ib < NB; ++ib) {
                v4d acc;
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[i] = T[(16 * ib + lg + 4 * i) * ld + 16 * jb + lr];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    acc = mfma(-T[(16 * ib + lr) * ld + 16 * kb + 4 * q + lg], T[(16 * jb + lr) * ld + 16 * kb + 4 * q + lg],
                               acc);
#pragma unroll
                for (int i = 0; i < 4; ++i) T[(16 * ib + lg + 4 * i) * ld + 16 * jb + lr] = acc[i];
            }
        wsync();
    }
    // (5) off-diagonal blocks of L^{-1}, block row by block row; the operands
    // of a block are loaded before its products
#pragma unroll
    for (int ib = 1; ib < NB; ++ib) {
        v4d z[NB > 1 ? NB - 1 : 1];
#pragma unroll
        for (int jb = 0; jb < ib; ++jb) {
            double av[NB][4], bv[NB][4], dv[4];
#pragma unroll
            for (int k = jb; k < ib; ++k)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    av[k][q] = T[(16 * ib + lr) * ld + 16 * k + 4 * q + lg];
                    bv[k][q] = T[(16 * k + 4 * q + lg) * ld + 16 * jb + lr];
                }
#pragma unroll
            for (int e = 0; e < 4; ++e) dv[e] = -T[(16 * ib + lr) * ld + 16 * ib + 4 * e + lg];
            v4d y0 = v4d{0.0, 0.0, 0.0, 0.0}, y1 = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = jb; k < ib; ++k)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (q & 1) y1 = mfma(av[k][q], bv[k][q], y1);
                    else y0 = mfma(av[k][q], bv[k][q], y0);
                }
            const v4d y = y0 + y1;
            v4d zz = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int e = 0; e < 4; ++e) zz = mfma(dv[e], y[e], zz);
            z[jb] = zz;
        }
        wsync();
#pragma unroll
        for (int jb = 0; jb < ib; ++jb)
#pragma unroll
            for (int i = 0; i < 4; ++i) T[(16 * ib + lg + 4 * i) * ld + 16 * jb + lr] = z[jb][i];
        wsync();
    }
    // zeros in the blocks above the diagonal
#pragma unroll
    for (int ib = 0; ib < NB; ++ib)
#pragma unroll
        for (int jb = ib + 1; jb < NB; ++jb)
#pragma unroll
            for (int i = 0; i < 4; ++i) T[(16 * ib + lg + 4 * i) * ld + 16 * jb + lr] = 0.0;
    wsync();
    *logdet = 0.5 * (log(pp) + double(pe) * 0.69314718055994530942);
    return bad;
}

__device__ __forceinline__ bool wave_chol_inv64(double* T, int ld, int n, double* logdet) {
    return wave_chol_inv<4>(T, ld, n, logdet);
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
    double mm[NT];  // reduction scratch
    double L[TB * MLD];
    double Li[TB * MLD];
    double kx[TB], ky[TB];
    int flag;
};

}  // namespace mra
