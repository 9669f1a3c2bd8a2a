// Learned surrogate of the MRA log-likelihood: a 3 -> 4 x 128 (SiLU) -> 1
// network in FP32 with its own forward, backward and Adam kernels on gfx950.
// The shapes, the loss and the update are stated in include/mra_mlp.h.
//
// Every dense step is one launch of a 64 x 64-tiled FP32 GEMM whose operands
// are addressed through strides, so the transposes of the backward pass need
// no copies; its epilogue adds the bias and applies SiLU (forward) or
// multiplies by SiLU' of the layer below (backward).  Sums over the batch
// (bias gradients, the loss) run in one workgroup per output with a fixed
// reduction order, so every result is reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "../../include/mra.h"
#include "../../include/mra_mlp.h"
#include "mra_internal.h"

namespace {

constexpr int W = MRA_MLP_WIDTH;
constexpr int NIN = 3;
constexpr int NHID = 4;
// offsets into the parameter vector
constexpr int64_t OFF_W1 = 0;
constexpr int64_t OFF_B1 = OFF_W1 + W * NIN;
constexpr int64_t OFF_W(int l) { return OFF_B1 + W + int64_t(l - 2) * (W * W + W); }  // l = 2..4
constexpr int64_t OFF_B(int l) { return OFF_W(l) + W * W; }
constexpr int64_t OFF_W5 = OFF_B(4) + W;
constexpr int64_t OFF_B5 = OFF_W5 + W;
constexpr int64_t NPARAM = OFF_B5 + 1;
static_assert(NPARAM == MRA_MLP_NPARAM, "parameter count");

constexpr int GT = 64;   // GEMM output tile
constexpr int GK = 16;   // K chunk
constexpr int GNT = 256; // threads

enum { EPI_PLAIN = 0, EPI_SILU = 1, EPI_DSILU = 2 };

struct Gemm {
    const float* A; int64_t sai, sak;  // A(i, k) = A[i sai + k sak]
    const float* B; int64_t sbk, sbj;  // B(k, j) = B[k sbk + j sbj]
    float* C; int64_t ldc;             // C[i ldc + j]
    int M, N, K;
    const float* bias;                 // [N] or null
    float* H;                          // EPI_SILU: silu(C) written here (ld ldc)
    const float* Zp;                   // EPI_DSILU: C *= silu'(Zp) (ld ldc)
    int epi;
};

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + expf(-z)); }

__global__ void __launch_bounds__(GNT) k_gemm(Gemm g) {
    __shared__ float As[GK][GT + 4];
    __shared__ float Bs[GK][GT + 4];
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
    float acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0f;
    for (int k0 = 0; k0 < g.K; k0 += GK) {
        // A chunk: 64 rows x 16 k; B chunk: 16 k x 64 columns; 4 elements per thread each
        float av[4], bv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * GNT;          // 0 .. 1023
            const int ai = e / GK, ak = e % GK;   // A: row-of-tile, k
            const int bk = e / GT, bj = e % GT;   // B: k, column-of-tile
            const int gi = i0 + ai, gk = k0 + ak, gk2 = k0 + bk, gj = j0 + bj;
            av[q] = (gi < g.M && gk < g.K) ? g.A[gi * g.sai + gk * g.sak] : 0.0f;
            bv[q] = (gk2 < g.K && gj < g.N) ? g.B[gk2 * g.sbk + gj * g.sbj] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * GNT;
            As[e % GK][e / GK] = av[q];
            Bs[e / GT][e % GT] = bv[q];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = As[kk][ty * 4 + r];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx * 4 + c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = fmaf(a[r], b[c], acc[r][c]);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = i0 + ty * 4 + r;
        if (i >= g.M) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int j = j0 + tx * 4 + c;
            if (j >= g.N) continue;
            float v = acc[r][c];
            if (g.bias) v += g.bias[j];
            const int64_t o = int64_t(i) * g.ldc + j;
            if (g.epi == EPI_DSILU) {
                const float z = g.Zp[o], s = sigm(z);
                v *= s * (1.0f + z * (1.0f - s));
            }
            g.C[o] = v;
            if (g.epi == EPI_SILU) g.H[o] = v * sigm(v);
        }
    }
}

// u = 2 (x - lo) / (hi - lo) - 1 per input column
__global__ void k_prep(const float* x, int64_t B, float* u, float l0, float l1, float l2, float s0, float s1,
                       float s2) {
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < B * NIN; e += int64_t(gridDim.x) * blockDim.x) {
        const int c = int(e % NIN);
        const float lo = c == 0 ? l0 : (c == 1 ? l1 : l2);
        const float sc = c == 0 ? s0 : (c == 1 ? s1 : s2);
        u[e] = (x[e] - lo) * sc - 1.0f;
    }
}

__global__ void k_out(const float* s, int64_t B, double ymean, double ystd, double* y) {
    for (int64_t b = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; b < B; b += int64_t(gridDim.x) * blockDim.x)
        y[b] = ymean + ystd * double(s[b]);
}

// loss (FP64 accumulation, fixed order) and dL/ds = 2 (s - t) / B
__global__ void __launch_bounds__(256) k_loss(const float* s, const double* y, int64_t B, double ymean, double ystd,
                                              float* dout, double* loss) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t b = threadIdx.x; b < B; b += 256) {
        const double t = (y[b] - ymean) / ystd;
        const double d = double(s[b]) - t;
        dout[b] = float(2.0 * d / double(B));
        acc += d * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) *loss = red[0] / double(B);
}

// out[j] = sum_i X[i ld + j] over i < M, one workgroup per column (FP64 accumulation)
__global__ void __launch_bounds__(256) k_colsum(const float* X, int64_t M, int64_t ld, float* out) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < M; i += 256) acc += double(X[i * ld + j]);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = float(red[0]);
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
        const float ge = g[e];
        const float me = b1 * m[e] + (1.0f - b1) * ge;
        const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
        m[e] = me;
        v[e] = ve;
        p[e] -= lr * (me * c1) / (sqrtf(ve * c2) + eps);
    }
}

hipError_t gemm(const Gemm& g, hipStream_t st) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    dim3 grid((g.N + GT - 1) / GT, (g.M + GT - 1) / GT);
    hipLaunchKernelGGL(k_gemm, grid, dim3(GNT), 0, st, g);
    return hipGetLastError();
}

Gemm mk(const float* A, int64_t sai, int64_t sak, const float* B, int64_t sbk, int64_t sbj, float* C, int64_t ldc,
        int M, int N, int K) {
    Gemm g{};
    g.A = A; g.sai = sai; g.sak = sak;
    g.B = B; g.sbk = sbk; g.sbj = sbj;
    g.C = C; g.ldc = ldc;
    g.M = M; g.N = N; g.K = K;
    g.epi = EPI_PLAIN;
    return g;
}

int grid1(int64_t n) { return int(std::min<int64_t>((n + 255) / 256, 4096)); }

}  // namespace

struct mra_mlp {
    float* p = nullptr;      // parameters
    float* g = nullptr;      // gradient
    float* m = nullptr;      // Adam first moment
    float* v = nullptr;      // Adam second moment
    int64_t step = 0;
    double xlo[3] = {-1, -1, -1}, xhi[3] = {1, 1, 1};
    double ymean = 0.0, ystd = 1.0;
    // batch workspace
    int64_t cap = 0;
    float *u = nullptr, *Z = nullptr, *H = nullptr, *D0 = nullptr, *D1 = nullptr, *s = nullptr, *ds = nullptr;
    float* xs = nullptr;     // device copy of host inputs
    double *ys = nullptr, *yo = nullptr, *lossd = nullptr;
    void release_ws() {
        for (void* q : {static_cast<void*>(u), static_cast<void*>(Z), static_cast<void*>(H), static_cast<void*>(D0),
                        static_cast<void*>(D1), static_cast<void*>(s), static_cast<void*>(ds), static_cast<void*>(xs),
                        static_cast<void*>(ys), static_cast<void*>(yo), static_cast<void*>(lossd)})
            if (q) (void)hipFree(q);
        u = Z = H = D0 = D1 = s = ds = xs = nullptr;
        ys = yo = lossd = nullptr;
        cap = 0;
    }
    ~mra_mlp() {
        release_ws();
        for (void* q : {static_cast<void*>(p), static_cast<void*>(g), static_cast<void*>(m), static_cast<void*>(v)})
            if (q) (void)hipFree(q);
    }
};

namespace {

// Workspace for batches of up to B rows (activations of all hidden layers are
// kept for the backward pass).
int ensure(mra_mlp* n, int64_t B) {
    if (B <= n->cap) return MRA_OK;
    n->release_ws();
    const size_t act = size_t(B) * W * sizeof(float);
    auto al = [](void** q, size_t bytes) { return hipMalloc(q, std::max<size_t>(bytes, 16)) == hipSuccess; };
    if (!al(reinterpret_cast<void**>(&n->u), size_t(B) * NIN * 4) || !al(reinterpret_cast<void**>(&n->Z), act * NHID) ||
        !al(reinterpret_cast<void**>(&n->H), act * NHID) || !al(reinterpret_cast<void**>(&n->D0), act) ||
        !al(reinterpret_cast<void**>(&n->D1), act) || !al(reinterpret_cast<void**>(&n->s), size_t(B) * 4) ||
        !al(reinterpret_cast<void**>(&n->ds), size_t(B) * 4) || !al(reinterpret_cast<void**>(&n->xs), size_t(B) * NIN * 4) ||
        !al(reinterpret_cast<void**>(&n->ys), size_t(B) * 8) || !al(reinterpret_cast<void**>(&n->yo), size_t(B) * 8) ||
        !al(reinterpret_cast<void**>(&n->lossd), 8)) {
        (void)hipGetLastError();
        n->release_ws();
        return mra::fail(MRA_ENOMEM, "device allocation of the network workspace failed");
    }
    n->cap = B;
    return MRA_OK;
}

// forward over B rows of device input x: activations into n->Z / n->H, output s
hipError_t forward(mra_mlp* n, const float* x, int64_t B, hipStream_t st) {
    const int Bi = int(B);
    float sc[3], lo[3];
    for (int c = 0; c < 3; ++c) {
        lo[c] = float(n->xlo[c]);
        sc[c] = float(2.0 / (n->xhi[c] - n->xlo[c]));
    }
    hipLaunchKernelGGL(k_prep, dim3(grid1(B * NIN)), dim3(256), 0, st, x, B, n->u, lo[0], lo[1], lo[2], sc[0], sc[1],
                       sc[2]);
    hipError_t e = hipGetLastError();
    if (e) return e;
    const int64_t act = B * W;
    // layer 1: Z1 = u W1^T + b1
    Gemm g = mk(n->u, NIN, 1, n->p + OFF_W1, 1, NIN, n->Z, W, Bi, W, NIN);
    g.bias = n->p + OFF_B1; g.epi = EPI_SILU; g.H = n->H;
    if ((e = gemm(g, st))) return e;
    for (int l = 2; l <= NHID; ++l) {
        g = mk(n->H + (l - 2) * act, W, 1, n->p + OFF_W(l), 1, W, n->Z + (l - 1) * act, W, Bi, W, W);
        g.bias = n->p + OFF_B(l); g.epi = EPI_SILU; g.H = n->H + (l - 1) * act;
        if ((e = gemm(g, st))) return e;
    }
    g = mk(n->H + (NHID - 1) * act, W, 1, n->p + OFF_W5, 1, 0, n->s, 1, Bi, 1, W);
    g.bias = n->p + OFF_B5;
    return gemm(g, st);
}

// gradient of the loss into n->g (forward must have run on the same batch;
// n->ds holds dL/ds)
hipError_t backward(mra_mlp* n, int64_t B, hipStream_t st) {
    const int Bi = int(B);
    const int64_t act = B * W;
    hipError_t e;
    // output layer: g_w5 = ds^T H4, g_b5 = sum ds
    Gemm g = mk(n->ds, 0, 1, n->H + (NHID - 1) * act, W, 1, n->g + OFF_W5, W, 1, W, Bi);
    if ((e = gemm(g, st))) return e;
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, st, n->ds, B, int64_t(1), n->g + OFF_B5);
    if ((e = hipGetLastError())) return e;
    // dZ4 = (ds w5^T) * silu'(Z4)
    float* dz = n->D0;
    float* dz_next = n->D1;
    g = mk(n->ds, 1, 0, n->p + OFF_W5, 0, 1, dz, W, Bi, W, 1);
    g.epi = EPI_DSILU; g.Zp = n->Z + (NHID - 1) * act;
    if ((e = gemm(g, st))) return e;
    for (int l = NHID; l >= 2; --l) {
        // g_Wl = dZl^T H_{l-1};  g_bl = column sums of dZl
        g = mk(dz, 1, W, n->H + (l - 2) * act, W, 1, n->g + OFF_W(l), W, W, W, Bi);
        if ((e = gemm(g, st))) return e;
        hipLaunchKernelGGL(k_colsum, dim3(W), dim3(256), 0, st, dz, B, int64_t(W), n->g + OFF_B(l));
        if ((e = hipGetLastError())) return e;
        // dZ_{l-1} = (dZl Wl) * silu'(Z_{l-1})
        g = mk(dz, W, 1, n->p + OFF_W(l), W, 1, dz_next, W, Bi, W, W);
        g.epi = EPI_DSILU; g.Zp = n->Z + (l - 2) * act;
        if ((e = gemm(g, st))) return e;
        std::swap(dz, dz_next);
    }
    // layer 1: g_W1 = dZ1^T u;  g_b1 = column sums of dZ1
    g = mk(dz, 1, W, n->u, NIN, 1, n->g + OFF_W1, NIN, W, NIN, Bi);
    if ((e = gemm(g, st))) return e;
    hipLaunchKernelGGL(k_colsum, dim3(W), dim3(256), 0, st, dz, B, int64_t(W), n->g + OFF_B1);
    return hipGetLastError();
}

#define MLPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return mra::fail(MRA_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

// Inputs of a training call on the device: x (B x 3) and y (B).
int stage_inputs(mra_mlp* n, const float* x, const double* y, int64_t B, bool dev, hipStream_t st,
                 const float** dx, const double** dy) {
    if (dev) {
        *dx = x;
        *dy = y;
        return MRA_OK;
    }
    MLPCHK(hipMemcpyAsync(n->xs, x, size_t(B) * NIN * 4, hipMemcpyHostToDevice, st));
    if (y) MLPCHK(hipMemcpyAsync(n->ys, y, size_t(B) * 8, hipMemcpyHostToDevice, st));
    *dx = n->xs;
    *dy = n->ys;
    return MRA_OK;
}

int loss_and_grad(mra_mlp* n, const float* x, const double* y, int64_t B, double* loss, bool dev, hipStream_t st) {
    const float* dx;
    const double* dy;
    int rc = stage_inputs(n, x, y, B, dev, st, &dx, &dy);
    if (rc) return rc;
    MLPCHK(forward(n, dx, B, st));
    double* dl = dev ? loss : n->lossd;
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, st, n->s, dy, B, n->ymean, n->ystd, n->ds, dl);
    MLPCHK(hipGetLastError());
    MLPCHK(backward(n, B, st));
    return MRA_OK;
}

}  // namespace

extern "C" int mra_mlp_create(const float* params, mra_mlp** out) {
    if (!out || !params) return mra::fail(MRA_EINVAL, "NULL argument");
    *out = nullptr;
    int rc = mra::check_device();
    if (rc) return rc;
    auto* n = new mra_mlp();
    const size_t bytes = NPARAM * sizeof(float);
    if (hipMalloc(&n->p, bytes) != hipSuccess || hipMalloc(&n->g, bytes) != hipSuccess ||
        hipMalloc(&n->m, bytes) != hipSuccess || hipMalloc(&n->v, bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete n;
        return mra::fail(MRA_ENOMEM, "device allocation of the network failed");
    }
    if (hipMemcpy(n->p, params, bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(n->g, 0, bytes) != hipSuccess || hipMemset(n->m, 0, bytes) != hipSuccess ||
        hipMemset(n->v, 0, bytes) != hipSuccess) {
        delete n;
        return mra::fail(MRA_EDEVICE, "initialising the network failed");
    }
    *out = n;
    return MRA_OK;
}

extern "C" int mra_mlp_set_scaling(mra_mlp* n, const double* x_lo, const double* x_hi, double y_mean, double y_std) {
    if (!n || !x_lo || !x_hi) return mra::fail(MRA_EINVAL, "NULL argument");
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(x_lo[c]) || !std::isfinite(x_hi[c]) || !(x_hi[c] > x_lo[c]))
            return mra::fail(MRA_EINVAL, "x_hi must exceed x_lo (finite)");
    if (!std::isfinite(y_mean) || !std::isfinite(y_std) || !(y_std > 0.0))
        return mra::fail(MRA_EINVAL, "y_std must be > 0 and y_mean finite");
    for (int c = 0; c < 3; ++c) { n->xlo[c] = x_lo[c]; n->xhi[c] = x_hi[c]; }
    n->ymean = y_mean;
    n->ystd = y_std;
    return MRA_OK;
}

extern "C" int mra_mlp_forward(mra_mlp* n, const float* x, int64_t B, double* y, void* stream) {
    if (!n || B < 0 || (B > 0 && (!x || !y))) return mra::fail(MRA_EINVAL, "NULL argument or B < 0");
    if (B == 0) return MRA_OK;
    const bool dev = mra::is_device_ptr(x);
    if (dev != mra::is_device_ptr(y)) return mra::fail(MRA_EINVAL, "x and y must be in the same memory space");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t chunk = 1 << 16;
    int rc = ensure(n, std::min(B, chunk));
    if (rc) return rc;
    for (int64_t b0 = 0; b0 < B; b0 += chunk) {
        const int64_t nb = std::min(chunk, B - b0);
        const float* dx = x + b0 * NIN;
        if (!dev) {
            MLPCHK(hipMemcpyAsync(n->xs, dx, size_t(nb) * NIN * 4, hipMemcpyHostToDevice, st));
            dx = n->xs;
        }
        MLPCHK(forward(n, dx, nb, st));
        double* dy = dev ? y + b0 : n->yo;
        hipLaunchKernelGGL(k_out, dim3(grid1(nb)), dim3(256), 0, st, n->s, nb, n->ymean, n->ystd, dy);
        MLPCHK(hipGetLastError());
        if (!dev) {
            MLPCHK(hipMemcpyAsync(y + b0, n->yo, size_t(nb) * 8, hipMemcpyDeviceToHost, st));
            MLPCHK(hipStreamSynchronize(st));
        }
    }
    return MRA_OK;
}

extern "C" int mra_mlp_loss_grad(mra_mlp* n, const float* x, const double* y, int64_t B, float* grad, double* loss,
                                 void* stream) {
    if (!n || !x || !y || B <= 0) return mra::fail(MRA_EINVAL, "NULL argument or B <= 0");
    if (B > (int64_t(1) << 20)) return mra::fail(MRA_EINVAL, "training batches hold at most 2^20 rows");
    const bool dev = mra::is_device_ptr(x);
    if (dev != mra::is_device_ptr(y) || (grad && dev != mra::is_device_ptr(grad)) ||
        (loss && dev != mra::is_device_ptr(loss)))
        return mra::fail(MRA_EINVAL, "x, y, grad and loss must be in the same memory space");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int rc = ensure(n, B);
    if (rc) return rc;
    if ((rc = loss_and_grad(n, x, y, B, loss, dev, st))) return rc;
    if (grad) MLPCHK(hipMemcpyAsync(grad, n->g, NPARAM * sizeof(float), dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    if (!dev) {
        if (loss) MLPCHK(hipMemcpyAsync(loss, n->lossd, 8, hipMemcpyDeviceToHost, st));
        MLPCHK(hipStreamSynchronize(st));
    }
    return MRA_OK;
}

extern "C" int mra_mlp_train_step(mra_mlp* n, const float* x, const double* y, int64_t B, float lr, float beta1,
                                  float beta2, float eps, double* loss, void* stream) {
    if (!n || !x || !y || B <= 0) return mra::fail(MRA_EINVAL, "NULL argument or B <= 0");
    if (B > (int64_t(1) << 20)) return mra::fail(MRA_EINVAL, "training batches hold at most 2^20 rows");
    if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return mra::fail(MRA_EINVAL, "lr > 0, 0 <= beta1, beta2 < 1 and eps > 0 required");
    const bool dev = mra::is_device_ptr(x);
    if (dev != mra::is_device_ptr(y) || (loss && dev != mra::is_device_ptr(loss)))
        return mra::fail(MRA_EINVAL, "x, y and loss must be in the same memory space");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int rc = ensure(n, B);
    if (rc) return rc;
    if ((rc = loss_and_grad(n, x, y, B, loss, dev, st))) return rc;
    n->step += 1;
    const double c1 = 1.0 / (1.0 - std::pow(double(beta1), double(n->step)));
    const double c2 = 1.0 / (1.0 - std::pow(double(beta2), double(n->step)));
    hipLaunchKernelGGL(k_adam, dim3(grid1(NPARAM)), dim3(256), 0, st, n->p, n->g, n->m, n->v, NPARAM, lr, beta1, beta2,
                       eps, float(c1), float(c2));
    MLPCHK(hipGetLastError());
    if (!dev) {
        if (loss) MLPCHK(hipMemcpyAsync(loss, n->lossd, 8, hipMemcpyDeviceToHost, st));
        MLPCHK(hipStreamSynchronize(st));
    }
    return MRA_OK;
}

extern "C" int mra_mlp_get_params(mra_mlp* n, float* params) {
    if (!n || !params) return mra::fail(MRA_EINVAL, "NULL argument");
    const bool dev = mra::is_device_ptr(params);
    MLPCHK(hipDeviceSynchronize());
    MLPCHK(hipMemcpy(params, n->p, NPARAM * sizeof(float), dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    return MRA_OK;
}

extern "C" void mra_mlp_free(mra_mlp* n) { delete n; }
