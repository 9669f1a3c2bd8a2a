// Partition build on the GPU (Sec. 1.2): the leaf of every observation by
// descent through the half-open regions, knot-coincidence elimination (a
// location equal to a knot of an ancestor above the finest level, both
// coordinates), NaN exclusion, and the observations grouped by leaf in input
// order (a stable radix sort of the leaf index).  Bit-identical to the host
// build: the same FP64 expressions for midpoints and knot bars, evaluated
// without contraction, on the region boxes the host computes.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <string>
#include <vector>

#include "../../include/mra.h"
#include "mra_internal.h"

namespace mra {

namespace {

__device__ __forceinline__ double bar_dev(double lo, double hi, int nb, double f, int p) {
#pragma clang fp contract(off)
    const double L = hi - lo;
    if (nb == 1) return lo + f * L;
    return (lo + f * L) + ((double(p) * L) * (1.0 - 2.0 * f)) / double(nb - 1);
}

struct LocArgs {
    const double *x, *y, *z, *box;
    int64_t n, lvl[MAXL_TREE + 1];
    int J, M, nx, ny;
    double offset;
    int nleaf;
};

// key[i]: the leaf (index within the finest level) of observation i, or nleaf
// when it has no value or coincides with a knot; counts[0] NaN values,
// counts[1] knot coincidences, counts[2] the first index outside the root and
// counts[3] the first non-finite location (atomic minima), leaf_cnt[k]
// observations per leaf.
__global__ void k_locate(LocArgs a, int* key, int* idx, unsigned long long* counts, int* leaf_cnt) {
#pragma clang fp contract(off)
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < a.n; i += int64_t(gridDim.x) * blockDim.x) {
        idx[i] = int(i);
        key[i] = a.nleaf;
        const double px = a.x[i], py = a.y[i];
        if (!isfinite(px) || !isfinite(py)) {
            atomicMin(&counts[3], (unsigned long long)i);
            continue;
        }
        if (isnan(a.z[i])) {
            atomicAdd(&counts[0], 1ull);
            continue;
        }
        const double* rb = a.box;
        if (px < rb[0] || px >= rb[1] || py < rb[2] || py >= rb[3]) {
            atomicMin(&counts[2], (unsigned long long)i);
            continue;
        }
        int64_t k = 0;
        bool on_knot = false;
        for (int m = 0; m + 1 < a.M; ++m) {
            const double* b = a.box + 4 * (a.lvl[m] + k);
            bool hx = false, hy = false;
            for (int p = 0; p < a.nx && !hx; ++p) hx = (px == bar_dev(b[0], b[1], a.nx, a.offset, p));
            for (int q = 0; q < a.ny && !hy; ++q) hy = (py == bar_dev(b[2], b[3], a.ny, a.offset, q));
            on_knot = on_knot || (hx && hy);
            const double mx = 0.5 * (b[0] + b[1]), my = 0.5 * (b[2] + b[3]);
            int c;
            if (a.J == 4) {
                c = (px >= mx ? 1 : 0) + (py >= my ? 2 : 0);
            } else {
                const bool sx = (b[1] - b[0]) >= (b[3] - b[2]);
                c = sx ? (px >= mx ? 1 : 0) : (py >= my ? 1 : 0);
            }
            k = a.J * k + c;
        }
        if (on_knot) {
            atomicAdd(&counts[1], 1ull);
            continue;
        }
        key[i] = int(k);
        atomicAdd(&leaf_cnt[k], 1);
    }
}

__global__ void k_gather(const double* x, const double* y, const double* z, const int* idx, int64_t n, double* ox,
                         double* oy, double* oz, int64_t* orig) {
    for (int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; j < n; j += int64_t(gridDim.x) * blockDim.x) {
        const int i = idx[j];
        ox[j] = x[i];
        oy[j] = y[i];
        oz[j] = z[i];
        orig[j] = i;
    }
}

__global__ void k_minmax(const double* x, const double* y, int64_t n, double* out4) {
    // out4: min x, max x, min y, max y (exact: order does not matter)
    __shared__ double red[4][256];
    double v[4] = {std::numeric_limits<double>::infinity(), -std::numeric_limits<double>::infinity(),
                   std::numeric_limits<double>::infinity(), -std::numeric_limits<double>::infinity()};
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        v[0] = fmin(v[0], x[i]); v[1] = fmax(v[1], x[i]);
        v[2] = fmin(v[2], y[i]); v[3] = fmax(v[3], y[i]);
    }
    for (int c = 0; c < 4; ++c) red[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + s]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + s]);
            red[2][threadIdx.x] = fmin(red[2][threadIdx.x], red[2][threadIdx.x + s]);
            red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out4[blockIdx.x] = red[0][0], out4[64 + blockIdx.x] = red[1][0],
                          out4[128 + blockIdx.x] = red[2][0], out4[192 + blockIdx.x] = red[3][0];
}

int64_t ipow_g(int64_t b, int e) {
    int64_t v = 1;
    while (e-- > 0) v *= b;
    return v;
}

}  // namespace

// The partition of device-resident x, y, z (n entries).  Fills t (boxes,
// level starts, ranges, counts; t.x/y/z/orig stay empty) and allocates the
// grouped device arrays *ox, *oy, *oz, *oorig (n_used entries).
int build_device_tree(const double* x, const double* y, const double* z, int64_t n, int J, int r, int M,
                      double offset, const double* domain4, HostTree& t, double** ox, double** oy, double** oz,
                      int64_t** oorig, std::string& err) {
    *ox = *oy = *oz = nullptr;
    *oorig = nullptr;
    if (n < 0 || (J != 2 && J != 4) || r < 1 || M < 1 || M > MAXL_TREE) {
        err = "invalid n, J (2 or 4), r (>= 1) or M (1..16)";
        return MRA_EINVAL;
    }
    if (n > (int64_t(1) << 31) - 1) {
        err = "n must fit in 31 bits";
        return MRA_EINVAL;
    }
    int nx = 1;
    while (static_cast<int64_t>(nx) * nx < r) ++nx;
    const int ny = r / nx;
    t.J = J; t.M = M; t.r = r; t.nx = nx; t.ny = ny; t.rhat = nx * ny;
    if (t.rhat > 64) {
        err = "r_hat > 64 is not supported (the kernel tiles hold at most 64 knots)";
        return MRA_EINVAL;
    }
    t.P = t.rhat <= 16 ? 16 : (t.rhat <= 32 ? 32 : 64);
    t.offset = offset > 0.0 ? offset : std::exp(1.0) / 100.0;
    t.n_in = n;
    if (static_cast<double>(M - 1) * std::log(static_cast<double>(J)) > std::log(4.0e7)) {
        err = "too many regions (J^(M-1) > 4e7)";
        return MRA_EINVAL;
    }
    t.nleaf = ipow_g(J, M - 1);
    t.lvl_start.assign(M + 1, 0);
    t.nreg = 0;
    for (int m = 0; m < M; ++m) { t.lvl_start[m] = t.nreg; t.nreg += ipow_g(J, m); }
    t.lvl_start[M] = t.nreg;

    std::vector<void*> tmp;
    auto dal = [&](void** p, size_t bytes) {
        if (hipMalloc(p, std::max<size_t>(bytes, 8)) != hipSuccess) return false;
        tmp.push_back(*p);
        return true;
    };
    auto cleanup = [&]() {
        for (void* p : tmp) (void)hipFree(p);
        tmp.clear();
    };
    const int grid = int(std::min<int64_t>((n + 255) / 256, 4096));
    // root region
    double root[4];
    if (domain4) {
        for (int c = 0; c < 4; ++c) root[c] = domain4[c];
        if (!(root[1] > root[0]) || !(root[3] > root[2])) {
            err = "domain4 must have xmax > xmin and ymax > ymin";
            return MRA_EINVAL;
        }
    } else {
        double mm[256];
        double* dmm = nullptr;
        if (!dal(reinterpret_cast<void**>(&dmm), 256 * sizeof(double))) { cleanup(); err = "device allocation failed"; return MRA_ENOMEM; }
        const int g = n > 0 ? int(std::min<int64_t>((n + 255) / 256, 64)) : 0;
        double xmin = std::numeric_limits<double>::infinity(), xmax = -xmin, ymin = xmin, ymax = -xmin;
        if (g > 0) {
            hipLaunchKernelGGL(k_minmax, dim3(g), dim3(256), 0, nullptr, x, y, n, dmm);
            if (hipMemcpy(mm, dmm, sizeof mm, hipMemcpyDeviceToHost) != hipSuccess) { cleanup(); err = "copy failed"; return MRA_EDEVICE; }
            for (int b = 0; b < g; ++b) {
                xmin = std::fmin(xmin, mm[b]); xmax = std::fmax(xmax, mm[64 + b]);
                ymin = std::fmin(ymin, mm[128 + b]); ymax = std::fmax(ymax, mm[192 + b]);
            }
        }
        if (n == 0) { xmin = ymin = 0.0; xmax = ymax = 1.0; }
        const double lx = xmax - xmin, ly = ymax - ymin;
        root[0] = xmin; root[1] = xmax + 0.01 * (lx > 0.0 ? lx : 1.0);
        root[2] = ymin; root[3] = ymax + 0.01 * (ly > 0.0 ? ly : 1.0);
    }
    // region boxes on the host (the same expressions as the host build)
    t.box.assign(4 * t.nreg, 0.0);
    for (int c = 0; c < 4; ++c) t.box[c] = root[c];
    for (int m = 0; m + 1 < M; ++m)
        for (int64_t k = 0; k < ipow_g(J, m); ++k) {
            const double* b = &t.box[4 * (t.lvl_start[m] + k)];
            const double mx = 0.5 * (b[0] + b[1]), my = 0.5 * (b[2] + b[3]);
            const bool sx = (b[1] - b[0]) >= (b[3] - b[2]);
            for (int j = 0; j < J; ++j) {
                double* c = &t.box[4 * (t.lvl_start[m + 1] + J * k + j)];
                c[0] = b[0]; c[1] = b[1]; c[2] = b[2]; c[3] = b[3];
                if (J == 4) {
                    if (j & 1) c[0] = mx; else c[1] = mx;
                    if (j & 2) c[2] = my; else c[3] = my;
                } else if (sx) {
                    if (j) c[0] = mx; else c[1] = mx;
                } else {
                    if (j) c[2] = my; else c[3] = my;
                }
            }
        }
    double* dbox = nullptr;
    int *key = nullptr, *idx = nullptr, *key2 = nullptr, *idx2 = nullptr, *leaf_cnt = nullptr;
    unsigned long long* dcnt = nullptr;
    if (!dal(reinterpret_cast<void**>(&dbox), t.box.size() * 8) || !dal(reinterpret_cast<void**>(&key), n * 4) ||
        !dal(reinterpret_cast<void**>(&idx), n * 4) || !dal(reinterpret_cast<void**>(&key2), n * 4) ||
        !dal(reinterpret_cast<void**>(&idx2), n * 4) || !dal(reinterpret_cast<void**>(&leaf_cnt), t.nleaf * 4) ||
        !dal(reinterpret_cast<void**>(&dcnt), 4 * 8)) {
        cleanup();
        err = "device allocation failed while building the tree";
        return MRA_ENOMEM;
    }
    const unsigned long long c0[4] = {0ull, 0ull, ~0ull, ~0ull};
    if (hipMemcpy(dbox, t.box.data(), t.box.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dcnt, c0, sizeof c0, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(leaf_cnt, 0, t.nleaf * 4) != hipSuccess) {
        cleanup();
        err = "device copy failed while building the tree";
        return MRA_EDEVICE;
    }
    LocArgs la{};
    la.x = x; la.y = y; la.z = z; la.box = dbox; la.n = n;
    for (int m = 0; m <= M; ++m) la.lvl[m] = t.lvl_start[m];
    la.J = J; la.M = M; la.nx = nx; la.ny = ny; la.offset = t.offset; la.nleaf = int(t.nleaf);
    if (n > 0) hipLaunchKernelGGL(k_locate, dim3(grid), dim3(256), 0, nullptr, la, key, idx, dcnt, leaf_cnt);
    unsigned long long cnt[4];
    std::vector<int> lc(t.nleaf);
    if (hipMemcpy(cnt, dcnt, sizeof cnt, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(lc.data(), leaf_cnt, t.nleaf * 4, hipMemcpyDeviceToHost) != hipSuccess) {
        cleanup();
        err = "device copy failed while building the tree";
        return MRA_EDEVICE;
    }
    if (cnt[3] != ~0ull) {
        cleanup();
        err = "non-finite location at index " + std::to_string(cnt[3]);
        return MRA_EINVAL;
    }
    if (cnt[2] != ~0ull) {
        cleanup();
        err = "observation " + std::to_string(cnt[2]) + " lies outside the root region";
        return MRA_EDOMAIN;
    }
    t.n_nan = int64_t(cnt[0]);
    t.n_elim = int64_t(cnt[1]);
    t.n_dup = 0;
    std::vector<int64_t> off(t.nleaf + 1, 0);
    for (int64_t k = 0; k < t.nleaf; ++k) off[k + 1] = off[k] + lc[k];
    t.n_used = off[t.nleaf];
    // stable grouping by leaf: radix sort of (leaf, input index) pairs
    int bits = 1;
    while ((int64_t(1) << bits) <= t.nleaf) ++bits;
    size_t tb = 0;
    void* tstore = nullptr;
    if (n > 0) {
        if (hipcub::DeviceRadixSort::SortPairs(nullptr, tb, key, key2, idx, idx2, int(n), 0, bits) != hipSuccess ||
            !dal(&tstore, tb) ||
            hipcub::DeviceRadixSort::SortPairs(tstore, tb, key, key2, idx, idx2, int(n), 0, bits) != hipSuccess) {
            cleanup();
            err = "radix sort of the leaf indices failed";
            return MRA_EDEVICE;
        }
    }
    const int64_t nu = t.n_used;
    if (hipMalloc(reinterpret_cast<void**>(ox), std::max<int64_t>(nu, 1) * 8) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(oy), std::max<int64_t>(nu, 1) * 8) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(oz), std::max<int64_t>(nu, 1) * 8) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(oorig), std::max<int64_t>(nu, 1) * 8) != hipSuccess) {
        cleanup();
        err = "device allocation of the grouped observations failed";
        return MRA_ENOMEM;
    }
    if (nu > 0)
        hipLaunchKernelGGL(k_gather, dim3(int(std::min<int64_t>((nu + 255) / 256, 4096))), dim3(256), 0, nullptr, x, y, z,
                           idx2, nu, *ox, *oy, *oz, *oorig);
    const hipError_t e = hipDeviceSynchronize();
    cleanup();
    if (e != hipSuccess) {
        err = std::string("tree build kernels failed: ") + hipGetErrorString(e);
        return MRA_EDEVICE;
    }
    // observation range of every region's subtree
    t.obs_lo.assign(t.nreg, 0);
    t.obs_hi.assign(t.nreg, 0);
    for (int m = 0; m < M; ++m) {
        const int64_t span = ipow_g(J, M - 1 - m);
        for (int64_t k = 0; k < ipow_g(J, m); ++k) {
            t.obs_lo[t.lvl_start[m] + k] = off[k * span];
            t.obs_hi[t.lvl_start[m] + k] = off[(k + 1) * span];
        }
    }
    return MRA_OK;
}

}  // namespace mra
