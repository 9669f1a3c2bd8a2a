// Measurement helpers: the achievable FP64 matrix-core rate of the device.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/mra.h"
#include "mra_internal.h"

namespace mra {

typedef double v4db __attribute__((ext_vector_type(4)));

// Every wave issues `iters` rounds of 8 independent v_mfma_f64_16x16x4f64
// (2048 flops each) on register operands; the accumulators are written out
// so that nothing is removed.
__global__ void __launch_bounds__(256) k_mfma_peak(double* out, int64_t iters, double a0) {
    v4db acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = v4db{0.0, 0.0, 0.0, 0.0};
    const double a = a0 + 1e-3 * (threadIdx.x & 15), b = 1.0 - 1e-3 * (threadIdx.x >> 4);
    for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace mra

using namespace mra;

extern "C" int mra_bench_mfma_f64(int64_t iters, double* tflops) {
    if (!tflops || iters < 1) return fail(MRA_EINVAL, "NULL output or iters < 1");
    int rc = check_device();
    if (rc) return rc;
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return fail(MRA_EDEVICE, "hipDeviceGetAttribute failed");
    const int blocks = cus * 8;  // 8 workgroups of 4 waves per CU
    double* out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.0f;
    if (hipMalloc(&out, size_t(blocks) * 256 * sizeof(double)) != hipSuccess) return fail(MRA_ENOMEM, "hipMalloc failed");
    rc = MRA_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = fail(MRA_EDEVICE, "hipEventCreate failed");
    } else {
        hipLaunchKernelGGL(k_mfma_peak, dim3(blocks), dim3(256), 0, nullptr, out, iters / 8 + 1, 0.5);  // warm-up
        (void)hipEventRecord(e0, nullptr);
        hipLaunchKernelGGL(k_mfma_peak, dim3(blocks), dim3(256), 0, nullptr, out, iters, 0.5);
        (void)hipEventRecord(e1, nullptr);
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.0f)
            rc = fail(MRA_EDEVICE, std::string("timing failed: ") + hipGetErrorString(hipGetLastError()));
        else
            *tflops = double(blocks) * 4.0 * double(iters) * 8.0 * 2048.0 / (double(ms) * 1e-3) / 1e12;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return rc;
}
