// Device diagnostic (not part of the sampling method): attainable matrix-core throughput of the
// three MFMA instructions the sampler uses, measured on the caller's device, so reported
// roofline fractions can be read against what the chip sustains as well as its data sheet.
#include <hip/hip_runtime.h>

#include "../../include/gmc.h"
#include "gmc_internal.hpp"

namespace gmc {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr int kAcc = 4;

// Each wave keeps kAcc independent 32x32 accumulators busy for `iters` rounds and writes one
// float per lane to out[block * 256 + thread] (out must hold gridDim.x * 256 floats).
template <int OP>
__global__ __launch_bounds__(256) void mfma_rate_kernel(float *out, int iters)
{
    f32x16 acc[kAcc];
#pragma unroll
    for (int j = 0; j < kAcc; ++j)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[j][i] = 0.0f;
    const int l = threadIdx.x;
    const float fa = 1e-3f * (l & 7), fb = 1e-3f * (l >> 3);
    bf16x8 ba, bb;
    i32x8 ia, ib;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        ba[i] = (__bf16)(fa + i);
        bb[i] = (__bf16)(fb - i);
        ia[i] = 0x38383838 + l;
        ib[i] = 0x30303030 + i;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kAcc; ++j) {
            if constexpr (OP == GMC_FP32) acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa, fb, acc[j], 0, 0, 0);
            if constexpr (OP == GMC_BF16) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ba, bb, acc[j], 0, 0, 0);
            if constexpr (OP == GMC_FP8_E4M3)
                acc[j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(ia, ib, acc[j], 0, 0, 0, 127, 0, 127);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < kAcc; ++j)
#pragma unroll
        for (int i = 0; i < 16; ++i) s += acc[j][i];
    out[blockIdx.x * blockDim.x + l] = s;
}

}  // namespace
}  // namespace gmc

extern "C" int gmc_probe_mfma_peak(int precision, int waves_per_simd, double *tflops)
{
    using namespace gmc;
    if (!tflops || precision < GMC_FP32 || precision > GMC_FP8_E4M3 || waves_per_simd < 1 || waves_per_simd > 4)
        return set_error(GMC_EINVAL, "gmc_probe_mfma_peak: bad argument");
    const int cu = device_cu_count();
    if (cu <= 0) return set_error(GMC_EDEVICE, "gmc_probe_mfma_peak: cannot query the device");
    const int blocks = cu * waves_per_simd, iters = 2000;
    float *out = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipMalloc(&out, sizeof(float) * 256 * (size_t)blocks);
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    float ms = 0.0f;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {   // first run warms the clocks up
        e = hipEventRecord(a, nullptr);
        if (precision == GMC_FP32) hipLaunchKernelGGL(mfma_rate_kernel<GMC_FP32>, dim3(blocks), dim3(256), 0, nullptr, out, iters);
        if (precision == GMC_BF16) hipLaunchKernelGGL(mfma_rate_kernel<GMC_BF16>, dim3(blocks), dim3(256), 0, nullptr, out, iters);
        if (precision == GMC_FP8_E4M3) hipLaunchKernelGGL(mfma_rate_kernel<GMC_FP8_E4M3>, dim3(blocks), dim3(256), 0, nullptr, out, iters);
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(b, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (out) (void)hipFree(out);
    if (e != hipSuccess) return set_hip_error(e, "gmc_probe_mfma_peak");
    const double mnk = precision == GMC_FP32 ? 32.0 * 32 * 2 : (precision == GMC_BF16 ? 32.0 * 32 * 16 : 32.0 * 32 * 64);
    const double flop = 2.0 * mnk * kAcc * iters * 4.0 /* waves per block */ * blocks;
    *tflops = flop / (ms * 1e-3) / 1e12;
    return GMC_OK;
}
