// Sustained FP64 rates of the GPU the library runs on: the ceiling that the
// row-system kernels (one v_fmac_f64 per core cell and entry) are measured
// against, next to the published peak. Three kernels with no memory traffic
// but one store per lane at the end:
//   0: independent v_fma_f64 chains (16 per lane, 8 steps per iteration);
//   1: v_mfma_f64_16x16x4f64 (4 independent accumulators);
//   2: both, interleaved in every wavefront.
// 2048 workgroups of 256 lanes (8 wavefronts per SIMD on 256 CUs).
#include "ptk_internal.h"
#include "ptucker.h"

namespace ptk {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int kRateBlocks = 2048, kRateThreads = 256;
constexpr int kChains = 16, kSteps = 8, kAcc = 4;

template <int MODE>
__global__ __launch_bounds__(kRateThreads) void k_fp64_rate(double *out, int iters, double s) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    double v[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) v[i] = s * (i + 1) + tid * 1e-9;
    d4 acc[kAcc];
#pragma unroll
    for (int i = 0; i < kAcc; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
    const double a = s + threadIdx.x * 1e-7, b = s * 0.5 - threadIdx.x * 1e-7;
    for (int it = 0; it < iters; ++it) {
        if constexpr (MODE >= 1) {
#pragma unroll
            for (int i = 0; i < kAcc; ++i)
                acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
        }
        if constexpr (MODE != 1) {
#pragma unroll
            for (int r = 0; r < kSteps; ++r)
#pragma unroll
                for (int i = 0; i < kChains; ++i) v[i] = __builtin_fma(v[i], a, b);
        }
    }
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) t += v[i];
#pragma unroll
    for (int i = 0; i < kAcc; ++i) t += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
    out[tid] = t;
}

template <int MODE>
hipError_t time_rate(double *buf, int iters, hipEvent_t e0, hipEvent_t e1, float *ms) {
    hipLaunchKernelGGL(k_fp64_rate<MODE>, dim3(kRateBlocks), dim3(kRateThreads), 0, 0, buf,
                       iters, 1.0000001);                       // warm-up
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(e0, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_fp64_rate<MODE>, dim3(kRateBlocks), dim3(kRateThreads), 0, 0, buf,
                       iters, 1.0000001);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipEventRecord(e1, 0)) != hipSuccess) return e;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
    return hipEventElapsedTime(ms, e0, e1);
}

}  // namespace
}  // namespace ptk

extern "C" ptk_status ptk_fp64_rates(int32_t iters, double *tflops_host) {
    using namespace ptk;
    if (iters < 1 || iters > 1000000 || !tflops_host) return PTK_E_INVALID;
    double *buf = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms[3] = {0.0f, 0.0f, 0.0f};
    hipError_t e = hipMalloc(&buf, sizeof(double) * kRateBlocks * kRateThreads);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = time_rate<0>(buf, iters, e0, e1, &ms[0]);
    if (e == hipSuccess) e = time_rate<1>(buf, iters, e0, e1, &ms[1]);
    if (e == hipSuccess) e = time_rate<2>(buf, iters, e0, e1, &ms[2]);
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (buf) (void)hipFree(buf);
    if (e != hipSuccess) return PTK_E_HIP;
    const double lanes = (double)kRateBlocks * kRateThreads;
    const double valu = lanes * iters * kSteps * kChains * 2.0;             // flop
    const double mfma = (lanes / 64.0) * iters * kAcc * 16.0 * 16.0 * 4.0 * 2.0;
    tflops_host[0] = valu / (ms[0] * 1e-3) * 1e-12;
    tflops_host[1] = mfma / (ms[1] * 1e-3) * 1e-12;
    tflops_host[2] = (valu + mfma) / (ms[2] * 1e-3) * 1e-12;
    return PTK_OK;
}
