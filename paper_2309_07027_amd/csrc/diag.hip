// diag.hip -- device diagnostics: an FP64 fused multiply-add throughput probe,
// the measured counterpart of the FP64 vector peak that the walk kernels are
// compared with.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace bbfg {

// Every lane runs kFmaChains independent chains x <- fma(x, a, b); the sums are
// stored so that no chain can be removed.  2 * kFmaChains * iters flops per lane.
constexpr int kFmaChains = 8;

__global__ __launch_bounds__(256) void fma_peak_kernel(double* out, uint32_t iters, double a, double b)
{
    double x[kFmaChains];
#pragma unroll
    for (int c = 0; c < kFmaChains; ++c) x[c] = 1e-3 * (double)threadIdx.x + (double)c;
#pragma unroll 4
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kFmaChains; ++c) x[c] = __builtin_fma(x[c], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kFmaChains; ++c) s += x[c];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

hipError_t launch_fma_peak(uint32_t blocks, uint32_t iters, double* out, hipStream_t s, double* flops)
{
    hipLaunchKernelGGL(fma_peak_kernel, dim3(blocks), dim3(256), 0, s, out, iters, 0.999999, 1e-7);
    *flops = 2.0 * kFmaChains * (double)iters * (double)blocks * 256.0;
    return hipGetLastError();
}

}  // namespace bbfg
