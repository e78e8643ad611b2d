// cc.hip -- gfx950 kernels of the Clifford & Clifford sampler step (Sec. 4).
//
// Step k of a sample draws the k-th output mode r_k with probability
// proportional to |perm A[(r_1..r_{k-1}, r), (pi_1..pi_k)]|^2.  Expanding that
// k x k permanent along its last row gives
//     w_r = | sum_{l=1..k} A[r, pi_l] * minor_l |^2,
//     minor_l = perm A[(r_1..r_{k-1}), (pi_1..pi_k) without pi_l],
// so one batch of k permanents of size k-1 (rows with multiplicities) serves
// every candidate row.  The minors come from the permanent engine; this kernel
// forms the weights of all candidates and draws r_k by inverse CDF.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cc_kernels.hpp"

namespace bbfg {

// A (rows x n) = the input columns of U (ideal), or of the 2m x 2m dilation
// [[se U, sl I], [sl U, -se I]] (lossy; inputs lie in the first m modes, so
// only the U blocks are ever selected).
__global__ void build_job_matrix_kernel(const double* __restrict__ U, int m, const int32_t* __restrict__ cols, int n,
                                        double se, double sl, int lossy, double* __restrict__ A)
{
    const int rows = lossy ? 2 * m : m;
    const int total = rows * n;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int r = e / n, b = e - r * n;
        const int ur = r < m ? r : r - m;
        const double f = lossy ? (r < m ? se : sl) : 1.0;
        const double* u = U + 2 * ((size_t)ur * m + cols[b]);
        A[2 * (size_t)e] = f * u[0];
        A[2 * (size_t)e + 1] = f * u[1];
    }
}

constexpr int kCCThreads = 256;

__global__ __launch_bounds__(kCCThreads) void cc_weights_kernel(const CCStep* __restrict__ steps,
                                                                const int32_t* __restrict__ pi,
                                                                const uint32_t* __restrict__ slot,
                                                                const double* __restrict__ minors,
                                                                const double* __restrict__ minor_err,
                                                                int32_t* __restrict__ drawn, double* __restrict__ wsum,
                                                                double* __restrict__ tv_est)
{
    const CCStep st = steps[blockIdx.x];
    __shared__ double w[kCCThreads];
    __shared__ double dw[kCCThreads];
    const int32_t* p = pi + st.pi_off;
    for (int r = threadIdx.x; r < st.rows; r += kCCThreads) {
        const double* arow = st.A + 2 * (size_t)r * st.n;
        double sr = 0.0, si = 0.0, e = 0.0;
        if (st.k == 1) {
            sr = arow[2 * p[0]];
            si = arow[2 * p[0] + 1];
        } else {
            for (int l = 0; l < st.k; ++l) {
                const double ar = arow[2 * p[l]], ai = arow[2 * p[l] + 1];
                const size_t q = slot[st.minor_off + l];
                const double mr = minors[2 * q];
                const double mi = minors[2 * q + 1];
                sr = __builtin_fma(ar, mr, sr);
                sr = __builtin_fma(-ai, mi, sr);
                si = __builtin_fma(ar, mi, si);
                si = __builtin_fma(ai, mr, si);
                e += __builtin_sqrt(ar * ar + ai * ai) * __builtin_sqrt(mr * mr + mi * mi) * minor_err[2 * q];
            }
        }
        w[r] = __builtin_fma(sr, sr, si * si);
        dw[r] = e * (2.0 * __builtin_sqrt(w[r]) + e);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double total = 0.0, dtotal = 0.0;
        for (int r = 0; r < st.rows; ++r) {
            total += w[r];
            dtotal += dw[r];
        }
        tv_est[blockIdx.x] = total > 0.0 ? dtotal / total : 0.0;
        const double target = st.u * total;
        double run = 0.0;
        int choice = -1;
        for (int r = 0; r < st.rows; ++r) {
            run += w[r];
            if (run > target) {
                choice = r;
                break;
            }
        }
        if (choice < 0)
            for (int r = st.rows - 1; r >= 0; --r)
                if (w[r] > 0.0) {
                    choice = r;
                    break;
                }
        drawn[blockIdx.x] = choice < 0 ? st.rows - 1 : choice;
        wsum[blockIdx.x] = total;
    }
}

hipError_t launch_build_job_matrix(const double* U, int m, const int32_t* cols, int n, double se, double sl, int lossy,
                                   double* A, hipStream_t s)
{
    const int rows = lossy ? 2 * m : m;
    const int total = rows * n;
    if (total == 0) return hipSuccess;
    const int blocks = (total + 255) / 256;
    hipLaunchKernelGGL(build_job_matrix_kernel, dim3(blocks), dim3(256), 0, s, U, m, cols, n, se, sl, lossy, A);
    return hipGetLastError();
}

hipError_t launch_cc_weights(uint32_t nsteps, const CCStep* steps, const int32_t* pi, const uint32_t* slot,
                             const double* minors, const double* minor_err, int32_t* drawn, double* wsum,
                             double* tv_est, hipStream_t s)
{
    if (nsteps == 0) return hipSuccess;
    hipLaunchKernelGGL(cc_weights_kernel, dim3(nsteps), dim3(kCCThreads), 0, s, steps, pi, slot, minors, minor_err,
                       drawn, wsum, tv_est);
    return hipGetLastError();
}

}  // namespace bbfg
