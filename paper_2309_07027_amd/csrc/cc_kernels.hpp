// cc_kernels.hpp -- launch interface of the sampler kernels (cc.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bbfg {

// One sample's step: candidates are the `rows` rows of the job matrix A
// (rows x n, device, interleaved complex); pi[pi_off .. pi_off+k) are the
// first k permuted columns; minors[slot[minor_off + l]] (complex) is the
// permanent of the prefix rows without column pi_l (unused when k == 1).
struct CCStep {
    const double* A;
    int32_t rows;
    int32_t n;
    int32_t k;
    uint32_t pi_off;
    uint32_t minor_off;
    uint32_t pad;
    double u;
};

hipError_t launch_build_job_matrix(const double* U, int m, const int32_t* cols, int n, double se, double sl, int lossy,
                                   double* A, hipStream_t s);
// minor_err[2 q] is the relative error estimate of minors[q] (the diagnostics
// that follow the results).  Per step: the drawn row, the total weight and an
// estimate of the total-variation distance between the step's draw
// distribution and the exact one: sum_r dw_r / sum_r w_r with
// dw_r = 2 |s_r| e_r + e_r^2, e_r = sum_l |A[r, pi_l]| |minor_l| err_l.
hipError_t launch_cc_weights(uint32_t nsteps, const CCStep* steps, const int32_t* pi, const uint32_t* slot,
                             const double* minors, const double* minor_err, int32_t* drawn, double* wsum,
                             double* tv_est, hipStream_t s);

}  // namespace bbfg
