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
hipError_t launch_cc_weights(uint32_t nsteps, const CCStep* steps, const int32_t* pi, const uint32_t* slot,
                             const double* minors, int32_t* drawn, double* wsum, hipStream_t s);

}  // namespace bbfg
