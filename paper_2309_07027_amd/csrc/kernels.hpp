// kernels.hpp -- launch interface between the host runtime and walk.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace bbfg {

const void* walk_single_fn(int n, int f32);
const void* walk_batch_fn(int bucket, int f32);
int batch_bucket_max(int nmax, int f32);
// smallest leave-one-column-out kernel for nmax columns (adds a 30-column one)
int minors_bucket_max(int nmax);

hipError_t launch_walk_single(int n, int f32, uint32_t grid, hipStream_t s, const WalkArgs& A, uint32_t item);
hipError_t launch_walk_batch(int bucket, int f32, uint32_t grid, hipStream_t s, const WalkArgs& A);
// uniform column multiplicities (items with col_pow >= 2), FP64, buckets 16 and
// 24 (at most 24 distinct columns)
const void* walk_cols_fn(int bucket);
const void* walk_cols_fn_b16();
const void* walk_cols_fn_b24();
hipError_t launch_walk_cols(int bucket, uint32_t grid, hipStream_t s, const WalkArgs& A);
// leave-one-column-out walks (items with targets > 0), FP64, same buckets
const void* walk_minors_fn(int bucket);
const void* walk_minors_fn_b16();
const void* walk_minors_fn_b24();
const void* walk_minors_fn_b30();
const void* walk_minors_fn_b32();
const void* walk_minors_fn_b48();
hipError_t launch_walk_minors(int bucket, uint32_t grid, hipStream_t s, const WalkArgs& A);
hipError_t launch_reset_counter(uint32_t* counter, hipStream_t s);
hipError_t launch_prep(uint32_t items, hipStream_t s, const PrepItem* it, const uint32_t* srcrow, const uint32_t* srccol,
                       double* a, double* a2, float* af, float* a2f);
hipError_t launch_finalize(uint32_t results, hipStream_t s, const PermDesc* descs, const uint32_t* res_item,
                           const double* partials, double* out, double* diag);
hipError_t launch_init_binom(double* tab, hipStream_t s);
// FP64 FMA throughput probe over `blocks` blocks of 256 lanes; *flops = the work
hipError_t launch_fma_peak(uint32_t blocks, uint32_t iters, double* out, hipStream_t s, double* flops);

}  // namespace bbfg
