// walk_device.hpp -- device-side reductions shared by the walk kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"
#include "walk_core.hpp"

namespace bbfg {

// Item of global unit u in a batched launch: a scalar binary search over the
// first units of the items of u's chunk (invariant ubase[lo] <= u < ubase[hi]).
__device__ __forceinline__ uint32_t item_of_unit(const WalkArgs& A, uint32_t u)
{
    kptr<uint32_t> base = kconst(A.ubase);
    kptr<uint32_t> chunk = kconst(A.uchunk);
    const uint32_t c = u >> kUnitChunkLog2;
    uint32_t lo = chunk[c];
    uint32_t hi = chunk[c + 1] + 1;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (base[mid] <= u) lo = mid;
        else hi = mid;
    }
    return uniform_u32(kconst(A.uorder)[lo]);
}

// Wavefront sum of the per-lane results in double-double (the butterfly leaves
// the same bits in every lane), then lane 0 stores the unit's partial record.
__device__ __forceinline__ void store_partial(double* partials, uint64_t slot, double r, double i, double a)
{
    ddv sr = {r, 0.0}, si = {i, 0.0};
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        ddv orr = {__shfl_xor(sr.hi, off), __shfl_xor(sr.lo, off)};
        ddv oi = {__shfl_xor(si.hi, off), __shfl_xor(si.lo, off)};
        const double oa = __shfl_xor(a, off);
        sr = dd_add(sr, orr);
        si = dd_add(si, oi);
        a = a + oa;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        double* p = partials + slot * kPartialDoubles;
        p[0] = sr.hi;
        p[1] = sr.lo;
        p[2] = si.hi;
        p[3] = si.lo;
        p[4] = a;
    }
}

// Every lane of the wavefront stores the same partial record (the butterfly
// leaves identical bits in all lanes), so the store needs no divergent branch.
__device__ __forceinline__ void store_partial_all_lanes(double* partials, uint64_t slot, double r, double i, double a)
{
    ddv sr = {r, 0.0}, si = {i, 0.0};
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        ddv orr = {__shfl_xor(sr.hi, off), __shfl_xor(sr.lo, off)};
        ddv oi = {__shfl_xor(si.hi, off), __shfl_xor(si.lo, off)};
        const double oa = __shfl_xor(a, off);
        sr = dd_add(sr, orr);
        si = dd_add(si, oi);
        a = a + oa;
    }
    double* p = partials + slot * kPartialDoubles;
    p[0] = sr.hi;
    p[1] = sr.lo;
    p[2] = si.hi;
    p[3] = si.lo;
    p[4] = a;
}

// The two halves of store_partial_all_lanes, for callers that have the sums
// and the magnitude sum at different times: slot's (re, im) double-double sums
// over the wavefront, then its magnitude sum.
__device__ __forceinline__ void store_partial_sums_all_lanes(double* partials, uint64_t slot, double r, double i)
{
    ddv sr = {r, 0.0}, si = {i, 0.0};
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        ddv orr = {__shfl_xor(sr.hi, off), __shfl_xor(sr.lo, off)};
        ddv oi = {__shfl_xor(si.hi, off), __shfl_xor(si.lo, off)};
        sr = dd_add(sr, orr);
        si = dd_add(si, oi);
    }
    double* p = partials + slot * kPartialDoubles;
    p[0] = sr.hi;
    p[1] = sr.lo;
    p[2] = si.hi;
    p[3] = si.lo;
}

__device__ __forceinline__ void store_partial_mag_all_lanes(double* partials, uint64_t slot, double a)
{
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) a += __shfl_xor(a, off);
    partials[slot * kPartialDoubles + 4] = a;
}

}  // namespace bbfg
