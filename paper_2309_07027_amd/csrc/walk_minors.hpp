// walk_minors.hpp -- gfx950 kernel of the batched leave-one-column-out walks
// (the Laplace minors of the Clifford & Clifford step, Sec. 4, evaluated with
// Eq. bbfgrepeated).  Each bucket (largest column count) is instantiated in a
// translation unit of its own, walk_minors_b<bucket>.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"
#include "walk_core.hpp"
#include "walk_device.hpp"

namespace bbfg {

// ---------------------------------------------------------------------------
// batched leave-one-column-out walks (Laplace minors of the sampler step):
// the same persistent loop; a unit of a K-column item yields minor_group(K)
// partial records, one per target column
// ---------------------------------------------------------------------------
// Unit partials of the targets: slots slot0 + t.
struct PartialSink {
    double* partials;
    uint64_t slot0;
    __device__ __forceinline__ void sum(int t, double r, double i)
    {
        store_partial_sums_all_lanes(partials, slot0 + (uint64_t)t, r, i);
    }
    __device__ __forceinline__ void mag(int t, double a) { store_partial_mag_all_lanes(partials, slot0 + (uint64_t)t, a); }
    __device__ __forceinline__ void no_mag(int t) { partials[(slot0 + (uint64_t)t) * kPartialDoubles + 4] = 0.0; }
};

template <int K>
__device__ __forceinline__ void minors_unit_store(const WalkArgs& A, const PermDesc& d, uint32_t u_local)
{
    constexpr int G = minor_group(K);
    PartialSink sink{A.partials, d.part_base + (uint64_t)u_local * G};
    walk_minors_unit<K, G, double>(A, d, u_local, threadIdx.x & (kWave - 1), sink);
}

template <int KMIN, int KMAX>
__device__ __forceinline__ void dispatch_minors(const WalkArgs& A, const PermDesc& d, uint32_t u_local)
{
    if constexpr (KMIN <= KMAX) {
        if (d.n == KMIN) minors_unit_store<KMIN>(A, d, u_local);
        else dispatch_minors<KMIN + 1, KMAX>(A, d, u_local);
    }
}

// Kernels for up to 30 columns are built for two wavefronts per SIMD (their
// paths fit 256 VGPRs; the few spilled values live outside the walk loops),
// wider ones for one.
template <int KMAX>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(KMAX <= 30 ? 2 : 1))) void walk_minors_batch_kernel(WalkArgs A)
{
    __shared__ uint32_t next_unit;
    for (;;) {
        if (threadIdx.x == 0) next_unit = atomicAdd(A.counter, 1u);
        __syncthreads();
        const uint32_t u = __builtin_amdgcn_readfirstlane(next_unit);
        __syncthreads();
        if (u >= A.total_units) break;
        const uint32_t item = item_of_unit(A, u);
        const PermDesc d = A.descs[item];
        dispatch_minors<2, KMAX>(A, d, u - (uint32_t)d.unit_base);
    }
}

}  // namespace bbfg
