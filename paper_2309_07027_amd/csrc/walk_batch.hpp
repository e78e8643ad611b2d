// walk_batch.hpp -- gfx950 persistent batch kernel of the generalized BB/FG
// permanent (Eq. bbfgrepeated), shared by the plain launches (walk.hip) and
// the launches with column multiplicities (walk_cols_b<bucket>.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"
#include "walk_core.hpp"
#include "walk_device.hpp"

namespace bbfg {

// ---------------------------------------------------------------------------
// batched launch: persistent wavefronts pull global units from a counter
// (units are numbered longest-first); each unit dispatches on its column count
// ---------------------------------------------------------------------------
template <int NMIN, int NMAX, typename Real, bool POW>
__device__ __forceinline__ void dispatch_unit(const WalkArgs& A, const PermDesc& d, uint32_t u_local, double& r,
                                              double& i, double& a)
{
    if constexpr (NMIN <= NMAX) {
        if (d.n == NMIN) {
            walk_unit<NMIN, Real, POW>(A, d, u_local, threadIdx.x & (kWave - 1), r, i, a);
        } else {
            dispatch_unit<NMIN + 1, NMAX, Real, POW>(A, d, u_local, r, i, a);
        }
    }
}

// The loop control is kept free of divergent branches: lane 0 takes the next
// unit from the counter and hands it to the wavefront through LDS between two
// barriers, so every lane leaves the loop at the same iteration.
// POW: items carry column multiplicities (their own kernels, walk_cols_b*.hip).
// The kernels for up to 24 columns are built for more wavefronts per SIMD than
// their registers would give: FP64 four (128 VGPRs; it would take 143 and
// three), FP32 six (80 VGPRs instead of 83 and five).  The few values that no
// longer fit are spilled outside the walk loop; the 4096-item batch ran 3 %
// (FP64) and 1 % (FP32) faster.
template <int NMAX, typename Real, bool POW>
constexpr int batch_waves_per_simd()
{
    if (NMAX != 24 || POW) return 1;
    return sizeof(Real) == 8 ? 4 : 6;
}

template <int NMAX, typename Real, bool POW = false>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(batch_waves_per_simd<NMAX, Real, POW>())))
void walk_batch_kernel(WalkArgs A)
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
        const uint32_t u_local = u - (uint32_t)d.unit_base;
        double r = 0.0, i = 0.0, a = 0.0;
        dispatch_unit<1, NMAX, Real, POW>(A, d, u_local, r, i, a);
        store_partial_all_lanes(A.partials, d.part_base + u_local, r, i, a);
    }
}

}  // namespace bbfg
