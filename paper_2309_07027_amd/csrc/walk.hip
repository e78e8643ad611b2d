// walk.hip -- gfx950 kernels of the generalized BB/FG permanent
// (arXiv:2309.07027, Eq. bbfg and Eq. bbfgrepeated, walked as in Sec. 2.1/2.2).
//
// Work decomposition (planned on the host):
//   * the C' addends are indexed by the sign counts Delta_k of the kept rows;
//   * a few digits are LANE digits: each of the 64 lanes of a wavefront owns one
//     value of them (the analogue of the fixed leading delta bits that give the
//     data-flow engine its concurrent streams, Sec. 3 and App. A.2);
//   * the LOW digits form a block of Q positions walked in reflected mixed-radix
//     Gray order, one row changing per step (Sec. 2.2); the changed row is the
//     same for every lane, so its values reach the lanes as scalar (SGPR)
//     operands;
//   * the HIGH digits number the blocks.
// A work unit is one wavefront's contiguous range of (block, position) pairs.
// At the start of every unit and every block the column sums are recomputed
// from scratch (Sec. 2.1 re-seeding), which bounds the drift of the updated
// sums.  Per-lane FP64 sums are reduced across the wavefront in double-double;
// the finalize kernel adds the unit partials of a permanent in a fixed order in
// double-double and applies the exact factor 2^{1-n}.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"
#include "kernels.hpp"
#include "walk_core.hpp"
#include "walk_batch.hpp"
#include "walk_device.hpp"

namespace bbfg {


// ---------------------------------------------------------------------------
// binomial table C(m, k), 0 <= k <= m <= kMaxN, built by Pascal's rule (exact)
// ---------------------------------------------------------------------------
__global__ void init_binom_kernel(double* tab)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int m = 0; m < kBinomDim; ++m)
        for (int k = 0; k < kBinomDim; ++k) {
            double v;
            if (k > m) v = 0.0;
            else if (k == 0 || k == m) v = 1.0;
            else v = tab[(m - 1) * kBinomDim + k - 1] + tab[(m - 1) * kBinomDim + k];
            tab[m * kBinomDim + k] = v;
        }
}

// ---------------------------------------------------------------------------
// prep: gather the kept rows of each matrix, and build the +-2a rows
// ---------------------------------------------------------------------------
__global__ void prep_rows_kernel(const PrepItem* __restrict__ items, const uint32_t* __restrict__ srcrow,
                                 const uint32_t* __restrict__ srccol, double* __restrict__ a, double* __restrict__ a2,
                                 float* __restrict__ af, float* __restrict__ a2f)
{
    const PrepItem it = items[blockIdx.x];
    const int n = it.n, r = it.r;
    const double* A = it.src;
    for (int e = threadIdx.x; e < r * n; e += blockDim.x) {
        const int k = e / n, j = e - k * n;
        const uint32_t col = it.srccol_off == kIdentityCols ? (uint32_t)j : srccol[it.srccol_off + j];
        const uint64_t src = it.src_off + (uint64_t)srcrow[it.srcrow_off + k] * (uint64_t)it.ld + (uint64_t)col;
        const double xr = A[2 * src], xi = A[2 * src + 1];
        const uint64_t da = it.a_off + (uint64_t)k * n + j;
        const uint64_t dp = it.a2_off + (uint64_t)(2 * k) * n + j;
        const uint64_t dm = dp + (uint64_t)n;
        if (it.f32) {
            const float fr = (float)xr, fi = (float)xi;
            af[2 * da] = fr;
            af[2 * da + 1] = fi;
            a2f[2 * dp] = 2.0f * fr;
            a2f[2 * dp + 1] = 2.0f * fi;
            a2f[2 * dm] = -2.0f * fr;
            a2f[2 * dm + 1] = -2.0f * fi;
        } else {
            a[2 * da] = xr;
            a[2 * da + 1] = xi;
            a2[2 * dp] = 2.0 * xr;
            a2[2 * dp + 1] = 2.0 * xi;
            a2[2 * dm] = -2.0 * xr;
            a2[2 * dm + 1] = -2.0 * xi;
        }
    }
}

// ---------------------------------------------------------------------------
// single-permanent launch: one wavefront per unit, grid = units
// ---------------------------------------------------------------------------
template <int N, typename Real>
__global__ __launch_bounds__(kWave) void walk_single_kernel(WalkArgs A, uint32_t item)
{
    const PermDesc d = A.descs[item];
    const uint32_t u = blockIdx.x;
    double r, i, a;
    walk_unit<N, Real>(A, d, u, threadIdx.x & (kWave - 1), r, i, a);
    store_partial(A.partials, d.part_base + u, r, i, a);
}

__global__ void reset_counter_kernel(uint32_t* counter)
{
    if (threadIdx.x == 0) *counter = 0u;
}

// ---------------------------------------------------------------------------
// finalize: fixed-order double-double sum of a permanent's unit partials
// ---------------------------------------------------------------------------
constexpr int kFinThreads = 256;

// One block per result: result b belongs to item res_item[b], target b - res_base.
__global__ __launch_bounds__(kFinThreads) void finalize_kernel(const PermDesc* __restrict__ descs,
                                                               const uint32_t* __restrict__ res_item,
                                                               const double* __restrict__ partials,
                                                               double* __restrict__ out, double* __restrict__ diag)
{
    const PermDesc d = descs[res_item[blockIdx.x]];
    const uint64_t stride = d.targets ? d.targets : 1u;
    const uint64_t target = blockIdx.x - d.res_base;
    ddv sr = {0.0, 0.0}, si = {0.0, 0.0};
    double sa = 0.0;
    for (uint64_t u = threadIdx.x; u < d.units; u += kFinThreads) {
        const double* p = partials + (d.part_base + u * stride + target) * kPartialDoubles;
        sr = dd_add(sr, {p[0], p[1]});
        si = dd_add(si, {p[2], p[3]});
        sa += p[4];
    }
    __shared__ double sh[kFinThreads * 5];
    sh[threadIdx.x * 5 + 0] = sr.hi;
    sh[threadIdx.x * 5 + 1] = sr.lo;
    sh[threadIdx.x * 5 + 2] = si.hi;
    sh[threadIdx.x * 5 + 3] = si.lo;
    sh[threadIdx.x * 5 + 4] = sa;
    __syncthreads();
    for (int s = kFinThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const double* o = sh + (threadIdx.x + s) * 5;
            double* m = sh + threadIdx.x * 5;
            ddv x = dd_add({m[0], m[1]}, {o[0], o[1]});
            ddv y = dd_add({m[2], m[3]}, {o[2], o[3]});
            m[0] = x.hi;
            m[1] = x.lo;
            m[2] = y.hi;
            m[3] = y.lo;
            m[4] = m[4] + o[4];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double re = (sh[0] + sh[1]) * d.scale;
        const double im = (sh[2] + sh[3]) * d.scale;
        const double mag = __builtin_sqrt(re * re + im * im);
        const double absum = sh[4] * d.scale;
        const double kappa = mag > 0.0 ? absum / mag : __builtin_inf();
        out[2 * blockIdx.x] = re;
        out[2 * blockIdx.x + 1] = im;
        diag[2 * blockIdx.x] = kappa * d.err_coeff;
        diag[2 * blockIdx.x + 1] = kappa;
    }
}

// ---------------------------------------------------------------------------
// host-side launch helpers
// ---------------------------------------------------------------------------
namespace {

template <typename Real, int... Ns>
struct SingleTable {
    static constexpr int count = sizeof...(Ns);
    static const void* ptr(int n)
    {
        const void* t[] = {reinterpret_cast<const void*>(&walk_single_kernel<Ns, Real>)...};
        return (n >= 1 && n <= count) ? t[n - 1] : nullptr;
    }
};

template <typename Real, int... Is>
const void* single_ptr_impl(int n, std::integer_sequence<int, Is...>)
{
    return SingleTable<Real, (Is + 1)...>::ptr(n);
}

}  // namespace

const void* walk_single_fn(int n, int f32)
{
    if (f32) return single_ptr_impl<float>(n, std::make_integer_sequence<int, kMaxNF32>{});
    return single_ptr_impl<double>(n, std::make_integer_sequence<int, kMaxN>{});
}

// Batch kernels by bucket of the largest column count.
static const int kBuckets[] = {16, 24, 32, 48};

int batch_bucket_max(int nmax, int f32)
{
    for (int b : kBuckets)
        if (nmax <= b && (!f32 || b <= kMaxNF32)) return b;
    return -1;
}

int minors_bucket_max(int nmax)
{
    if (nmax > 24 && nmax <= 30) return 30;
    return batch_bucket_max(nmax, 0);
}

const void* walk_batch_fn(int bucket, int f32)
{
    if (f32) {
        switch (bucket) {
        case 16: return reinterpret_cast<const void*>(&walk_batch_kernel<16, float>);
        case 24: return reinterpret_cast<const void*>(&walk_batch_kernel<24, float>);
        default: return nullptr;
        }
    }
    switch (bucket) {
    case 16: return reinterpret_cast<const void*>(&walk_batch_kernel<16, double>);
    case 24: return reinterpret_cast<const void*>(&walk_batch_kernel<24, double>);
    case 32: return reinterpret_cast<const void*>(&walk_batch_kernel<32, double>);
    case 48: return reinterpret_cast<const void*>(&walk_batch_kernel<48, double>);
    default: return nullptr;
    }
}

// Column-power items have every distinct column at multiplicity >= 2, so at
// most BBFG_MAX_N / 2 = 24 distinct columns: two buckets.
const void* walk_cols_fn(int bucket)
{
    switch (bucket) {
    case 16: return walk_cols_fn_b16();
    case 24: return walk_cols_fn_b24();
    default: return nullptr;
    }
}

hipError_t launch_walk_cols(int bucket, uint32_t grid, hipStream_t s, const WalkArgs& A)
{
    const void* fn = walk_cols_fn(bucket);
    if (!fn) return hipErrorInvalidValue;
    void* args[] = {const_cast<WalkArgs*>(&A)};
    return hipLaunchKernel(fn, dim3(grid), dim3(kWave), args, 0, s);
}

const void* walk_minors_fn(int bucket)
{
    switch (bucket) {
    case 16: return walk_minors_fn_b16();
    case 24: return walk_minors_fn_b24();
    case 30: return walk_minors_fn_b30();
    case 32: return walk_minors_fn_b32();
    case 48: return walk_minors_fn_b48();
    default: return nullptr;
    }
}

hipError_t launch_walk_minors(int bucket, uint32_t grid, hipStream_t s, const WalkArgs& A)
{
    const void* fn = walk_minors_fn(bucket);
    if (!fn) return hipErrorInvalidValue;
    void* args[] = {const_cast<WalkArgs*>(&A)};
    return hipLaunchKernel(fn, dim3(grid), dim3(kWave), args, 0, s);
}

hipError_t launch_walk_single(int n, int f32, uint32_t grid, hipStream_t s, const WalkArgs& A, uint32_t item)
{
    const void* fn = walk_single_fn(n, f32);
    if (!fn) return hipErrorInvalidValue;
    void* args[] = {const_cast<WalkArgs*>(&A), &item};
    return hipLaunchKernel(fn, dim3(grid), dim3(kWave), args, 0, s);
}

hipError_t launch_walk_batch(int bucket, int f32, uint32_t grid, hipStream_t s, const WalkArgs& A)
{
    const void* fn = walk_batch_fn(bucket, f32);
    if (!fn) return hipErrorInvalidValue;
    void* args[] = {const_cast<WalkArgs*>(&A)};
    return hipLaunchKernel(fn, dim3(grid), dim3(kWave), args, 0, s);
}

hipError_t launch_reset_counter(uint32_t* counter, hipStream_t s)
{
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, counter);
    return hipGetLastError();
}

hipError_t launch_prep(uint32_t items, hipStream_t s, const PrepItem* it, const uint32_t* srcrow, const uint32_t* srccol,
                       double* a, double* a2, float* af, float* a2f)
{
    if (items == 0) return hipSuccess;
    hipLaunchKernelGGL(prep_rows_kernel, dim3(items), dim3(256), 0, s, it, srcrow, srccol, a, a2, af, a2f);
    return hipGetLastError();
}

hipError_t launch_finalize(uint32_t results, hipStream_t s, const PermDesc* descs, const uint32_t* res_item,
                           const double* partials, double* out, double* diag)
{
    if (results == 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3(results), dim3(kFinThreads), 0, s, descs, res_item, partials, out, diag);
    return hipGetLastError();
}

hipError_t launch_init_binom(double* tab, hipStream_t s)
{
    hipLaunchKernelGGL(init_binom_kernel, dim3(1), dim3(64), 0, s, tab);
    return hipGetLastError();
}

}  // namespace bbfg
