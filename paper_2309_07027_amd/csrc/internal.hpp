// internal.hpp -- data structures shared by the host planner and the gfx950
// kernels of the generalized BB/FG permanent (arXiv:2309.07027, Sec. 2).
#pragma once

#include <cstdint>

namespace bbfg {

constexpr int kWave = 64;       // CDNA wavefront width
constexpr int kMaxN = 48;       // largest column count of the FP64 path
constexpr int kMaxNF32 = 24;    // largest column count of the FP32 path
constexpr int kBinomDim = kMaxN + 1;

// How the sign count Delta_k of a row is obtained inside a work unit.
//   FIXED: the row has no free sign (the pivot with M = 1); coefficient = base.
//   LANE : a lane-prefix digit; Delta = (lane_index / stride) % radix.
//   HIGH : a per-segment digit;  Delta = (h / stride) % radix, h = block index.
//   LOW  : a Gray-walked digit;  Delta = reflected decode of the position t
//          inside the block (Sec. 2.2 reflected n-ary Gray code).
enum RowKind : int32_t { ROW_FIXED = 0, ROW_LANE = 1, ROW_HIGH = 2, ROW_LOW = 3 };

// One kept row.  Column-sum coefficient = base - 2 * Delta  (Eq. Deltak), where
// base = M'_k + (1 if the row is the pivot).  Weight factor (-1)^Delta C(mp, Delta).
struct RowInfo {
    int32_t base;
    int32_t kind;
    uint32_t radix;   // mp + 1
    uint32_t stride;  // product of the radices of the earlier digits of the same kind
    int32_t mp;       // M'_k
    int32_t pad;
};

// Gray-walk table entry for position t of a block: the +-2a row that is added
// when stepping from t-1 to t, and the signed low-digit weight at t:
//   s(t) = prod_{low k} (-1)^{Delta_k(t)} C(M'_k, Delta_k(t)).
// The planner numbers the kept rows so that low digit i is kept row i; a table
// then depends on the radices of the low digits only and is shared by every
// permanent with the same low radices.
struct TabEntry {
    uint32_t row;  // index into the 2r x n array of +-2a rows (2i: +2a_i, 2i+1: -2a_i)
    uint32_t pad;
    double s;
};

// Device descriptor of one permanent.
struct PermDesc {
    uint64_t a_off;          // element offset of the r x n kept rows (complex)
    uint64_t a2_off;         // element offset of the 2r x n +-2a rows (complex)
    const TabEntry* tab;     // Gray table (Q entries, device memory)
    uint64_t unit_base;      // slot of this permanent's unit 0 in the partial arrays
    uint64_t units;          // number of units  (= groups * units_per_group)
    uint64_t units_per_group;
    uint64_t span;           // block positions per lane group (H * Q)
    uint32_t rowinfo_off;    // entry offset of the r RowInfo records
    int32_t n;               // columns
    int32_t r;               // kept rows
    uint32_t Q;              // Gray block length
    uint32_t lane_product;   // number of valid lane indices
    uint32_t groups;         // lane groups
    double scale;            // 2^{1-n} of the permanents computed (n - 1 columns of them for minors)
    double err_coeff;        // u * (n + sqrt(Q)), u the unit roundoff: error estimate = kappa * err_coeff
    uint64_t part_base;      // first partial slot; unit u, target t -> part_base + u * max(1, targets) + t
    uint32_t targets;        // 0: one permanent of the n columns.  G > 0: the G permanents that each
                             //   leave out one of the last G columns (Laplace minors)
    uint32_t res_base;       // index of the first result
    uint32_t col_pow;        // every one of the n (distinct) columns has multiplicity col_pow
                             //   (Eq. bbfgrepeated): the product is (prod_j c_j)^col_pow
    uint32_t mag_every;      // leave-one-column-out walks: units whose index in their lane group is
                             //   a multiple of mag_every sample the magnitude estimate (>= 1)
};

// Leave-one-column-out walks over K columns cover the targets in groups of
// minor_group(K): one group keeps K column sums, G prefix products and G
// accumulators per lane (4K + 8G FP64 registers).  Up to 30 columns the groups
// stay small enough for two wavefronts per SIMD (<= 256 VGPRs): up to 24
// columns groups of at most 27 - K/2 targets, at 25-30 columns two groups (the
// kernel for up to 30 columns is built for two wavefronts per SIMD).  Above,
// where the sums are long and work dominates, one wavefront per SIMD with the
// fewest groups that fit 512 registers without spilling to scratch does fewer
// products per addend (one group up to 36 columns: K + 2G - 4 complex products
// instead of about 1.6 times that), which measured 1.2-1.25 times faster at
// 31-36 columns than three groups at two wavefronts; at 25-30 columns two
// groups at two wavefronts measured 4-9 % faster than one group at one.
constexpr int minor_group(int K)
{
    int gmax = K <= 24 ? 27 - K / 2 : (K <= 30 ? (K + 1) / 2 : 54 - K / 2);
    if (gmax < 1) gmax = 1;
    if (gmax > K) gmax = K;
    const int groups = (K + gmax - 1) / gmax;
    return (K + groups - 1) / groups;
}

// Leave-one-column-out walks estimate each target's sum of |addend| from about
// this many sampled units per lane group (64 lanes each), all units if fewer.
constexpr uint64_t kMagUnitsPerGroup = 32;
inline uint32_t mag_every_for(uint64_t units_per_group)
{
    const uint64_t e = units_per_group / kMagUnitsPerGroup;
    return e > 1 ? (uint32_t)e : 1u;
}

constexpr uint32_t kUnitChunkLog2 = 6;
constexpr uint32_t kUnitChunk = 1u << kUnitChunkLog2;

// Sizes of the partial record of one unit: a complex double-double (4 doubles)
// plus the sum of |addend| (1 double).
constexpr int kPartialDoubles = 5;

// Gather job for one matrix: element (k, j) of the kept rows is
//   src[src_off + srcrow[srcrow_off + k] * ld + col(j)]   (complex elements)
// with col(j) = j when srccol_off == kIdentityCols, else srccol[srccol_off + j].
constexpr uint32_t kIdentityCols = 0xFFFFFFFFu;
struct PrepItem {
    const double* src;
    uint64_t src_off;
    uint64_t a_off;
    uint64_t a2_off;
    uint32_t srcrow_off;
    uint32_t srccol_off;
    uint32_t ld;
    int32_t n;
    int32_t r;
    int32_t f32;
};

// Kernel arguments of the walk kernels (passed by value).
struct WalkArgs {
    const PermDesc* descs;
    const RowInfo* rowinfo;
    const double* a;     // FP64 kept rows (interleaved complex)
    const double* a2;    // FP64 +-2a rows
    const float* af;     // FP32 copies
    const float* a2f;
    const double* binom; // kBinomDim x kBinomDim
    double* partials;    // kPartialDoubles per unit slot
    // batch: units are numbered item by item in "unit order"; position p of that
    // order is item uorder[p], whose units start at ubase[p] (ubase has one more
    // entry: the total).  uchunk[c] is the position of the item holding unit
    // c * kUnitChunk (one more entry: the last position), which bounds the
    // search for the item of a unit to the items of its chunk.
    const uint32_t* ubase;
    const uint32_t* uorder;
    const uint32_t* uchunk;
    uint32_t* counter;          // batch: next unit
    uint32_t total_units;       // batch: number of units
    uint32_t nitem;             // batch: number of items
};

}  // namespace bbfg
