// plan.hpp -- host planner of the generalized BB/FG permanent walk.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "internal.hpp"

namespace bbfg {

struct PlanParams {
    uint32_t q_max = 4096;     // largest Gray block length (rows of multiplicity <= 3)
    uint32_t q_max_heavy = 512;  // largest Gray block length when some M'_k > 3
    uint64_t l_min = 256;      // shortest unit (positions per lane) for small permanents
    uint64_t l_target = 4096;  // preferred unit length for large permanents
};

// Decomposition of one permanent (see walk.hip for how the kernel uses it).
struct HostPlan {
    int n = 0;                     // columns
    int r = 0;                     // kept rows (M_k > 0)
    std::vector<int> src_row;      // kept row -> user row
    std::vector<int> mult;         // M_k of the kept rows
    int pivot = -1;                // kept index of the row with one copy held at +1
    std::vector<RowInfo> rows;     // per kept row
    std::vector<int> lane_digits;  // kept indices, fastest first
    std::vector<int> high_digits;
    std::vector<int> low_digits;
    uint32_t lane_product = 1;
    uint32_t groups = 1;
    uint32_t Q = 1;
    uint64_t H = 1;
    uint64_t span = 1;             // H * Q
    uint64_t units_per_group = 1;
    uint64_t units = 1;
    uint64_t n_addends = 1;        // C'
    double err_coeff = 1.0;
    std::vector<TabEntry> table;   // Q entries
};

// Plans perm(A, M) for the n_rows multiplicities `mult` (sum == n_cols), for a
// device with `slots` resident walk wavefronts.  Returns 0 or a bbfg_status and
// sets `err`.
int build_plan(const int32_t* mult, int n_rows, int n_cols, uint64_t slots, const PlanParams& pp, HostPlan& out,
               std::string& err);

// Reflected mixed-radix Gray code (digit 0 fastest): Delta_k at position t.
void gray_digits(uint64_t t, const uint32_t* radix, int nd, uint32_t* delta);

uint64_t binom_u64(int m, int k);

}  // namespace bbfg
