// plan.hpp -- host planner of the generalized BB/FG permanent walk.
#pragma once

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "internal.hpp"

namespace bbfg {

struct PlanParams {
    uint32_t q_max = 4096;     // largest Gray block length (rows of multiplicity <= 3)
    uint32_t q_max_heavy = 512;  // largest Gray block length when some M'_k > 3
    // single launches: units fill every resident wavefront slot when the sum allows
    uint64_t l_floor = 16;     // shortest unit (positions per lane) of a single launch
    uint64_t l_target = 1024;  // unit length of sums larger than one round of slots
    // batched launches: units of a fixed length, so an item's split depends on its
    // own shape only (0 = use the single-launch rule)
    uint64_t l_batch = 0;
    // Eq. ryser with row multiplicities instead of Eq. bbfgrepeated: every kept
    // row is a digit s_k in [0, M_k] (no pivot), column sums sum_k s_k a_kj
    // (walked as base 0, coefficient -2 s_k), weight (-1)^{s_k} C(M_k, s_k)
    bool ryser = false;
};

using TablePtr = std::shared_ptr<const std::vector<TabEntry>>;

// Gray table of low digits with radices `radix` (digit 0 fastest); entry rows
// index the +-2a rows of kept row = digit index.
int make_gray_table(const std::vector<uint32_t>& radix, std::vector<TabEntry>& out, std::string& err);

// Tables shared between plans with the same low radices.
struct TableCache {
    std::map<std::vector<uint32_t>, TablePtr> tables;
    size_t entries = 0;
    int get(const std::vector<uint32_t>& radix, TablePtr* out, std::string& err);
};

// Decomposition of one permanent (see walk.hip for how the kernel uses it).
// Kept rows are numbered low digits first (in low-digit order), then the other
// rows in input order.
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
    int scale_log2 = 0;            // the walk's sum times 2^scale_log2 is the permanent
    std::vector<uint32_t> low_radix;  // radices of the low digits (table key)
    TablePtr table;                // Q entries
    // scratch of one evaluation (run_perms, under the context's lock): the
    // evaluation that last placed this plan's row records, their offset and the
    // device copy of its table, so items sharing the plan find them without a
    // lookup
    mutable uint64_t slot_call = 0;
    mutable size_t slot_rowinfo = 0;
    mutable const TabEntry* slot_table = nullptr;
};

// Plans perm(A, M) for the n_rows multiplicities `mult` (sum == n_cols), for a
// device with `slots` resident walk wavefronts.  Returns 0 or a bbfg_status and
// sets `err`.
// Tables come from `cache` when given, else are built for this plan.
int build_plan(const int32_t* mult, int n_rows, int n_cols, uint64_t slots, const PlanParams& pp, HostPlan& out,
               std::string& err, TableCache* cache = nullptr);

// Reflected mixed-radix Gray code (digit 0 fastest): Delta_k at position t.
void gray_digits(uint64_t t, const uint32_t* radix, int nd, uint32_t* delta);

uint64_t binom_u64(int m, int k);

}  // namespace bbfg
