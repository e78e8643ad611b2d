// plan.cpp -- host planner of the generalized BB/FG permanent walk
// (arXiv:2309.07027, Sec. 2.1 and 2.2, Eq. bbfgrepeated).
//
// The sum of Eq. (bbfgrepeated) runs over the box prod_k [0, M'_k] of sign
// counts Delta_k (one copy of the pivot row is held at +1, so M'_p = M_p - 1).
// Each row with M'_k >= 1 is a digit of radix M'_k + 1.  The planner splits the
// digits into
//   LANE digits: enumerated across the 64 lanes of a wavefront (more than one
//                wavefront per unit-range when their product exceeds 64);
//   LOW digits : walked inside a block of Q = prod radix positions in reflected
//                mixed-radix Gray order, so consecutive positions differ in one
//                digit by +-1 and the column sums change by -+2 a_k (Eq. Deltak);
//   HIGH digits: numbering the blocks.
// Work units are equal contiguous ranges of (block, position) pairs per lane
// group.  Any bijective enumeration of the addends gives the same exact sum;
// the order only affects rounding, and every unit and block start recomputes
// its column sums from scratch.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>

#include "../../include/bbfg.h"

namespace bbfg {

uint64_t binom_u64(int m, int k)
{
    if (k < 0 || k > m) return 0;
    unsigned __int128 c = 1;
    for (int i = 1; i <= k; ++i) c = c * (unsigned)(m - k + i) / (unsigned)i;
    return (uint64_t)c;
}

void gray_digits(uint64_t t, const uint32_t* radix, int nd, uint32_t* delta)
{
    // counter digit d_k = (t / P_k) % R_k with P_k = prod_{l<k} R_l; the digit
    // is reflected when the number formed by the higher digits, q_k, is odd.
    uint64_t rest = t;
    for (int k = 0; k < nd; ++k) {
        const uint32_t dg = (uint32_t)(rest % radix[k]);
        rest /= radix[k];
        delta[k] = (rest & 1u) ? (radix[k] - 1u - dg) : dg;
    }
}

namespace {

// prod_i (-1)^delta_i C(radix_i - 1, delta_i)
double signed_weight(const std::vector<uint32_t>& radix, const uint32_t* delta)
{
    double w = 1.0;
    for (size_t i = 0; i < radix.size(); ++i) {
        const double b = (double)binom_u64((int)radix[i] - 1, (int)delta[i]);
        w *= (delta[i] & 1u) ? -b : b;
    }
    return w;
}

// Subset of digit radices whose product fills whole wavefronts best.
std::vector<int> choose_lane_digits(const std::vector<int>& digits, const std::vector<RowInfo>& rows,
                                    uint64_t total)
{
    constexpr uint32_t kCap = 4 * kWave;
    if (total <= kWave) return digits;  // the whole sum fits in one wavefront
    // reachable[p] = bitmask (over positions in `digits`) with product p
    std::vector<int64_t> mask(kCap + 1, -1);
    mask[1] = 0;
    for (size_t i = 0; i < digits.size() && i < 62; ++i) {
        const uint32_t R = rows[(size_t)digits[i]].radix;
        for (int p = (int)kCap; p >= 1; --p) {
            if (mask[(size_t)p] < 0 || mask[(size_t)p] >> i & 1) continue;
            const uint64_t q = (uint64_t)p * R;
            if (q <= kCap && mask[(size_t)q] < 0) mask[(size_t)q] = mask[(size_t)p] | ((int64_t)1 << i);
        }
    }
    int best = 1;
    double best_eff = -1.0;
    for (int p = 1; p <= (int)kCap; ++p) {
        if (mask[(size_t)p] < 0) continue;
        const double groups = std::ceil((double)p / kWave);
        const double eff = (double)p / (groups * kWave);
        // prefer higher lane efficiency; among equals, the fewest wavefront groups
        if (eff > best_eff + 1e-9) {
            best_eff = eff;
            best = p;
        }
    }
    std::vector<int> out;
    for (size_t i = 0; i < digits.size() && i < 62; ++i)
        if (mask[(size_t)best] >> i & 1) out.push_back(digits[i]);
    return out;
}

}  // namespace

int make_gray_table(const std::vector<uint32_t>& radix, std::vector<TabEntry>& out, std::string& err)
{
    const int nl = (int)radix.size();
    uint64_t Q = 1;
    for (uint32_t R : radix) {
        if (R < 1) { err = "internal: radix 0"; return BBFG_ERANGE; }
        Q *= R;
        if (Q > (1u << 24)) { err = "internal: Gray table too long"; return BBFG_ERANGE; }
    }
    std::vector<uint32_t> cur((size_t)nl), prev((size_t)nl);
    out.assign((size_t)Q, TabEntry{0u, 0u, 0.0});
    for (uint32_t t = 0; t < (uint32_t)Q; ++t) {
        gray_digits(t, radix.data(), nl, cur.data());
        TabEntry e{0u, 0u, signed_weight(radix, cur.data())};
        if (t > 0) {
            int changed = -1, ndiff = 0, step = 0;
            for (int i = 0; i < nl; ++i)
                if (cur[(size_t)i] != prev[(size_t)i]) {
                    ++ndiff;
                    changed = i;
                    step = (int)cur[(size_t)i] - (int)prev[(size_t)i];
                }
            if (ndiff != 1 || (step != 1 && step != -1)) { err = "internal: Gray step"; return BBFG_ERANGE; }
            // Delta up by one: coefficient M' - 2 Delta drops by 2 -> add -2 a_i
            e.row = (uint32_t)(2 * changed + (step > 0 ? 1 : 0));
        }
        out[t] = e;
        prev = cur;
    }
    return BBFG_OK;
}

int TableCache::get(const std::vector<uint32_t>& radix, TablePtr* out, std::string& err)
{
    auto it = tables.find(radix);
    if (it != tables.end()) {
        *out = it->second;
        return BBFG_OK;
    }
    auto t = std::make_shared<std::vector<TabEntry>>();
    const int rc = make_gray_table(radix, *t, err);
    if (rc) return rc;
    entries += t->size();
    tables.emplace(radix, t);
    *out = t;
    return BBFG_OK;
}

int build_plan(const int32_t* mult, int n_rows, int n_cols, uint64_t slots, const PlanParams& pp, HostPlan& P,
               std::string& err, TableCache* cache)
{
    P = HostPlan();
    if (n_rows < 0) { err = "n_rows < 0"; return BBFG_EINVAL; }
    if (n_cols < 0) { err = "n_cols < 0"; return BBFG_EINVAL; }
    if (n_cols > kMaxN) { err = "n_cols exceeds BBFG_MAX_N"; return BBFG_ERANGE; }
    if (n_rows > 0 && !mult) { err = "row_mult is NULL"; return BBFG_EINVAL; }
    int64_t sum = 0;
    for (int i = 0; i < n_rows; ++i) {
        if (mult[i] < 0) { err = "negative row multiplicity"; return BBFG_EINVAL; }
        sum += mult[i];
    }
    if (sum != n_cols) {
        char b[128];
        std::snprintf(b, sizeof b, "sum(row_mult) = %lld != n_cols = %d", (long long)sum, n_cols);
        err = b;
        return BBFG_EINVAL;
    }
    P.n = n_cols;
    for (int i = 0; i < n_rows; ++i)
        if (mult[i] > 0) {
            P.src_row.push_back(i);
            P.mult.push_back(mult[i]);
        }
    P.r = (int)P.src_row.size();
    if (P.n == 0) return BBFG_OK;

    // pivot: first kept row with the smallest multiplicity (Sec. 2.2 moves a
    // non-repeated row to the top when one exists).  The Ryser sum has none:
    // every row copy is in or out of the subset.
    P.pivot = -1;
    if (!pp.ryser) {
        P.pivot = 0;
        for (int k = 1; k < P.r; ++k)
            if (P.mult[(size_t)k] < P.mult[(size_t)P.pivot]) P.pivot = k;
    }
    // BB/FG: 2^{1-n} times the walk; Ryser: the walk's column sums are -2 times
    // the subset sums, and (-1)^n (-2)^{-n} = 2^{-n}
    P.scale_log2 = pp.ryser ? -P.n : 1 - P.n;

    P.rows.resize((size_t)P.r);
    std::vector<int> digits;
    for (int k = 0; k < P.r; ++k) {
        RowInfo& x = P.rows[(size_t)k];
        x.mp = P.mult[(size_t)k] - (k == P.pivot ? 1 : 0);
        x.base = pp.ryser ? 0 : x.mp + (k == P.pivot ? 1 : 0);
        x.radix = (uint32_t)x.mp + 1u;
        x.stride = 1;
        x.kind = ROW_FIXED;
        x.pad = 0;
        if (x.mp >= 1) digits.push_back(k);
    }
    P.n_addends = 1;
    for (int k : digits) P.n_addends *= P.rows[(size_t)k].radix;

    // lane digits
    P.lane_digits = choose_lane_digits(digits, P.rows, P.n_addends);
    std::vector<char> used((size_t)P.r, 0);
    P.lane_product = 1;
    for (int k : P.lane_digits) {
        P.rows[(size_t)k].kind = ROW_LANE;
        P.rows[(size_t)k].stride = P.lane_product;
        P.lane_product *= P.rows[(size_t)k].radix;
        used[(size_t)k] = 1;
    }
    P.groups = (P.lane_product + kWave - 1) / kWave;

    // low digits: largest radices first, while the block stays <= q_max.  The
    // column sums drift by about u * |a| per Gray step and the coefficients
    // M' - 2 Delta grow with the multiplicities, so blocks are kept shorter
    // (re-seeded more often) when a row has M' > 3.
    int max_mp = 0;
    for (const RowInfo& x : P.rows) max_mp = std::max(max_mp, x.mp);
    const uint32_t q_max = max_mp > 3 ? std::min(pp.q_max, pp.q_max_heavy) : pp.q_max;
    std::vector<int> rest;
    for (int k : digits)
        if (!used[(size_t)k]) rest.push_back(k);
    std::vector<int> by_radix = rest;
    std::stable_sort(by_radix.begin(), by_radix.end(),
                     [&](int a, int b) { return P.rows[(size_t)a].radix > P.rows[(size_t)b].radix; });
    P.Q = 1;
    for (int k : by_radix) {
        const uint64_t q = (uint64_t)P.Q * P.rows[(size_t)k].radix;
        if (q <= q_max) {
            P.rows[(size_t)k].kind = ROW_LOW;
            P.rows[(size_t)k].stride = P.Q;
            P.Q = (uint32_t)q;
            P.low_digits.push_back(k);
            used[(size_t)k] = 1;
        }
    }
    P.H = 1;
    for (int k : rest)
        if (!used[(size_t)k]) {
            P.rows[(size_t)k].kind = ROW_HIGH;
            if (P.H > 0xFFFFFFFFull) { err = "high digit stride overflow"; return BBFG_ERANGE; }
            P.rows[(size_t)k].stride = (uint32_t)P.H;
            P.H *= P.rows[(size_t)k].radix;
            P.high_digits.push_back(k);
            used[(size_t)k] = 1;
        }
    P.span = P.H * P.Q;
    if ((uint64_t)P.lane_product * P.span != P.n_addends) { err = "internal: digit split mismatch"; return BBFG_ERANGE; }

    // renumber the kept rows: low digits first, so that a Gray table depends on
    // the low radices only
    {
        std::vector<int> order(P.low_digits.begin(), P.low_digits.end());
        std::vector<char> is_low((size_t)P.r, 0);
        for (int k : P.low_digits) is_low[(size_t)k] = 1;
        for (int k = 0; k < P.r; ++k)
            if (!is_low[(size_t)k]) order.push_back(k);
        std::vector<int> new_index((size_t)P.r);
        for (int i = 0; i < P.r; ++i) new_index[(size_t)order[(size_t)i]] = i;
        std::vector<int> src_row((size_t)P.r), mult_k((size_t)P.r);
        std::vector<RowInfo> rows((size_t)P.r);
        for (int i = 0; i < P.r; ++i) {
            src_row[(size_t)i] = P.src_row[(size_t)order[(size_t)i]];
            mult_k[(size_t)i] = P.mult[(size_t)order[(size_t)i]];
            rows[(size_t)i] = P.rows[(size_t)order[(size_t)i]];
        }
        P.src_row.swap(src_row);
        P.mult.swap(mult_k);
        P.rows.swap(rows);
        if (P.pivot >= 0) P.pivot = new_index[(size_t)P.pivot];
        for (auto* v : {&P.lane_digits, &P.low_digits, &P.high_digits})
            for (int& k : *v) k = new_index[(size_t)k];
    }

    // Gray table of the low digits
    P.low_radix.clear();
    for (int k : P.low_digits) P.low_radix.push_back(P.rows[(size_t)k].radix);
    if (cache) {
        const int rc = cache->get(P.low_radix, &P.table, err);
        if (rc) return rc;
    } else {
        auto t = std::make_shared<std::vector<TabEntry>>();
        const int rc = make_gray_table(P.low_radix, *t, err);
        if (rc) return rc;
        P.table = t;
    }
    if (P.table->size() != P.Q) { err = "internal: table length"; return BBFG_ERANGE; }

    // work units: equal contiguous (block, position) ranges per lane group
    const uint64_t total = (uint64_t)P.groups * P.span;  // wavefront-steps
    const uint64_t S = slots > 0 ? slots : 1;
    uint64_t units;
    if (pp.l_batch > 0) {
        units = (total + pp.l_batch - 1) / pp.l_batch;
    } else if (total < S * pp.l_floor) {
        units = (total + pp.l_floor - 1) / pp.l_floor;
    } else {
        const double k = std::max(1.0, std::nearbyint((double)total / ((double)S * (double)pp.l_target)));
        units = S * (uint64_t)k;
    }
    uint64_t upg = std::max<uint64_t>(1, units / P.groups);
    upg = std::min<uint64_t>(upg, P.span);
    P.units_per_group = upg;
    P.units = upg * P.groups;
    if (P.units > 0xFFFFFFFFull) { err = "too many work units"; return BBFG_ERANGE; }
    P.err_coeff = (double)P.n + std::sqrt((double)P.Q);
    return BBFG_OK;
}

}  // namespace bbfg
