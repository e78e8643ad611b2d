// autotune.cpp -- unit length of batched launches, tuned on the device.
//
// A batched launch splits every permanent into units of L Gray positions per
// lane (one wavefront each).  Short units cost re-seeding and reductions;
// long units leave wavefronts idle at the end of the launch.  The best L
// depends on the column count n (seeding costs O(r n), a step O(n)), so it is
// tuned per n: a synthetic batch of n-photon permanents (photons placed at
// random on 60 modes, as in the sampling workloads) is timed for each
// candidate L and, among those within 2 % of the fastest per addend, the
// longest is kept (the shortest for the minors kind); the plain kinds' picks are
// then made non-increasing in n, the minors' picks median-filtered over n.
// Untuned n use a default.
// Each candidate's timed launch of the plain kinds holds about 2^28 addends (at
// most 16384 items, distinct matrices repeated; milliseconds at large n,
// against tens of microseconds of launch noise).  Each candidate's rate comes
// from the median of three launches after a warm-up launch.
// The leave-one-column-out walks of the sampler (kind BBFG_MINORS) end every
// unit with one reduction per target column, so they are tuned on their own.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <vector>

#include "runtime.hpp"
#include "sampler.hpp"

using namespace bbfg;

namespace {

const uint64_t kCandidates[] = {64, 128, 256, 512, 1024, 2048, 4096};

// Synthetic batch: `count` items of n photons on 60 modes with `cols` columns
// (n, or n + 1 for minors); entries of modulus 1/sqrt(n) with pseudo-random
// phases (the values do not affect the timing).
void synthetic_batch(int n, int cols, int count, uint64_t seed, std::vector<double>& A, std::vector<int64_t>& aoff,
                     std::vector<int32_t>& rows, std::vector<int32_t>& mult, std::vector<int64_t>& moff)
{
    constexpr int kModes = 60;
    A.clear();
    aoff.clear();
    rows.clear();
    mult.clear();
    moff.clear();
    uint64_t c = 0;
    for (int it = 0; it < count; ++it) {
        int cnt[kModes] = {0};
        for (int p = 0; p < n; ++p) cnt[(splitmix64_draw(seed, c++) >> 32) % kModes]++;
        aoff.push_back((int64_t)A.size() / 2);
        moff.push_back((int64_t)mult.size());
        int r = 0;
        for (int k = 0; k < kModes; ++k)
            if (cnt[k]) {
                mult.push_back(cnt[k]);
                ++r;
                for (int j = 0; j < cols; ++j) {
                    const double ph = (double)(splitmix64_draw(seed, c++) >> 11) * 0x1.0p-53 * 6.283185307179586;
                    A.push_back(std::cos(ph) / std::sqrt((double)n));
                    A.push_back(std::sin(ph) / std::sqrt((double)n));
                }
            }
        rows.push_back(r);
    }
}

}  // namespace

extern "C" {

int bbfg_autotune(int32_t n_lo, int32_t n_hi, int32_t precision, const char* cache_path)
try {
    if (precision != BBFG_FP64 && precision != BBFG_FP32 && precision != BBFG_MINORS)
        return set_error(BBFG_EINVAL, "bad precision");
    const int kind = precision;
    const bool minors = kind == BBFG_MINORS;
    const int f32 = kind == BBFG_FP32 ? 1 : 0;
    const int max_n = f32 ? kMaxNF32 : (minors ? kMaxN - 1 : kMaxN);
    if (n_lo < 1 || n_hi < n_lo || n_hi > max_n) return set_error(BBFG_ERANGE, "n range [%d, %d] invalid", n_lo, n_hi);
    Context* c = nullptr;
    BBFG_TRY(get_context(&c));
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    hipStream_t s = current_stream();
    for (int n = n_lo; n <= n_hi; ++n) {
        std::vector<double> A;
        std::vector<int64_t> aoff, moff;
        std::vector<int32_t> rows, mult;
        // distinct synthetic items (an item of n photons on 60 modes has fewer
        // than 2^{n-1} addends).  Plain kinds: repeated until the launch holds
        // about 2^28 addends.  Minors: at most 256 items, as one sampling step
        // of a batch of samples launches (short launches are what it runs).
        const int distinct =
            (int)std::max<int64_t>(2, std::min<int64_t>(minors ? 256 : 1024, (int64_t(1) << 31) >> (n - 1)));
        const int cols = minors ? n + 1 : n;
        synthetic_batch(n, cols, distinct, 0x5eedULL * (uint64_t)n + (minors ? 7 : 0), A, aoff, rows, mult, moff);
        int count = distinct;
        if (!minors) {
            uint64_t per = 0;
            for (int i = 0; i < distinct; ++i) {
                std::shared_ptr<const HostPlan> pl;
                BBFG_TRY(get_plan(*c, mult.data() + moff[(size_t)i], rows[(size_t)i], n, kind, PLAN_BATCH, &pl));
                per += pl->n_addends;
            }
            const double want = std::ldexp(1.0, 28) / (double)std::max<uint64_t>(1, per) * distinct;
            count = (int)std::min(16384.0, std::max((double)distinct, std::ceil(want)));
        }
        DevBuf dA;
        BBFG_TRY(dA.ensure(sizeof(double) * A.size()));
        BBFG_HIP(hipMemcpyAsync(dA.p, A.data(), sizeof(double) * A.size(), hipMemcpyHostToDevice, s));
        BBFG_HIP(hipStreamSynchronize(s));
        std::vector<std::pair<uint64_t, double>> rates;  // (L, addends per ms)
        for (uint64_t L : kCandidates) {
            c->batch_L[std::make_pair(n, kind)] = L;
            ++c->plan_epoch;
            std::vector<PermItem> items;
            std::deque<std::vector<int32_t>> keep;
            std::vector<uint32_t> slot((size_t)cols);
            uint64_t addends = 0, nres = 0;
            for (int rep_item = 0; rep_item < count; ++rep_item) {
                const int i = rep_item % distinct;
                PermItem it;
                it.src = dA.as<double>();
                it.src_off = (uint64_t)aoff[(size_t)i];
                it.ld = (uint32_t)cols;
                it.n_rows = rows[(size_t)i];
                it.n = n;
                it.mult = mult.data() + moff[(size_t)i];
                BBFG_TRY(get_plan(*c, it.mult, it.n_rows, n, kind, PLAN_BATCH, &it.plan));
                addends += it.plan->n_addends;
                if (minors) {
                    keep.emplace_back((size_t)cols);
                    for (int j = 0; j < cols; ++j) keep.back()[(size_t)j] = j;
                    const int32_t* ident = keep.back().data();
                    const size_t first = items.size();
                    add_minor_items(it, ident, keep, items, nres, slot.data());
                    for (size_t q = first; q < items.size(); ++q) nres += (uint64_t)items[q].targets;
                } else {
                    items.push_back(std::move(it));
                }
            }
            std::vector<double> ms;
            for (int rep = 0; rep < 4; ++rep) {
                RunResult rr;
                BBFG_TRY(run_perms(*c, items, f32, false, nullptr, nullptr, &rr));
                if (rep > 0) ms.push_back(rr.kernel_ms);  // the first launch brings tables and clocks up
            }
            std::sort(ms.begin(), ms.end());
            rates.push_back({L, (double)addends / ms[ms.size() / 2]});
        }
        // Within 2 % of the best rate: plain batches take the longest unit (fewer
        // units, less per-unit reduction), the sampler's minors the shortest (its
        // steps are often small, and short units spread them over the device).
        double best_rate = 0.0;
        for (auto& r : rates) best_rate = std::max(best_rate, r.second);
        uint64_t best_L = kDefaultBatchUnit;
        bool found = false;
        for (auto& r : rates)
            if (r.second >= 0.98 * best_rate && (!found || (minors ? r.first < best_L : r.first > best_L))) {
                best_L = r.first;
                found = true;
            }
        c->batch_L[std::make_pair(n, kind)] = best_L;
        ++c->plan_epoch;
        dA.release();
    }
    // Plain kinds: a unit's duration grows with n at a fixed L while its fixed
    // costs do not, so the best L does not grow with n.  Picks within 2 % of the
    // best rate are flat optima, so the tuned lengths are made non-increasing in n
    // over the tuned range (the shorter of two near-equal picks).
    // The minors kind keeps the shortest pick within 2 %, which jumps where the
    // rate is flat over several lengths (1024 at one n between 256s): each pick is
    // replaced by the median of itself and its tuned neighbours.
    if (!minors) {
        for (int n = n_lo + 1; n <= n_hi; ++n) {
            uint64_t& L = c->batch_L[std::make_pair(n, kind)];
            L = std::min(L, c->batch_L[std::make_pair(n - 1, kind)]);
        }
    } else if (n_hi - n_lo >= 2) {
        std::vector<uint64_t> picks;
        for (int n = n_lo; n <= n_hi; ++n) picks.push_back(c->batch_L[std::make_pair(n, kind)]);
        for (int n = n_lo + 1; n < n_hi; ++n) {
            uint64_t w[3] = {picks[(size_t)(n - 1 - n_lo)], picks[(size_t)(n - n_lo)], picks[(size_t)(n + 1 - n_lo)]};
            std::sort(w, w + 3);
            c->batch_L[std::make_pair(n, kind)] = w[1];
        }
    }
    ++c->plan_epoch;
    if (cache_path) {
        FILE* f = std::fopen(cache_path, "w");
        if (!f) return set_error(BBFG_EINVAL, "cannot write %s", cache_path);
        for (auto& kv : c->batch_L)
            std::fprintf(f, "%d %d %llu\n", kv.first.second, kv.first.first, (unsigned long long)kv.second);
        std::fclose(f);
    }
    return BBFG_OK;
}
BBFG_API_CATCH

int bbfg_autotune_load(const char* cache_path)
try {
    if (!cache_path) return set_error(BBFG_EINVAL, "cache_path is NULL");
    Context* c = nullptr;
    BBFG_TRY(get_context(&c));
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    return load_autotune_file(*c, cache_path);
}
BBFG_API_CATCH

int bbfg_batch_unit_length(int32_t n_cols, int32_t precision, uint64_t* unit_length)
try {
    if (!unit_length) return set_error(BBFG_EINVAL, "unit_length is NULL");
    if (precision != BBFG_FP64 && precision != BBFG_FP32 && precision != BBFG_MINORS)
        return set_error(BBFG_EINVAL, "bad precision");
    const int max_n = precision == BBFG_FP32 ? kMaxNF32 : (precision == BBFG_MINORS ? kMaxN - 1 : kMaxN);
    if (n_cols < 1 || n_cols > max_n) return set_error(BBFG_ERANGE, "n_cols out of range");
    Context* c = nullptr;
    BBFG_TRY(get_context(&c));
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    *unit_length = batch_unit_length(*c, n_cols, precision);
    return BBFG_OK;
}
BBFG_API_CATCH

}  // extern "C"
