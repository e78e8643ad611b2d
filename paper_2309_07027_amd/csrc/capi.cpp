// capi.cpp -- the C ABI of include/bbfg.h: permanents and planning diagnostics.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "runtime.hpp"
#include "sampler.hpp"

using namespace bbfg;

namespace {

int write_results(void* out, const double* vals, size_t count)
{
    if (is_device_ptr(out)) {
        BBFG_HIP(hipMemcpyAsync(out, vals, sizeof(double) * 2 * count, hipMemcpyHostToDevice, current_stream()));
        BBFG_HIP(hipStreamSynchronize(current_stream()));
    } else {
        std::memcpy(out, vals, sizeof(double) * 2 * count);
    }
    return BBFG_OK;
}

// Makes the `elems` complex elements at A available on the device.
int device_view(Context& c, const bbfg_c128* A, uint64_t elems, const double** out)
{
    if (elems == 0) {
        *out = nullptr;
        return BBFG_OK;
    }
    if (is_device_ptr(A)) {
        *out = reinterpret_cast<const double*>(A);
        return BBFG_OK;
    }
    BBFG_TRY(c.staging.ensure(sizeof(bbfg_c128) * elems));
    BBFG_HIP(hipMemcpyAsync(c.staging.p, A, sizeof(bbfg_c128) * elems, hipMemcpyHostToDevice, current_stream()));
    *out = c.staging.as<double>();
    return BBFG_OK;
}

thread_local double t_batch_kernel_ms = 0.0;
thread_local bool t_batch_graph = false;

}  // namespace

extern "C" {

const char* bbfg_last_error(void) { return last_error(); }

int bbfg_version(void) { return BBFG_VERSION; }

int bbfg_init(void)
try {
    Context* c = nullptr;
    BBFG_TRY(get_context(&c));
    return noalloc_setup();
}
BBFG_API_CATCH

int bbfg_set_cache_limits(uint64_t max_plans, uint64_t max_table_entries)
try {
    Context* c = nullptr;
    BBFG_TRY(get_context(&c));
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->plan_cap = max_plans ? (size_t)max_plans : 16384;
    c->table_entry_cap = max_table_entries ? (size_t)max_table_entries : (size_t(4) << 20);
    return BBFG_OK;
}
BBFG_API_CATCH

int bbfg_set_stream(void* hip_stream)
{
    set_current_stream(reinterpret_cast<hipStream_t>(hip_stream));
    return BBFG_OK;
}

}  // extern "C"

namespace {

// One permanent in one launch that fills the device: Eq. bbfgrepeated, or
// Eq. ryser with row multiplicities (ryser), over the same walk.
int single_perm(const bbfg_c128* A, int32_t n_rows, const int32_t* row_mult, int32_t n_cols, bbfg_c128* out,
                bbfg_info* info, bool ryser)
{
    if (!out) return set_error(BBFG_EINVAL, "out is NULL");
    BBFG_TRY(validate_shape(row_mult, n_rows, n_cols, kMaxN));
    if (n_cols > 0 && !A) return set_error(BBFG_EINVAL, "A is NULL");
    if (info) std::memset(info, 0, sizeof *info);
    if (n_cols == 0) {
        const double one[2] = {1.0, 0.0};
        if (info) {
            info->kappa = 1.0;
            info->n_addends = 1;
        }
        return write_results(out, one, 1);
    }
    Context* c = nullptr;
    BBFG_TRY(get_context(&c));
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    const double* Ad = nullptr;
    BBFG_TRY(device_view(*c, A, (uint64_t)n_rows * (uint64_t)n_cols, &Ad));
    std::vector<PermItem> items(1);
    items[0].src = Ad;
    items[0].src_off = 0;
    items[0].ld = (uint32_t)n_cols;
    items[0].n_rows = n_rows;
    items[0].n = n_cols;
    items[0].mult = row_mult;
    BBFG_TRY(get_plan(*c, row_mult, n_rows, n_cols, 0, PLAN_SINGLE, &items[0].plan, 0, ryser));
    double res[2], diag[2];
    RunResult rr;
    BBFG_TRY(run_perms(*c, items, 0, true, res, diag, &rr));
    if (info) {
        bool mult = false;
        for (int32_t i = 0; i < n_rows; ++i) mult = mult || row_mult[i] > 1;
        info->rel_err_est = diag[0];
        info->kappa = diag[1];
        info->n_addends = items[0].plan->n_addends;
        info->n_units = rr.units;
        info->kernel_ms = rr.kernel_ms;
        info->flops = (double)items[0].plan->n_addends * walk_flops(n_cols, mult);
    }
    return write_results(out, res, 1);
}

}  // namespace

extern "C" {

int perm_bbfg(const bbfg_c128* A, int32_t n_rows, const int32_t* row_mult, int32_t n_cols, bbfg_c128* out,
              bbfg_info* info)
try {
    return single_perm(A, n_rows, row_mult, n_cols, out, info, false);
}
BBFG_API_CATCH

int perm_ryser(const bbfg_c128* A, int32_t n_rows, const int32_t* row_mult, int32_t n_cols, bbfg_c128* out,
               bbfg_info* info)
try {
    return single_perm(A, n_rows, row_mult, n_cols, out, info, true);
}
BBFG_API_CATCH

int perm_batch(int32_t batch, const bbfg_c128* A_packed, const int64_t* A_offset, const int32_t* n_rows,
               const int32_t* row_mult_packed, const int64_t* row_mult_offset, const int32_t* n_cols,
               int32_t precision, bbfg_c128* out, double* rel_err_est)
try {
    if (batch < 0) return set_error(BBFG_EINVAL, "batch = %d < 0", batch);
    if (batch == 0) return BBFG_OK;
    if (!out || !A_offset || !n_rows || !row_mult_offset || !n_cols)
        return set_error(BBFG_EINVAL, "NULL array argument");
    if (precision != BBFG_FP64 && precision != BBFG_FP32 && precision != BBFG_RYSER)
        return set_error(BBFG_EINVAL, "precision = %d is none of BBFG_FP64, BBFG_FP32, BBFG_RYSER", precision);
    const int f32 = precision == BBFG_FP32 ? 1 : 0;
    const bool ryser = precision == BBFG_RYSER;
    const int max_n = f32 ? kMaxNF32 : kMaxN;
    uint64_t extent = 0;
    bool any = false;
    for (int32_t b = 0; b < batch; ++b) {
        if (A_offset[b] < 0 || row_mult_offset[b] < 0) return set_error(BBFG_EINVAL, "negative offset at item %d", b);
        if (n_rows[b] > 0 && !row_mult_packed) return set_error(BBFG_EINVAL, "row_mult_packed is NULL");
        const int rc = validate_shape(n_rows[b] > 0 ? row_mult_packed + row_mult_offset[b] : nullptr, n_rows[b],
                                      n_cols[b], max_n);
        if (rc != BBFG_OK) return set_error(rc, "item %d: %s", b, last_error());
        if (n_cols[b] > 0) {
            any = true;
            extent = std::max<uint64_t>(extent, (uint64_t)A_offset[b] + (uint64_t)n_rows[b] * (uint64_t)n_cols[b]);
        }
    }
    if (any && !A_packed) return set_error(BBFG_EINVAL, "A_packed is NULL");
    std::vector<double> res(2 * (size_t)batch, 0.0), diag(2 * (size_t)batch, 0.0);
    t_batch_kernel_ms = 0.0;
    if (any) {
        Context* c = nullptr;
        BBFG_TRY(get_context(&c));
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        const double* Ad = nullptr;
        BBFG_TRY(device_view(*c, A_packed, extent, &Ad));
        // same shapes and multiplicities as the last batch (and unchanged unit
        // lengths): its plans are reused
        Context::BatchMemo& memo = c->batch_memo;
        std::vector<int32_t> flat;
        for (int32_t b = 0; b < batch; ++b)
            if (n_cols[b] > 0) flat.insert(flat.end(), row_mult_packed + row_mult_offset[b],
                                           row_mult_packed + row_mult_offset[b] + n_rows[b]);
        const bool hit = memo.epoch == c->plan_epoch && memo.f32 == precision && memo.n_rows.size() == (size_t)batch &&
                         std::equal(memo.n_rows.begin(), memo.n_rows.end(), n_rows) &&
                         std::equal(memo.n_cols.begin(), memo.n_cols.end(), n_cols) && memo.mult == flat;
        std::vector<PermItem> items;
        std::vector<int32_t> idx;
        items.reserve((size_t)batch);
        for (int32_t b = 0; b < batch; ++b) {
            if (n_cols[b] == 0) continue;
            PermItem it;
            it.src = Ad;
            it.ld = (uint32_t)n_cols[b];
            it.src_off = (uint64_t)A_offset[b];
            it.n_rows = n_rows[b];
            it.n = n_cols[b];
            it.mult = row_mult_packed + row_mult_offset[b];
            if (hit) it.plan = memo.plans[items.size()];
            else BBFG_TRY(get_plan(*c, it.mult, it.n_rows, it.n, f32, PLAN_BATCH, &it.plan, 0, ryser));
            items.push_back(std::move(it));
            idx.push_back(b);
        }
        if (!hit) {
            memo.epoch = c->plan_epoch;
            memo.f32 = precision;
            memo.n_rows.assign(n_rows, n_rows + batch);
            memo.n_cols.assign(n_cols, n_cols + batch);
            memo.mult.swap(flat);
            memo.plans.clear();
            for (auto& it : items) memo.plans.push_back(it.plan);
        }
        std::vector<double> r2(2 * items.size()), d2(2 * items.size());
        RunResult rr;
        BBFG_TRY(run_perms(*c, items, f32, false, r2.data(), d2.data(), &rr, true, true));
        t_batch_graph = rr.graph;
        t_batch_kernel_ms = rr.kernel_ms;
        for (size_t i = 0; i < items.size(); ++i) {
            res[2 * (size_t)idx[i]] = r2[2 * i];
            res[2 * (size_t)idx[i] + 1] = r2[2 * i + 1];
            diag[2 * (size_t)idx[i]] = d2[2 * i];
        }
    }
    for (int32_t b = 0; b < batch; ++b)
        if (n_cols[b] == 0) {
            res[2 * (size_t)b] = 1.0;
            res[2 * (size_t)b + 1] = 0.0;
        }
    if (rel_err_est)
        for (int32_t b = 0; b < batch; ++b) rel_err_est[b] = diag[2 * (size_t)b];
    return write_results(out, res.data(), (size_t)batch);
}
BBFG_API_CATCH

int perm_minors(const bbfg_c128* A, int32_t n_rows, const int32_t* row_mult, int32_t n_cols, bbfg_c128* out,
                double* rel_err_est)
try {
    if (!out) return set_error(BBFG_EINVAL, "out is NULL");
    if (n_cols < 1) return set_error(BBFG_EINVAL, "n_cols = %d < 1", n_cols);
    if (n_cols > kMaxN) return set_error(BBFG_ERANGE, "n_cols = %d exceeds the maximum %d", n_cols, kMaxN);
    BBFG_TRY(validate_shape(row_mult, n_rows, n_cols - 1, kMaxN - 1));
    if (!A) return set_error(BBFG_EINVAL, "A is NULL");
    std::vector<double> res(2 * (size_t)n_cols, 0.0);
    if (n_cols == 1) {
        res[0] = 1.0;  // the empty permanent
        if (rel_err_est) rel_err_est[0] = 0.0;
        return write_results(out, res.data(), 1);
    }
    Context* c = nullptr;
    BBFG_TRY(get_context(&c));
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    const double* Ad = nullptr;
    BBFG_TRY(device_view(*c, A, (uint64_t)n_rows * (uint64_t)n_cols, &Ad));
    PermItem proto;
    proto.src = Ad;
    proto.src_off = 0;
    proto.ld = (uint32_t)n_cols;
    proto.n_rows = n_rows;
    proto.n = n_cols - 1;
    proto.mult = row_mult;
    // a lone call splits its sums to fill the device (the sampler's minors use
    // the batch split, which depends on the item's shape only)
    BBFG_TRY(get_plan(*c, row_mult, n_rows, n_cols - 1, kKindMinors, PLAN_SINGLE, &proto.plan));
    std::vector<int32_t> cols((size_t)n_cols);
    for (int32_t j = 0; j < n_cols; ++j) cols[(size_t)j] = j;
    std::deque<std::vector<int32_t>> keep;
    std::vector<PermItem> items;
    std::vector<uint32_t> slot((size_t)n_cols);
    add_minor_items(proto, cols.data(), keep, items, 0, slot.data());
    size_t nres = 0;
    for (auto& it : items) nres += (size_t)it.targets;
    std::vector<double> r2(2 * nres), d2(2 * nres);
    RunResult rr;
    BBFG_TRY(run_perms(*c, items, 0, false, r2.data(), d2.data(), &rr));
    t_batch_kernel_ms = rr.kernel_ms;
    for (int32_t l = 0; l < n_cols; ++l) {
        res[2 * (size_t)l] = r2[2 * (size_t)slot[(size_t)l]];
        res[2 * (size_t)l + 1] = r2[2 * (size_t)slot[(size_t)l] + 1];
        if (rel_err_est) rel_err_est[l] = d2[2 * (size_t)slot[(size_t)l]];
    }
    return write_results(out, res.data(), (size_t)n_cols);
}
BBFG_API_CATCH

int perm_bbfg_cols(const bbfg_c128* A, int32_t n_rows, const int32_t* row_mult, int32_t n_cols, const int32_t* col_mult,
                   bbfg_c128* out, bbfg_info* info)
try {
    if (!out) return set_error(BBFG_EINVAL, "out is NULL");
    if (n_cols < 0) return set_error(BBFG_EINVAL, "n_cols = %d < 0", n_cols);
    if (n_cols > 0 && !col_mult) return set_error(BBFG_EINVAL, "col_mult is NULL");
    int64_t n = 0;
    std::vector<int32_t> kept;  // distinct columns with N_j > 0
    for (int32_t j = 0; j < n_cols; ++j) {
        if (col_mult[j] < 0) return set_error(BBFG_EINVAL, "col_mult[%d] = %d < 0", j, col_mult[j]);
        n += col_mult[j];
        if (n > kMaxN) return set_error(BBFG_ERANGE, "sum(col_mult) exceeds the maximum %d", kMaxN);
        if (col_mult[j] > 0) kept.push_back(j);
    }
    BBFG_TRY(validate_shape(row_mult, n_rows, (int32_t)n, kMaxN));
    if (info) std::memset(info, 0, sizeof *info);
    if (n == 0) {
        const double one[2] = {1.0, 0.0};
        if (info) {
            info->kappa = 1.0;
            info->n_addends = 1;
        }
        return write_results(out, one, 1);
    }
    if (!A) return set_error(BBFG_EINVAL, "A is NULL");
    Context* c = nullptr;
    BBFG_TRY(get_context(&c));
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    const double* Ad = nullptr;
    BBFG_TRY(device_view(*c, A, (uint64_t)n_rows * (uint64_t)n_cols, &Ad));
    bool uniform = true;
    for (int32_t j : kept) uniform = uniform && col_mult[j] == col_mult[kept[0]];
    const int e = col_mult[kept[0]];
    std::vector<int32_t> cmap;
    std::vector<PermItem> items(1);
    PermItem& it = items[0];
    it.src = Ad;
    it.ld = (uint32_t)n_cols;
    it.n_rows = n_rows;
    it.n = (int)n;
    it.mult = row_mult;
    bool single = true;
    if (uniform && e >= 2) {
        // (prod_j c_j)^e over the distinct columns: one sum per distinct column
        // and about n / e complex products per addend
        cmap = kept;
        it.col_pow = e;
        it.arena_cols = (int)kept.size();
        single = false;
    } else {
        // mixed multiplicities: the column-expanded matrix (repeated columns
        // gathered on the device) -- per-column powers inside the product would
        // serialise its multiply chains
        for (int32_t j : kept)
            for (int32_t t = 0; t < col_mult[j]; ++t) cmap.push_back(j);
    }
    it.col_map = cmap.data();
    if (single) BBFG_TRY(get_plan(*c, row_mult, n_rows, (int)n, 0, PLAN_SINGLE, &it.plan));
    else BBFG_TRY(get_plan(*c, row_mult, n_rows, (int)n, kKindCols, PLAN_SINGLE, &it.plan, it.arena_cols));
    double res[2], diag[2];
    RunResult rr;
    BBFG_TRY(run_perms(*c, items, 0, single, res, diag, &rr));
    if (info) {
        bool mult = false;
        for (int32_t i = 0; i < n_rows; ++i) mult = mult || row_mult[i] > 1;
        info->rel_err_est = diag[0];
        info->kappa = diag[1];
        info->n_addends = it.plan->n_addends;
        info->n_units = rr.units;
        info->kernel_ms = rr.kernel_ms;
        // C distinct column sums and C - 1 products, then (.)^e by binary powering
        const int C = it.arena_cols > 0 ? it.arena_cols : (int)n;
        int pw = 0;
        if (it.col_pow >= 2) {
            int top = 31;
            while (!((it.col_pow >> top) & 1)) --top;
            pw = top + __builtin_popcount((unsigned)it.col_pow) - 1;
        }
        info->flops = (double)it.plan->n_addends * (8.0 * C - 4.0 + 6.0 * pw + (mult ? 2.0 : 0.0));
    }
    return write_results(out, res, 1);
}
BBFG_API_CATCH

double perm_batch_last_kernel_ms(void) { return t_batch_kernel_ms; }

int perm_batch_last_was_graph(void) { return t_batch_graph ? 1 : 0; }

int bbfg_plan_query(const int32_t* row_mult, int32_t n_rows, int32_t n_cols, int32_t slots, bbfg_plan_summary* out)
try {
    if (!out) return set_error(BBFG_EINVAL, "out is NULL");
    BBFG_TRY(validate_shape(row_mult, n_rows, n_cols, kMaxN));
    if (slots < 0) return set_error(BBFG_EINVAL, "slots < 0");
    uint64_t S = (uint64_t)slots;
    if (slots == 0 && n_cols > 0) {
        Context* c = nullptr;
        BBFG_TRY(get_context(&c));
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        BBFG_TRY(walk_slots(*c, n_cols, 0, &S));
    }
    HostPlan P;
    std::string err;
    const int rc = build_plan(row_mult, n_rows, n_cols, S, PlanParams(), P, err);
    if (rc != BBFG_OK) return set_error(rc, "%s", err.c_str());
    std::memset(out, 0, sizeof *out);
    out->n_cols = P.n;
    out->n_rows_kept = P.r;
    out->pivot_row = P.pivot >= 0 ? P.src_row[(size_t)P.pivot] : -1;
    out->n_lane_digits = (int32_t)P.lane_digits.size();
    out->n_high_digits = (int32_t)P.high_digits.size();
    out->n_low_digits = (int32_t)P.low_digits.size();
    out->lane_product = P.lane_product;
    out->lane_groups = P.groups;
    out->low_count = P.Q;
    out->high_count = P.H;
    out->n_addends = P.n_addends;
    out->n_units = P.n == 0 ? 0 : P.units;
    return BBFG_OK;
}
BBFG_API_CATCH

int bbfg_gray_table(const int32_t* radices, int32_t n_digits, int32_t max_len, int32_t* changed_digit,
                    int32_t* direction)
try {
    if (n_digits < 0 || n_digits > 64 || (n_digits > 0 && !radices) || !changed_digit || !direction)
        return set_error(BBFG_EINVAL, "bad arguments");
    uint64_t len = 1;
    std::vector<uint32_t> R((size_t)n_digits);
    for (int i = 0; i < n_digits; ++i) {
        if (radices[i] < 1) return set_error(BBFG_EINVAL, "radix[%d] = %d < 1", i, radices[i]);
        R[(size_t)i] = (uint32_t)radices[i];
        len *= (uint64_t)radices[i];
        if (len > (uint64_t)std::max(0, max_len)) return set_error(BBFG_ERANGE, "Gray code longer than max_len");
    }
    std::vector<uint32_t> cur((size_t)n_digits), prev((size_t)n_digits);
    for (uint64_t t = 0; t < len; ++t) {
        gray_digits(t, R.data(), n_digits, cur.data());
        changed_digit[t] = -1;
        direction[t] = 0;
        if (t > 0)
            for (int i = 0; i < n_digits; ++i)
                if (cur[(size_t)i] != prev[(size_t)i]) {
                    changed_digit[t] = i;
                    direction[t] = (int)cur[(size_t)i] - (int)prev[(size_t)i];
                }
        prev = cur;
    }
    return BBFG_OK;
}
BBFG_API_CATCH

int bbfg_fp64_fma_peak(double* tflops, double* ms)
try {
    if (!tflops) return set_error(BBFG_EINVAL, "tflops is NULL");
    Context* c = nullptr;
    BBFG_TRY(get_context(&c));
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    hipStream_t s = current_stream();
    const uint32_t blocks = 8u * (uint32_t)c->n_cu;  // 32 wavefronts per compute unit
    DevBuf out;
    BBFG_TRY(out.ensure(sizeof(double) * 256 * (size_t)blocks));
    double flops = 0.0;
    BBFG_HIP(launch_fma_peak(blocks, 65536, out.as<double>(), s, &flops));  // warm-up: clocks ramp
    BBFG_HIP(hipEventRecord(c->ws.ev0, s));
    BBFG_HIP(launch_fma_peak(blocks, 262144, out.as<double>(), s, &flops));
    BBFG_HIP(hipEventRecord(c->ws.ev1, s));
    BBFG_HIP(hipStreamSynchronize(s));
    float t = 0.f;
    BBFG_HIP(hipEventElapsedTime(&t, c->ws.ev0, c->ws.ev1));
    *tflops = flops / ((double)t * 1e-3) / 1e12;
    if (ms) *ms = t;
    return BBFG_OK;
}
BBFG_API_CATCH

int bbfg_walk_occupancy(int32_t n_cols, int32_t precision, int32_t* waves_per_cu, int32_t* n_cu)
try {
    const int f32 = precision == BBFG_FP32 ? 1 : 0;
    const bool minors = precision == BBFG_MINORS;
    const bool cols = precision == BBFG_COLS;
    if (n_cols < (minors ? 2 : 1) || n_cols > (f32 ? kMaxNF32 : kMaxN)) return set_error(BBFG_ERANGE, "n_cols out of range");
    Context* c = nullptr;
    BBFG_TRY(get_context(&c));
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    uint64_t S = 0;
    if (minors || cols) {
        int waves = 1;
        const int bucket = minors ? minors_bucket_max(n_cols) : batch_bucket_max(n_cols, 0);
        if (bucket < 0) return set_error(BBFG_ERANGE, "no kernel for %d columns", n_cols);
        BBFG_TRY(batch_waves(*c, bucket, minors ? kKindMinors : kKindCols, &waves));
        S = (uint64_t)waves * (uint64_t)c->n_cu;
    } else {
        BBFG_TRY(walk_slots(*c, n_cols, f32, &S));
    }
    if (waves_per_cu) *waves_per_cu = (int32_t)(S / (uint64_t)c->n_cu);
    if (n_cu) *n_cu = c->n_cu;
    return BBFG_OK;
}
BBFG_API_CATCH

}  // extern "C"
