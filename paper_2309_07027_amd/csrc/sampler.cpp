// sampler.cpp -- Clifford & Clifford boson sampling (arXiv:2309.07027, Sec. 4)
// on top of the batched generalized BB/FG permanent.
//
// One sample (ideal, or lossy via the 2m x 2m dilation of Sec. 4):
//   1. the n input columns (mode i taken s_i times, Eq. bs_p) are put in a
//      uniformly random order pi (Fisher-Yates);
//   2. for k = 1..n the output mode r_k is drawn with probability proportional
//      to |perm A[(r_1..r_{k-1}, r), (pi_1..pi_k)]|^2; by Laplace expansion
//      along row r this needs only the k permanents of the prefix rows
//      (repeated rows -> multiplicities, Eq. bbfgrepeated) with one of the k
//      columns removed;
//   3. the sample is the occupation of the first m output modes.
// Random numbers (SplitMix64) for sample s of a job with seed `seed`:
//   key_s = draw(seed, s); draws 0..n-2 run Fisher-Yates for i = n-1 .. 1
//   (draw n-1-i, j = ((x >> 32) * (i + 1)) >> 32); draw n-1+(k-1) gives the
//   uniform u = (x >> 11) * 2^-53 of step k.
// Uniform loss taken out at the input (Sec. 4, bs_sample_extracted): a loss
// that acts alike on every mode commutes with U, so each input photon b (the
// b-th column) is kept when draw 2n-1+b gives u < 1 - loss; the kept columns,
// in pi's order, are the sample's columns, one step each, on U's m modes.
#include "sampler.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <deque>
#include <map>

#include "cc_kernels.hpp"

namespace bbfg {

uint64_t splitmix64_draw(uint64_t key, uint64_t c)
{
    uint64_t z = key + (c + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int cc_validate(const void* U, int m, const int32_t* occ, int n_samples, double loss)
{
    if (!U) return set_error(BBFG_EINVAL, "U is NULL");
    if (!occ) return set_error(BBFG_EINVAL, "input_occupation is NULL");
    if (!(loss >= 0.0 && loss < 1.0)) return set_error(BBFG_EINVAL, "loss = %g is outside [0, 1)", loss);
    if (m < 1) return set_error(BBFG_EINVAL, "m = %d < 1", m);
    if (m > (loss > 0.0 ? 128 : 256)) return set_error(BBFG_ERANGE, "m = %d exceeds the maximum", m);
    if (n_samples < 0) return set_error(BBFG_EINVAL, "n_samples < 0");
    int64_t n = 0;
    for (int i = 0; i < m; ++i) {
        if (occ[i] < 0) return set_error(BBFG_EINVAL, "input_occupation[%d] < 0", i);
        n += occ[i];
    }
    if (n > kMaxN) return set_error(BBFG_ERANGE, "%lld photons exceed BBFG_MAX_N", (long long)n);
    return BBFG_OK;
}

size_t cc_job_footprint(int m, int n, int n_samples, double loss)
{
    const size_t rows = loss > 0.0 ? 2 * (size_t)m : (size_t)m;
    const size_t nn = (size_t)n;
    // job matrix + U copy + the share of the step working set at k = n
    return 16 * rows * nn + 16 * (size_t)m * (size_t)m + (size_t)n_samples * (48 * nn * nn * nn + 4096);
}

int cc_job_init(Context& c, CCJob& job, const double* U, bool U_on_device, int m, const int32_t* occ, int n_samples,
                double loss, uint64_t seed, bool stage_pinned)
{
    hipStream_t s = current_stream();
    job.m = m;
    job.loss = loss;
    job.keep = 1.0;
    job.rows = loss > 0.0 ? 2 * m : m;
    job.seed = seed;
    job.n_samples = n_samples;
    job.cols.clear();
    for (int i = 0; i < m; ++i)
        for (int t = 0; t < occ[i]; ++t) job.cols.push_back(i);
    job.n = (int)job.cols.size();
    job.samples.assign((size_t)n_samples, CCSample());
    job.out.assign((size_t)n_samples * (size_t)m, 0);
    job.started = job.finished = 0;
    job.kernel_ms = 0.0;
    job.n_addends = 0;
    job.tv_max = 0.0;
    if (job.n == 0) return BBFG_OK;
    // device: [U (m x m), when on the host | cols (n int32)], then A
    const size_t ubytes = U_on_device ? 0 : 16 * (size_t)m * (size_t)m;
    const size_t ucap = (ubytes + 255) / 256 * 256;
    BBFG_TRY(job.dev_in.ensure(ucap + 4 * (size_t)job.n));
    char* in = job.dev_in.as<char>();
    const double* Ud = U_on_device ? U : reinterpret_cast<const double*>(in);
    int32_t* cols_d = reinterpret_cast<int32_t*>(in + ucap);
    if (stage_pinned) {
        BBFG_TRY(job.host_in.ensure(ucap + 4 * (size_t)job.n));
        char* h = job.host_in.as<char>();
        if (ubytes) std::memcpy(h, U, ubytes);
        std::memcpy(h + ucap, job.cols.data(), 4 * (size_t)job.n);
        BBFG_HIP(hipMemcpyAsync(in, h, ucap + 4 * (size_t)job.n, hipMemcpyHostToDevice, s));
    } else {
        if (ubytes) BBFG_HIP(hipMemcpyAsync(in, U, ubytes, hipMemcpyHostToDevice, s));
        BBFG_HIP(hipMemcpyAsync(cols_d, job.cols.data(), 4 * (size_t)job.n, hipMemcpyHostToDevice, s));
    }
    BBFG_TRY(job.A.ensure(16 * (size_t)job.rows * (size_t)job.n));
    const double eta = 1.0 - loss;
    BBFG_HIP(launch_build_job_matrix(Ud, m, cols_d, job.n, std::sqrt(eta), std::sqrt(1.0 - eta), loss > 0.0 ? 1 : 0,
                                     job.A.as<double>(), s));
    return BBFG_OK;
}

int cc_lossy_job_matrix(const double* T, int m, const int32_t* occ, std::vector<double>& A, double* keep)
{
    using cd = std::complex<double>;
    const cd* t = reinterpret_cast<const cd*>(T);
    // H = T^H T (Hermitian), all of it for the row sums of the bound
    std::vector<cd> H((size_t)m * (size_t)m);
    for (int j = 0; j < m; ++j)
        for (int k = 0; k < m; ++k) {
            cd acc(0.0, 0.0);
            for (int i = 0; i < m; ++i) acc += std::conj(t[(size_t)i * m + j]) * t[(size_t)i * m + k];
            H[(size_t)j * m + k] = acc;
        }
    double bound = 0.0;
    for (int j = 0; j < m; ++j) {
        double row = 0.0;
        for (int k = 0; k < m; ++k) row += std::abs(H[(size_t)j * m + k]);
        bound = std::max(bound, row);
    }
    *keep = std::min(bound, 1.0);
    // the rest T' = T / sqrt(keep): its Gram matrix is H / keep
    const double inv = *keep > 0.0 ? 1.0 / *keep : 1.0;
    const double scale = *keep > 0.0 ? 1.0 / std::sqrt(*keep) : 1.0;
    // G = I - T'^H T' (upper triangle); overwritten by the trailing updates below
    std::vector<cd> G((size_t)m * (size_t)m), R((size_t)m * (size_t)m, cd(0.0, 0.0));
    for (int j = 0; j < m; ++j)
        for (int k = j; k < m; ++k)
            G[(size_t)j * m + k] = (j == k ? cd(1.0, 0.0) : cd(0.0, 0.0)) - H[(size_t)j * m + k] * inv;
    // right-looking Cholesky of the upper triangle: row j of R from the pivot,
    // then the trailing block loses the outer product of that row
    constexpr double kTol = 1e-10;
    for (int j = 0; j < m; ++j) {
        const double d = G[(size_t)j * m + j].real();
        if (d < -kTol) return set_error(BBFG_EINVAL, "T is not a contraction: pivot %d of I - T^H T is %g", j, d);
        if (d <= 0.0) continue;  // a zero pivot (lossless direction) leaves row j of R at zero
        const double rjj = std::sqrt(d);
        R[(size_t)j * m + j] = rjj;
        for (int k = j + 1; k < m; ++k) R[(size_t)j * m + k] = G[(size_t)j * m + k] / rjj;
        for (int k = j + 1; k < m; ++k)
            for (int l = k; l < m; ++l) G[(size_t)k * m + l] -= std::conj(R[(size_t)j * m + k]) * R[(size_t)j * m + l];
    }
    std::vector<int> cols;
    for (int i = 0; i < m; ++i)
        for (int q = 0; q < occ[i]; ++q) cols.push_back(i);
    const size_t n = cols.size();
    A.assign(2 * (size_t)(2 * m) * n, 0.0);
    for (int r = 0; r < 2 * m; ++r)
        for (size_t b = 0; b < n; ++b) {
            const cd x = r < m ? t[(size_t)r * m + cols[b]] * scale : R[(size_t)(r - m) * m + cols[b]];
            A[2 * ((size_t)r * n + b)] = x.real();
            A[2 * ((size_t)r * n + b) + 1] = x.imag();
        }
    return BBFG_OK;
}

int cc_job_init_matrix(Context& c, CCJob& job, const double* A_host, int rows, int m, const int32_t* occ,
                       int n_samples, uint64_t seed, bool stage_pinned)
{
    (void)c;
    hipStream_t s = current_stream();
    job.m = m;
    job.loss = 0.0;
    job.keep = 1.0;
    job.rows = rows;
    job.seed = seed;
    job.n_samples = n_samples;
    job.cols.clear();
    for (int i = 0; i < m; ++i)
        for (int t = 0; t < occ[i]; ++t) job.cols.push_back(i);
    job.n = (int)job.cols.size();
    job.samples.assign((size_t)n_samples, CCSample());
    job.out.assign((size_t)n_samples * (size_t)m, 0);
    job.started = job.finished = 0;
    job.kernel_ms = 0.0;
    job.n_addends = 0;
    job.tv_max = 0.0;
    if (job.n == 0) return BBFG_OK;
    const size_t bytes = 16 * (size_t)rows * (size_t)job.n;
    BBFG_TRY(job.A.ensure(bytes));
    if (stage_pinned) {
        BBFG_TRY(job.host_in.ensure(bytes));
        std::memcpy(job.host_in.p, A_host, bytes);
        BBFG_HIP(hipMemcpyAsync(job.A.p, job.host_in.p, bytes, hipMemcpyHostToDevice, s));
    } else {
        BBFG_HIP(hipMemcpyAsync(job.A.p, A_host, bytes, hipMemcpyHostToDevice, s));
    }
    return BBFG_OK;
}

namespace {

void finish_sample(CCJob& job, int s)
{
    const CCSample& S = job.samples[(size_t)s];
    int32_t* o = job.out.data() + (size_t)s * (size_t)job.m;
    for (int i = 0; i < job.m; ++i) o[i] = 0;
    for (int32_t r : S.prefix)
        if (r < job.m) o[r]++;
    job.tv_max = std::max(job.tv_max, S.tv);
    job.finished++;
}

}  // namespace

void cc_start_sample(CCJob& job, int s)
{
    CCSample& S = job.samples[(size_t)s];
    S.key = splitmix64_draw(job.seed, (uint64_t)s);
    S.k = 1;
    S.tv = 0.0;
    S.prefix.clear();
    S.pi.resize((size_t)job.n);
    for (int b = 0; b < job.n; ++b) S.pi[(size_t)b] = b;
    for (int i = job.n - 1; i >= 1; --i) {
        const uint64_t x = splitmix64_draw(S.key, (uint64_t)(job.n - 1 - i));
        const int j = (int)(((x >> 32) * (uint64_t)(i + 1)) >> 32);
        std::swap(S.pi[(size_t)i], S.pi[(size_t)j]);
    }
    S.steps = job.n;
    if (job.keep < 1.0) {
        std::vector<char> alive((size_t)job.n);
        for (int b = 0; b < job.n; ++b) {
            const uint64_t x = splitmix64_draw(S.key, (uint64_t)(2 * job.n - 1 + b));
            alive[(size_t)b] = (double)(x >> 11) * 0x1.0p-53 < job.keep;
        }
        int kept = 0;
        for (int l = 0; l < job.n; ++l)
            if (alive[(size_t)S.pi[(size_t)l]]) S.pi[(size_t)kept++] = S.pi[(size_t)l];
        S.pi.resize((size_t)kept);
        S.steps = kept;
    }
    if (S.steps == 0) finish_sample(job, s);  // every photon lost: an empty sample
}


void add_minor_items(const PermItem& proto, const int32_t* cols, std::deque<std::vector<int32_t>>& keep,
                     std::vector<PermItem>& items, uint64_t res_first, uint32_t* slot)
{
    const int K = proto.plan->n + 1;
    const int G = minor_group(K);
    const int groups = (K + G - 1) / G;
    uint64_t res = res_first;
    for (int gi = 0; gi < groups; ++gi) {
        // targets [t0, t0 + G); the last group may reach back into the previous
        // one, whose results own those columns
        const int t0 = std::min(gi * G, K - G);
        keep.emplace_back();
        std::vector<int32_t>& cm = keep.back();
        for (int l = 0; l < K; ++l)
            if (l < t0 || l >= t0 + G) cm.push_back(cols[l]);
        for (int l = t0; l < t0 + G; ++l) cm.push_back(cols[l]);
        PermItem it = proto;
        it.col_map = cm.data();
        it.targets = G;
        items.push_back(std::move(it));
        for (int t = 0; t < G; ++t)
            if (t0 + t >= gi * G) slot[t0 + t] = (uint32_t)(res + (uint64_t)t);
        res += (uint64_t)G;
    }
}

int cc_step_begin(Context& c, Workspace& w, std::vector<ActiveSample>& act, CCPending& p, uint64_t* addends)
{
    hipStream_t s = current_stream();
    p = CCPending();
    std::vector<PermItem> items;
    std::deque<std::vector<int32_t>> keep;  // multiplicities, row and column maps (stable addresses)
    std::vector<CCStep> steps;
    std::vector<int32_t> pis;
    std::vector<uint32_t> slots;            // result index of each minor
    std::vector<size_t>& act_of_step = p.act_of_step;
    uint64_t nres = 0;
    for (size_t ai = 0; ai < act.size(); ++ai) {
        CCJob& J = *act[ai].job;
        CCSample& S = J.samples[(size_t)act[ai].s];
        if (J.n == 0 || S.k > S.steps) continue;
        const int k = S.k;
        CCStep st;
        std::memset(&st, 0, sizeof st);
        st.A = J.A.as<double>();
        st.rows = J.rows;
        st.n = J.n;
        st.k = k;
        st.pi_off = (uint32_t)pis.size();
        for (int l = 0; l < k; ++l) pis.push_back(S.pi[(size_t)l]);
        const uint64_t x = splitmix64_draw(S.key, (uint64_t)(J.n - 1 + (k - 1)));
        st.u = (double)(x >> 11) * 0x1.0p-53;
        if (k >= 2) {
            // the k minors share the prefix rows: one joint walk over k columns.
            // Rows are listed by multiplicity (then mode), so the plan depends on
            // the multiset of multiplicities only and is shared by many steps.
            std::map<int32_t, int32_t> cnt;
            for (int32_t r : S.prefix) cnt[r]++;
            std::vector<std::pair<int32_t, int32_t>> rm(cnt.begin(), cnt.end());  // (mode, count)
            std::sort(rm.begin(), rm.end(), [](const std::pair<int32_t, int32_t>& a, const std::pair<int32_t, int32_t>& b) {
                return a.second != b.second ? a.second < b.second : a.first < b.first;
            });
            keep.emplace_back();
            std::vector<int32_t>& rowmap = keep.back();
            keep.emplace_back();
            std::vector<int32_t>& mult = keep.back();
            for (auto& kv : rm) {
                rowmap.push_back(kv.first);
                mult.push_back(kv.second);
            }
            PermItem proto;
            BBFG_TRY(get_plan(c, mult.data(), (int)mult.size(), k - 1, BBFG_MINORS, PLAN_BATCH, &proto.plan));
            proto.src = J.A.as<double>();
            proto.src_off = 0;
            proto.ld = (uint32_t)J.n;
            proto.n_rows = (int)mult.size();
            proto.n = k - 1;
            proto.mult = mult.data();
            proto.row_map = rowmap.data();
            st.minor_off = (uint32_t)slots.size();
            slots.resize(slots.size() + (size_t)k);
            const size_t first = items.size();
            add_minor_items(proto, S.pi.data(), keep, items, nres, slots.data() + st.minor_off);
            for (size_t i = first; i < items.size(); ++i) nres += (uint64_t)items[i].targets;
            if (addends) *addends += (uint64_t)k * proto.plan->n_addends;
            bool bunched = false;
            for (int32_t x : mult) bunched = bunched || x > 1;
            p.flops += (double)proto.plan->n_addends * minors_flops(k, bunched);
        }
        steps.push_back(st);
        act_of_step.push_back(ai);
    }
    if (steps.empty()) return BBFG_OK;
    RunResult rr;
    if (!items.empty()) BBFG_TRY(run_perms(c, w, items, 0, false, nullptr, nullptr, &rr, false));
    p.has_items = !items.empty();

    Layout L;
    const size_t o_steps = L.add(sizeof(CCStep) * steps.size());
    const size_t o_pi = L.add(sizeof(int32_t) * pis.size());
    const size_t o_slot = L.add(sizeof(uint32_t) * std::max<size_t>(1, slots.size()));
    const size_t o_drawn = L.add(sizeof(int32_t) * steps.size());
    const size_t o_wsum = L.add(sizeof(double) * steps.size());
    const size_t o_tv = L.add(sizeof(double) * steps.size());
    BBFG_TRY(w.cc_hmeta.ensure(L.size));
    BBFG_TRY(w.cc_meta.ensure(L.size));
    char* H = w.cc_hmeta.as<char>();
    char* D = w.cc_meta.as<char>();
    std::memcpy(H + o_steps, steps.data(), sizeof(CCStep) * steps.size());
    std::memcpy(H + o_pi, pis.data(), sizeof(int32_t) * pis.size());
    if (!slots.empty()) std::memcpy(H + o_slot, slots.data(), sizeof(uint32_t) * slots.size());
    BBFG_HIP(hipMemcpyAsync(D, H, o_drawn, hipMemcpyHostToDevice, s));
    // the minors' diagnostics follow their nres results (run_perms)
    BBFG_HIP(launch_cc_weights((uint32_t)steps.size(), reinterpret_cast<const CCStep*>(D + o_steps),
                               reinterpret_cast<const int32_t*>(D + o_pi),
                               reinterpret_cast<const uint32_t*>(D + o_slot), w.results.as<double>(),
                               w.results.as<double>() + 2 * nres, reinterpret_cast<int32_t*>(D + o_drawn),
                               reinterpret_cast<double*>(D + o_wsum), reinterpret_cast<double*>(D + o_tv), s));
    BBFG_HIP(hipMemcpyAsync(H + o_drawn, D + o_drawn, L.size - o_drawn, hipMemcpyDeviceToHost, s));
    BBFG_HIP(hipEventRecord(w.done, s));
    p.o_drawn = o_drawn;
    p.o_tv = o_tv;
    p.queued = true;
    return BBFG_OK;
}

int cc_step_end(Workspace& w, std::vector<ActiveSample>& act, CCPending& p, double* kernel_ms, double* flops)
{
    if (!p.queued) return BBFG_OK;
    p.queued = false;
    BBFG_HIP(hipEventSynchronize(w.done));
    if (p.has_items && kernel_ms) {
        float ms = 0.f;
        BBFG_HIP(hipEventElapsedTime(&ms, w.ev0, w.ev1));
        *kernel_ms += ms;
    }
    if (flops) *flops += p.flops;
    const int32_t* drawn = reinterpret_cast<const int32_t*>(w.cc_hmeta.as<char>() + p.o_drawn);
    const double* tv = reinterpret_cast<const double*>(w.cc_hmeta.as<char>() + p.o_tv);
    for (size_t i = 0; i < p.act_of_step.size(); ++i) {
        ActiveSample& a = act[p.act_of_step[i]];
        CCSample& S = a.job->samples[(size_t)a.s];
        S.prefix.push_back(drawn[i]);
        S.tv += tv[i];
        S.k++;
        if (S.k > S.steps) finish_sample(*a.job, a.s);
    }
    return BBFG_OK;
}

int cc_step(Context& c, std::vector<ActiveSample>& act, double* kernel_ms, uint64_t* addends, double* host_s,
            double* wait_s, double* flops)
{
    using Clock = std::chrono::steady_clock;
    const auto t0 = Clock::now();
    CCPending p;
    BBFG_TRY(cc_step_begin(c, c.ws, act, p, addends));
    const auto t1 = Clock::now();
    BBFG_TRY(cc_step_end(c.ws, act, p, kernel_ms, flops));
    if (host_s) *host_s += std::chrono::duration<double>(t1 - t0).count();
    if (wait_s) *wait_s += std::chrono::duration<double>(Clock::now() - t1).count();
    return BBFG_OK;
}

}  // namespace bbfg

using namespace bbfg;

namespace {

// Every sample of a job, in lock-step waves of at most 1024 samples.
int run_job(Context& c, CCJob& job, int32_t* out_occupation, bbfg_info* info)
{
    constexpr int kWaveSamples = 1024;
    double kms = 0.0, fl = 0.0;
    uint64_t adds = 0;
    for (int s0 = 0; s0 < job.n_samples; s0 += kWaveSamples) {
        const int s1 = std::min(job.n_samples, s0 + kWaveSamples);
        std::vector<ActiveSample> act;
        int max_steps = 0;
        for (int s = s0; s < s1; ++s) {
            cc_start_sample(job, s);
            const int st = job.samples[(size_t)s].steps;
            if (st > 0) act.push_back({&job, s});  // an empty sample is finished at its start
            max_steps = std::max(max_steps, st);
        }
        for (int k = 1; k <= max_steps; ++k) BBFG_TRY(cc_step(c, act, &kms, &adds, nullptr, nullptr, &fl));
    }
    std::memcpy(out_occupation, job.out.data(), sizeof(int32_t) * job.out.size());
    if (info) {
        info->kernel_ms = kms;
        info->n_addends = adds;
        info->rel_err_est = job.tv_max;
        info->flops = fl;
    }
    return BBFG_OK;
}

}  // namespace

extern "C" int bs_sample(const bbfg_c128* U, int32_t m, const int32_t* input_occupation, int32_t n_samples,
                         double loss, uint64_t seed, int32_t* out_occupation, bbfg_info* info)
try {
    BBFG_TRY(cc_validate(U, m, input_occupation, n_samples, loss));
    if (n_samples > 0 && !out_occupation) return set_error(BBFG_EINVAL, "out_occupation is NULL");
    if (info) std::memset(info, 0, sizeof *info);
    if (n_samples == 0) return BBFG_OK;
    int64_t n = 0;
    for (int i = 0; i < m; ++i) n += input_occupation[i];
    if (n == 0) {
        std::memset(out_occupation, 0, sizeof(int32_t) * (size_t)n_samples * (size_t)m);
        return BBFG_OK;
    }
    Context* c = nullptr;
    BBFG_TRY(get_context(&c));
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    CCJob job;
    BBFG_TRY(cc_job_init(*c, job, reinterpret_cast<const double*>(U), is_device_ptr(U), m, input_occupation, n_samples,
                         loss, seed));
    return run_job(*c, job, out_occupation, info);
}
BBFG_API_CATCH

extern "C" int bs_sample_extracted(const bbfg_c128* U, int32_t m, const int32_t* input_occupation, int32_t n_samples,
                                   double loss, uint64_t seed, int32_t* out_occupation, bbfg_info* info)
try {
    BBFG_TRY(cc_validate(U, m, input_occupation, n_samples, loss));
    if (n_samples > 0 && !out_occupation) return set_error(BBFG_EINVAL, "out_occupation is NULL");
    if (info) std::memset(info, 0, sizeof *info);
    if (n_samples == 0) return BBFG_OK;
    int64_t n = 0;
    for (int i = 0; i < m; ++i) n += input_occupation[i];
    if (n == 0) {
        std::memset(out_occupation, 0, sizeof(int32_t) * (size_t)n_samples * (size_t)m);
        return BBFG_OK;
    }
    Context* c = nullptr;
    BBFG_TRY(get_context(&c));
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    CCJob job;
    // the job matrix of the ideal experiment (U's m rows); the loss acts on the inputs
    BBFG_TRY(cc_job_init(*c, job, reinterpret_cast<const double*>(U), is_device_ptr(U), m, input_occupation, n_samples,
                         0.0, seed));
    job.keep = 1.0 - loss;
    return run_job(*c, job, out_occupation, info);
}
BBFG_API_CATCH

extern "C" int bs_sample_lossy(const bbfg_c128* T, int32_t m, const int32_t* input_occupation, int32_t n_samples,
                               uint64_t seed, int32_t* out_occupation, bbfg_info* info)
try {
    // the lossy bounds (2m candidate rows)
    BBFG_TRY(cc_validate(T, m, input_occupation, n_samples, 0.5));
    if (n_samples > 0 && !out_occupation) return set_error(BBFG_EINVAL, "out_occupation is NULL");
    std::vector<double> Th(2 * (size_t)m * (size_t)m);
    if (is_device_ptr(T)) {
        BBFG_HIP(hipMemcpy(Th.data(), T, sizeof(double) * Th.size(), hipMemcpyDeviceToHost));
    } else {
        std::memcpy(Th.data(), T, sizeof(double) * Th.size());
    }
    std::vector<double> A;
    double keep = 1.0;
    BBFG_TRY(cc_lossy_job_matrix(Th.data(), m, input_occupation, A, &keep));
    if (info) std::memset(info, 0, sizeof *info);
    if (n_samples == 0) return BBFG_OK;
    int64_t n = 0;
    for (int i = 0; i < m; ++i) n += input_occupation[i];
    if (n == 0) {
        std::memset(out_occupation, 0, sizeof(int32_t) * (size_t)n_samples * (size_t)m);
        return BBFG_OK;
    }
    Context* c = nullptr;
    BBFG_TRY(get_context(&c));
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    CCJob job;
    BBFG_TRY(cc_job_init_matrix(*c, job, A.data(), 2 * m, m, input_occupation, n_samples, seed));
    job.keep = keep;
    return run_job(*c, job, out_occupation, info);
}
BBFG_API_CATCH
