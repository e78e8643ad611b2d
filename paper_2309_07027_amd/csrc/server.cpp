// server.cpp -- continuous-batching boson-sampling server.
//
// The paper scales Clifford & Clifford sampling by running one sampler per
// accelerator and gathering the samples (Sec. 4).  On one GPU the analogue is
// to keep many sampling jobs in flight and to evaluate the current step of all
// of them together: a worker thread admits queued jobs while the device-memory
// budget and the active-job limit allow, keeps every admitted job's matrix and
// sample state resident, and advances the unfinished samples of every active
// job step by step, each step ONE batched leave-one-column-out launch (all
// minors, uneven sizes) and ONE weights-and-draw launch.  The samples are
// split into two halves whose steps alternate on the device, so the host
// prepares one half while the other runs.  Jobs admitted later simply join the
// next step of each half.  A job's samples depend only on its
// own arguments (the per-item work split and the reduction orders are fixed by
// the item's shape), so they are bitwise identical to bs_sample's.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sampler.hpp"

using namespace bbfg;
using Clock = std::chrono::steady_clock;

namespace {

struct SJob {
    uint64_t id = 0;
    std::vector<double> U;  // host copy, m x m complex
    std::vector<double> A;  // lossy-matrix jobs: the 2m x n job matrix (host), else empty
    int m = 0;
    std::vector<int32_t> occ;
    int n_samples = 0;
    double loss = 0.0;
    double keep = 1.0;      // input-loss and lossy-matrix jobs: each photon kept with this probability
    uint64_t seed = 0;
    size_t footprint = 0;
    Clock::time_point t_submit, t_done;
    int state = 0;  // 0 queued, 1 active, 2 done, 3 failed, 4 cancelled
    bool cancel = false;  // cancellation requested while active
    double tv = 0.0;      // the finished job's largest per-sample error estimate
    int err_code = 0;
    std::string err;
    std::unique_ptr<CCJob> cc;
    std::vector<int32_t> out;
    int half = 0;        // pipeline half that advances this job's samples
    double weight = 0;   // its share of a half's work (for balancing)
};

}  // namespace

struct bbfg_server {
    Context* ctx = nullptr;
    int device = 0;
    size_t budget = 0;
    int max_active = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    uint64_t next_id = 1;
    std::deque<std::shared_ptr<SJob>> queue;
    std::vector<std::shared_ptr<SJob>> active;  // worker thread only
    // sampler states of retired jobs, kept for reuse: freeing device memory
    // would wait for the step in flight (worker thread only)
    std::vector<std::unique_ptr<CCJob>> spare;
    std::unordered_map<uint64_t, std::shared_ptr<SJob>> jobs;
    size_t used = 0;
    size_t outstanding = 0;  // queued + active
    bbfg_server_stats st{};
    hipStream_t stream = nullptr;
    int init_error = BBFG_OK;  // the worker could not set up its workspaces
    std::string init_message;

    void run();
    void run_guarded();
    void fail_active(int code, const std::string& msg);
};

void bbfg_server::fail_active(int code, const std::string& msg)
{
    // nothing queued on the stream may still read the jobs' device memory
    (void)hipStreamSynchronize(stream);
    std::lock_guard<std::mutex> lk(mu);
    for (auto& j : active) {
        j->state = 3;
        j->err_code = code;
        j->err = msg;
        j->t_done = Clock::now();
        j->cc.reset();
        used -= j->footprint;
        --outstanding;
    }
    active.clear();
    cv_done.notify_all();
}

// The worker's entry: an exception (a failed host allocation) stops the worker
// and fails every job it holds; later submissions are refused.
void bbfg_server::run_guarded()
{
    int code = BBFG_OK;
    try {
        run();
        return;
    } catch (const std::bad_alloc&) {
        code = BBFG_ENOMEM;
    } catch (...) {
        code = BBFG_EDEVICE;
    }
    fail_active(code, "server worker stopped");
    std::lock_guard<std::mutex> lk(mu);
    init_error = code;
    init_message = "server worker stopped";
    for (auto& j : queue) {
        j->state = 3;
        j->err_code = code;
        j->err = init_message;
        j->t_done = Clock::now();
        --outstanding;
    }
    queue.clear();
    cv_done.notify_all();
}

// Every active job belongs to one of two halves (a new job joins the half with
// less work; a lone job thus runs full-size steps).  The halves alternate:
// while the device runs one half's step, the worker applies the other half's
// draws, retires finished jobs, admits new ones and queues that half's next
// step, so the device does not wait for the host between steps.  Each half has
// its own workspace.
void bbfg_server::run()
{
    (void)hipSetDevice(device);
    set_current_stream(stream);
    struct Half {
        Workspace ws;
        std::vector<ActiveSample> act;
        CCPending pend;
    };
    Half half[2];
    double half_work[2] = {0.0, 0.0};  // weights of the active jobs of each half
    for (Half& h : half) {
        const int rc = h.ws.init();
        if (rc != BBFG_OK) {
            std::lock_guard<std::mutex> lk(mu);
            init_error = rc;
            init_message = last_error();
        }
    }
    int which = 0;
    for (;;) {
        Half& h = half[which];
        const auto t0 = Clock::now();
        int rc = BBFG_OK;
        // 1. the draws of this half's step in flight
        if (h.pend.queued) {
            double wms = 0.0, fl = 0.0;
            rc = cc_step_end(h.ws, h.act, h.pend, &wms, &fl);
            const double dt = std::chrono::duration<double>(Clock::now() - t0).count();
            std::lock_guard<std::mutex> lk(mu);
            st.wait_s += dt;
            st.busy_s += dt;
            st.iterations++;
            st.walk_ms += wms;
            st.flops += fl;
        }
        if (rc != BBFG_OK) {
            half[0].pend.queued = half[1].pend.queued = false;
            fail_active(rc, last_error());
            half_work[0] = half_work[1] = 0.0;
            continue;
        }
        // 2. retire finished jobs, admit queued ones (or sleep when idle)
        std::vector<std::shared_ptr<SJob>> admitted;
        {
            std::unique_lock<std::mutex> lk(mu);
            std::vector<std::shared_ptr<SJob>> keep;
            for (auto& j : active) {
                const bool done = j->cc->n == 0 || j->cc->finished == j->n_samples;
                // a cancelled job leaves with its own half, whose step has just
                // ended (no queued step reads its samples any more)
                const bool cancelled = j->cancel && j->half == which;
                if (!done && !cancelled) {
                    keep.push_back(j);
                    continue;
                }
                if (cancelled) {
                    j->state = 4;
                } else {
                    j->out = j->cc->out;
                    j->tv = j->cc->tv_max;
                    j->state = 2;
                    st.jobs_done++;
                    st.samples_done += (uint64_t)j->n_samples;
                }
                spare.push_back(std::move(j->cc));
                half_work[j->half] -= j->weight;
                j->t_done = Clock::now();
                used -= j->footprint;
                --outstanding;
            }
            if (keep.size() != active.size()) cv_done.notify_all();
            active.swap(keep);
            for (;;) {
                while (!stop && init_error == BBFG_OK && !queue.empty() &&
                       (int)(active.size() + admitted.size()) < max_active) {
                    auto& j = queue.front();
                    const bool empty = active.empty() && admitted.empty();
                    if (!empty && used + j->footprint > budget) break;  // wait for memory to free up
                    used += j->footprint;
                    j->state = 1;
                    admitted.push_back(j);
                    queue.pop_front();
                }
                const bool other_busy = half[which ^ 1].pend.queued;
                if (!active.empty() || !admitted.empty() || other_busy || stop) break;
                if (init_error != BBFG_OK && !queue.empty()) break;
                cv_work.wait(lk);
            }
            if (stop && active.empty() && admitted.empty() && !half[0].pend.queued && !half[1].pend.queued) return;
            const uint64_t na = active.size() + admitted.size();
            if (na > st.max_active) st.max_active = na;
            if (init_error != BBFG_OK) {
                // the worker cannot run steps: fail what is queued
                for (auto& j : queue) {
                    j->state = 3;
                    j->err_code = init_error;
                    j->err = init_message;
                    j->t_done = Clock::now();
                    --outstanding;
                }
                queue.clear();
                cv_done.notify_all();
            }
        }
        // 3. set up admitted jobs, queue this half's next step
        const auto t1 = Clock::now();
        {
            std::lock_guard<std::recursive_mutex> clk(ctx->mu);
            for (auto& j : admitted) {
                if (!spare.empty()) {
                    j->cc = std::move(spare.back());
                    spare.pop_back();
                } else {
                    j->cc = std::make_unique<CCJob>();
                }
                if (!j->A.empty())
                    rc = cc_job_init_matrix(*ctx, *j->cc, j->A.data(), 2 * j->m, j->m, j->occ.data(), j->n_samples,
                                            j->seed, true);
                else
                    rc = cc_job_init(*ctx, *j->cc, j->U.data(), false, j->m, j->occ.data(), j->n_samples, j->loss,
                                     j->seed, true);
                if (rc != BBFG_OK) break;
                j->cc->keep = j->keep;
                for (int s = 0; s < j->n_samples; ++s) cc_start_sample(*j->cc, s);
                // work ~ samples x the addends of the last (largest) steps
                j->weight = (double)j->n_samples * std::ldexp(1.0, std::min(j->cc->n, 60));
                j->half = half_work[1] < half_work[0] ? 1 : 0;
                half_work[j->half] += j->weight;
                std::lock_guard<std::mutex> lk(mu);
                active.push_back(j);
            }
            if (rc == BBFG_OK) {
                h.act.clear();
                for (auto& j : active)
                    if (j->half == which)
                        for (int s = 0; s < j->n_samples; ++s)
                            if (j->cc->n > 0 && j->cc->samples[(size_t)s].k <= j->cc->samples[(size_t)s].steps)
                                h.act.push_back({j->cc.get(), s});
                if (!h.act.empty()) rc = cc_step_begin(*ctx, h.ws, h.act, h.pend, nullptr);
            }
        }
        if (rc != BBFG_OK) {
            {
                std::lock_guard<std::mutex> lk(mu);
                for (auto& j : admitted)
                    if (std::find(active.begin(), active.end(), j) == active.end()) active.push_back(j);
            }
            half[0].pend.queued = half[1].pend.queued = false;
            fail_active(rc, last_error());
            half_work[0] = half_work[1] = 0.0;
            continue;
        }
        {
            const double dt = std::chrono::duration<double>(Clock::now() - t1).count();
            std::lock_guard<std::mutex> lk(mu);
            st.host_s += dt;
            st.busy_s += dt;
        }
        which ^= 1;
    }
}

namespace {

// How a job's loss is simulated.
enum class LossMode { kDilation, kMatrix, kInput };

// Queues a job.  kDilation: the scalar loss by the 2m x 2m dilation;
// kMatrix: U is the m x m lossy interferometer matrix T and the job matrix
// [T; R] is built (and T validated) here; kInput: the scalar loss applied to
// the input photons, survivors sampled with U (bs_sample_extracted).
int submit_job(bbfg_server* srv, const bbfg_c128* U, int32_t m, const int32_t* input_occupation, int32_t n_samples,
               double loss, uint64_t seed, LossMode mode, uint64_t* job_id)
{
    const bool lossy_matrix = mode == LossMode::kMatrix;
    if (!srv || !job_id) return set_error(BBFG_EINVAL, "NULL argument");
    BBFG_TRY(cc_validate(U, m, input_occupation, n_samples, lossy_matrix ? 0.5 : loss));
    auto j = std::make_shared<SJob>();
    j->m = m;
    j->U.resize(2 * (size_t)m * (size_t)m);
    if (is_device_ptr(U)) {
        BBFG_HIP(hipMemcpy(j->U.data(), U, sizeof(double) * j->U.size(), hipMemcpyDeviceToHost));
    } else {
        std::memcpy(j->U.data(), U, sizeof(double) * j->U.size());
    }
    if (lossy_matrix) {
        BBFG_TRY(cc_lossy_job_matrix(j->U.data(), m, input_occupation, j->A, &j->keep));
        j->U.clear();
    }
    j->occ.assign(input_occupation, input_occupation + m);
    int n = 0;
    for (int i = 0; i < m; ++i) n += input_occupation[i];
    j->n_samples = n_samples;
    j->loss = mode == LossMode::kDilation ? loss : 0.0;
    if (mode == LossMode::kInput) j->keep = 1.0 - loss;  // kMatrix: set with the job matrix above
    j->seed = seed;
    j->footprint = cc_job_footprint(m, n, n_samples, lossy_matrix ? 0.5 : j->loss);
    j->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->init_error != BBFG_OK) return set_error(srv->init_error, "%s", srv->init_message.c_str());
    j->id = srv->next_id++;
    srv->jobs[j->id] = j;
    srv->queue.push_back(j);
    srv->outstanding++;
    srv->st.jobs_submitted++;
    if (srv->queue.size() > srv->st.max_queued) srv->st.max_queued = srv->queue.size();
    *job_id = j->id;
    srv->cv_work.notify_one();
    return BBFG_OK;
}

}  // namespace

extern "C" {

int bs_server_create(size_t hbm_budget_bytes, int32_t max_active_jobs, bbfg_server** srv)
try {
    if (!srv) return set_error(BBFG_EINVAL, "srv is NULL");
    if (max_active_jobs < 1) return set_error(BBFG_EINVAL, "max_active_jobs < 1");
    Context* c = nullptr;
    BBFG_TRY(get_context(&c));
    auto s = std::make_unique<bbfg_server>();
    s->ctx = c;
    s->device = c->device;
    s->max_active = max_active_jobs;
    if (hbm_budget_bytes == 0) {
        size_t freeb = 0, total = 0;
        BBFG_HIP(hipMemGetInfo(&freeb, &total));
        hbm_budget_bytes = total / 4;
    }
    s->budget = hbm_budget_bytes;
    BBFG_HIP(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
    bbfg_server* raw = s.get();
    s->worker = std::thread([raw] { raw->run_guarded(); });
    *srv = s.release();
    return BBFG_OK;
}
BBFG_API_CATCH

int bs_server_submit(bbfg_server* srv, const bbfg_c128* U, int32_t m, const int32_t* input_occupation,
                     int32_t n_samples, double loss, uint64_t seed, uint64_t* job_id)
try {
    return submit_job(srv, U, m, input_occupation, n_samples, loss, seed, LossMode::kDilation, job_id);
}
BBFG_API_CATCH

int bs_server_submit_extracted(bbfg_server* srv, const bbfg_c128* U, int32_t m, const int32_t* input_occupation,
                               int32_t n_samples, double loss, uint64_t seed, uint64_t* job_id)
try {
    return submit_job(srv, U, m, input_occupation, n_samples, loss, seed, LossMode::kInput, job_id);
}
BBFG_API_CATCH

int bs_server_submit_lossy(bbfg_server* srv, const bbfg_c128* T, int32_t m, const int32_t* input_occupation,
                           int32_t n_samples, uint64_t seed, uint64_t* job_id)
try {
    return submit_job(srv, T, m, input_occupation, n_samples, 0.0, seed, LossMode::kMatrix, job_id);
}
BBFG_API_CATCH

int bs_server_poll(bbfg_server* srv, uint64_t job_id, int32_t* out_occupation, double* latency_s, double* err_est)
try {
    if (!srv) return set_error(BBFG_EINVAL, "srv is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(job_id);
    if (it == srv->jobs.end()) return set_error(BBFG_ENOTFOUND, "unknown job %llu", (unsigned long long)job_id);
    auto j = it->second;
    if (j->state == 0 || j->state == 1) return set_error(BBFG_EBUSY, "job %llu not finished", (unsigned long long)job_id);
    if (j->state == 3) {
        srv->jobs.erase(it);
        return set_error(j->err_code ? j->err_code : BBFG_EDEVICE, "job failed: %s", j->err.c_str());
    }
    if (j->state == 4) {
        srv->jobs.erase(it);
        return set_error(BBFG_ECANCELED, "job %llu was cancelled", (unsigned long long)job_id);
    }
    if (j->n_samples > 0 && !out_occupation) return set_error(BBFG_EINVAL, "out_occupation is NULL");
    if (j->n_samples > 0) std::memcpy(out_occupation, j->out.data(), sizeof(int32_t) * j->out.size());
    if (latency_s) *latency_s = std::chrono::duration<double>(j->t_done - j->t_submit).count();
    if (err_est) *err_est = j->tv;
    srv->jobs.erase(it);
    return BBFG_OK;
}
BBFG_API_CATCH

int bs_server_cancel(bbfg_server* srv, uint64_t job_id)
try {
    if (!srv) return set_error(BBFG_EINVAL, "srv is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(job_id);
    if (it == srv->jobs.end()) return set_error(BBFG_ENOTFOUND, "unknown job %llu", (unsigned long long)job_id);
    auto j = it->second;
    if (j->state == 0) {
        // still queued: it never reaches the device
        auto q = std::find(srv->queue.begin(), srv->queue.end(), j);
        if (q != srv->queue.end()) srv->queue.erase(q);
        j->state = 4;
        j->t_done = Clock::now();
        --srv->outstanding;
        srv->st.jobs_cancelled++;
        srv->cv_done.notify_all();
    } else if (j->state == 1) {
        // active: the worker retires it at the end of its half's current step
        if (!j->cancel) srv->st.jobs_cancelled++;
        j->cancel = true;
    } else {
        // finished (or failed) and not polled yet: its result is dropped
        srv->jobs.erase(it);
    }
    return BBFG_OK;
}
BBFG_API_CATCH

int bs_server_drain(bbfg_server* srv)
try {
    if (!srv) return set_error(BBFG_EINVAL, "srv is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [srv] { return srv->outstanding == 0; });
    return BBFG_OK;
}
BBFG_API_CATCH

int bs_server_stats(bbfg_server* srv, bbfg_server_stats* out)
try {
    if (!srv || !out) return set_error(BBFG_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->st;
    return BBFG_OK;
}
BBFG_API_CATCH

int bs_server_destroy(bbfg_server* srv)
try {
    if (!srv) return set_error(BBFG_EINVAL, "srv is NULL");
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv_work.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    if (srv->stream) (void)hipStreamDestroy(srv->stream);
    delete srv;
    return BBFG_OK;
}
BBFG_API_CATCH

}  // extern "C"
