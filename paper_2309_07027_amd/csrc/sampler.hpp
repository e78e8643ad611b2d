// sampler.hpp -- Clifford & Clifford sampling engine (Sec. 4) shared by
// bs_sample and the serving loop.
#pragma once

#include <cstdint>
#include <deque>
#include <vector>

#include "runtime.hpp"

namespace bbfg {

// SplitMix64 (Steele, Lea & Flood 2014; S. Vigna's constants): the c-th
// output of the generator seeded with `key`.
uint64_t splitmix64_draw(uint64_t key, uint64_t c);

struct CCSample {
    uint64_t key = 0;
    int k = 1;                    // next step (1-based); > steps when finished
    int steps = 0;                // photons sampled (n, or the survivors of an input loss)
    std::vector<int32_t> pi;      // column order
    std::vector<int32_t> prefix;  // drawn output rows r_1 .. r_{k-1}
    double tv = 0.0;              // sum over its steps of the draw-distribution error estimates
};

struct CCJob {
    int m = 0;          // modes reported
    int rows = 0;       // candidate rows (m, or 2m when lossy)
    int n = 0;          // photons
    int n_samples = 0;
    double loss = 0.0;
    double keep = 1.0;  // < 1: uniform loss taken out at the input, each photon kept with this probability
    uint64_t seed = 0;
    std::vector<int32_t> cols;  // input mode of each column (expanded occupation)
    DevBuf A;                   // rows x n complex, device
    DevBuf dev_in;              // U (when given on the host) and cols, device
    PinnedBuf host_in;          // pinned staging of dev_in (stage_pinned)
    std::vector<CCSample> samples;
    int started = 0;
    int finished = 0;
    std::vector<int32_t> out;   // n_samples x m
    double kernel_ms = 0.0;
    uint64_t n_addends = 0;
    // largest tv over the finished samples: an estimate of the total-variation
    // distance between a sample's law as computed and the exact law (each step's
    // estimate from the minors' error estimates, summed over the steps)
    double tv_max = 0.0;
};

struct ActiveSample {
    CCJob* job;
    int s;
};

// Appends the items of one leave-one-column-out walk: the K = proto.plan->n + 1
// columns cols[0..K) (source columns of the matrix of proto), in groups of
// minor_group(K) targets; each group's column map lists its other columns first
// and its targets last.  The items' results follow result index res_first in
// item order; slot[l] receives the result index of the permanent without
// column l.  Column maps are kept alive in `keep`.
void add_minor_items(const PermItem& proto, const int32_t* cols, std::deque<std::vector<int32_t>>& keep,
                     std::vector<PermItem>& items, uint64_t res_first, uint32_t* slot);

// Host validation of sampling arguments (no device work).
int cc_validate(const void* U, int m, const int32_t* occ, int n_samples, double loss);

// Device bytes a job holds while active (its matrices plus a working-set share).
size_t cc_job_footprint(int m, int n, int n_samples, double loss);

// Copies U (host or device) into the job's own device memory and queues the
// build of the job matrix on the current stream (no synchronisation; a host U
// must stay valid until the queued copy has run).  The job's device buffers
// are grow-only: a CCJob can be reused for another job without new
// allocations when it is large enough.
// stage_pinned: the host-side inputs go through job.host_in (pinned), so the
// copies are queued without waiting for work already on the stream.
int cc_job_init(Context& c, CCJob& job, const double* U, bool U_on_device, int m, const int32_t* occ, int n_samples,
                double loss, uint64_t seed, bool stage_pinned = false);

// Non-uniform loss (Sec. 4): the uniform part of T's loss, *keep (the
// Gershgorin bound max_j sum_k |(T^H T)_jk| of T^H T's largest eigenvalue,
// capped at 1: exact for uniform and input losses), is taken out at the input
// (each photon survives with that probability), and the 2m x n job matrix of
// photons entering the input modes of the rest, T' = T / sqrt(*keep) (host,
// row-major complex), is built: the input columns of the isometry [T'; R], R
// the upper-triangular Cholesky factor of I - T'^H T'.  Any B with B^H B =
// I - T'^H T' gives the same law on the first m output modes; R is one.
// Fails with BBFG_EINVAL when T is not a contraction (a pivot of I - T^H T
// below -1e-10).
int cc_lossy_job_matrix(const double* T, int m, const int32_t* occ, std::vector<double>& A, double* keep);

// As cc_job_init, with the job matrix built on the host (rows x n complex,
// e.g. by cc_lossy_job_matrix): rows candidate output modes, the first m
// reported.
int cc_job_init_matrix(Context& c, CCJob& job, const double* A_host, int rows, int m, const int32_t* occ,
                       int n_samples, uint64_t seed, bool stage_pinned = false);

// Draws sample s's column order (Fisher-Yates with SplitMix64) and, when the
// job keeps photons with probability keep < 1, its surviving photons; a sample
// left without photons is finished at once (an all-zero occupation).
void cc_start_sample(CCJob& job, int s);

// One step of every listed sample, in two halves so that a caller can prepare
// another step while this one runs:
//   cc_step_begin queues (in workspace w, on the current stream) all the
//     samples' minors in one batched leave-one-column-out launch, then one
//     weights-and-draw launch and the download of the draws;
//   cc_step_end waits for them and applies the draws.  Finished samples are
//     written to job.out and counted in job.finished.
// Between the two calls w, the samples and their jobs must stay untouched.
struct CCPending {
    std::vector<size_t> act_of_step;  // step i advances act[act_of_step[i]]
    size_t o_drawn = 0;               // offset of the draws in w.cc_hmeta
    size_t o_tv = 0;                  // offset of the steps' error estimates in w.cc_hmeta
    bool has_items = false;           // a minors launch was queued (timed by w.ev0/ev1)
    double flops = 0.0;               // algorithmic flops of the queued minors walks
    bool queued = false;
};
int cc_step_begin(Context& c, Workspace& w, std::vector<ActiveSample>& act, CCPending& p, uint64_t* addends);
// kernel_ms / flops (nullable) accumulate the step's walk time and algorithmic flops.
int cc_step_end(Workspace& w, std::vector<ActiveSample>& act, CCPending& p, double* kernel_ms,
                double* flops = nullptr);

// Both halves back to back in the context's workspace.  host_s / wait_s
// (nullable) accumulate the seconds spent preparing the step on the host and
// waiting for the device.
int cc_step(Context& c, std::vector<ActiveSample>& act, double* kernel_ms, uint64_t* addends,
            double* host_s = nullptr, double* wait_s = nullptr, double* flops = nullptr);

}  // namespace bbfg
