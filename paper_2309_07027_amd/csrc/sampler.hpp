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
    int k = 1;                    // next step (1-based); > n when finished
    std::vector<int32_t> pi;      // column order
    std::vector<int32_t> prefix;  // drawn output rows r_1 .. r_{k-1}
};

struct CCJob {
    int m = 0;          // modes reported
    int rows = 0;       // candidate rows (m, or 2m when lossy)
    int n = 0;          // photons
    int n_samples = 0;
    double loss = 0.0;
    uint64_t seed = 0;
    std::vector<int32_t> cols;  // input mode of each column (expanded occupation)
    DevBuf A;                   // rows x n complex, device
    std::vector<CCSample> samples;
    int started = 0;
    int finished = 0;
    std::vector<int32_t> out;   // n_samples x m
    double kernel_ms = 0.0;
    uint64_t n_addends = 0;
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

// Copies U (host or device), builds the job matrix on the device.
int cc_job_init(Context& c, CCJob& job, const double* U, bool U_on_device, int m, const int32_t* occ, int n_samples,
                double loss, uint64_t seed);

// Draws sample s's column order (Fisher-Yates with SplitMix64).
void cc_start_sample(CCJob& job, int s);

// Advances every listed sample by one step: all their minors in one batched
// permanent launch, then one weights-and-draw launch.  Finished samples are
// written to job.out and counted in job.finished.
int cc_step(Context& c, std::vector<ActiveSample>& act, double* kernel_ms, uint64_t* addends);

}  // namespace bbfg
