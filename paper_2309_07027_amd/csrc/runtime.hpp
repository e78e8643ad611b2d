// runtime.hpp -- device context, memory, errors and the permanent engine.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <exception>
#include <new>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/bbfg.h"
#include "internal.hpp"
#include "kernels.hpp"
#include "plan.hpp"

namespace bbfg {

// ---- errors (thread-local message) ----------------------------------------
int set_error(int code, const char* fmt, ...);
const char* last_error();
// Algorithmic FP64 flops per addend (an FMA counts 2): the walk of n columns
// (2n column-sum adds, n - 1 complex products, the accumulate, and the weight
// when some M > 1), and a leave-one-column-out walk over K columns (K sums, the
// prefix, suffix and combining products of the K minors, 3(K - 2), the K
// accumulates, and the weight on both product chains when some M > 1).
inline double walk_flops(int n, bool mult) { return 8.0 * n - (mult ? 2.0 : 4.0); }
inline double minors_flops(int K, bool mult) { return 22.0 * K - (mult ? 32.0 : 36.0); }

// Host-side validation of one matrix shape (before any device work).
int validate_shape(const int32_t* mult, int32_t n_rows, int32_t n_cols, int max_n);

#define BBFG_HIP(expr)                                                                              \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return ::bbfg::set_error(BBFG_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Catch clauses of the C entry points (function-try-blocks): no C++ exception
// crosses the C ABI; a failed host allocation is BBFG_ENOMEM.
#define BBFG_API_CATCH                                                                              \
    catch (const std::bad_alloc&) { return ::bbfg::set_error(BBFG_ENOMEM, "host memory allocation failed"); } \
    catch (const std::exception& e_) { return ::bbfg::set_error(BBFG_EDEVICE, "internal error: %s", e_.what()); } \
    catch (...) { return ::bbfg::set_error(BBFG_EDEVICE, "internal error"); }

#define BBFG_TRY(expr)            \
    do {                          \
        int s_ = (expr);          \
        if (s_ != BBFG_OK) return s_; \
    } while (0)

// ---- growable buffers -------------------------------------------------------
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    int ensure(size_t bytes);
    void release();
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

struct PinnedBuf {
    void* p = nullptr;
    size_t cap = 0;
    PinnedBuf() = default;
    PinnedBuf(const PinnedBuf&) = delete;
    PinnedBuf& operator=(const PinnedBuf&) = delete;
    ~PinnedBuf() { release(); }
    int ensure(size_t bytes);
    void release();
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

// Byte layout helper for one upload of several arrays.
struct Layout {
    size_t size = 0;
    size_t add(size_t bytes, size_t align = 256)
    {
        size = (size + align - 1) / align * align;
        const size_t off = size;
        size += bytes;
        return off;
    }
};

// ---- workspaces ----------------------------------------------------------------
// Buffers of one evaluation in flight: the metadata image (pinned host and
// device), gathered rows, unit partials, results, the sampler step's metadata,
// the persistent-launch counter and timing events.  Grow-only and reused; a
// workspace holds one evaluation at a time (the device context has one, the
// sampling server two, so that it can prepare one step while another runs).
struct Workspace {
    DevBuf arena_d, arena_f, meta, partials, results, counter, cc_meta;
    PinnedBuf hmeta, hres, cc_hmeta;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, done = nullptr;
    Workspace() = default;
    Workspace(const Workspace&) = delete;
    Workspace& operator=(const Workspace&) = delete;
    ~Workspace();
    int init();  // events and counter (once, on the current device)
};

// A Gray table resident in device memory.  The entry holds the host table, so
// that its address (the key) cannot be reused by another table while the entry
// exists.  A table is uploaded in stream order by the first evaluation that
// needs it (no host wait: a small copy queued behind a persistent walk would
// wait for the whole walk); until the upload is known to be complete, `ready`
// is the event recorded after it on `stream`, which other streams wait for.
using EventPtr = std::shared_ptr<std::remove_pointer_t<hipEvent_t>>;
struct DevTable {
    TablePtr host;
    const TabEntry* dev = nullptr;
    EventPtr ready;
    hipStream_t stream = nullptr;
};

// ---- per-device context -------------------------------------------------------
struct Context {
    int device = -1;
    int n_cu = 0;
    std::recursive_mutex mu;
    double* binom = nullptr;
    DevBuf staging;
    Workspace ws;
    std::map<std::pair<int, int>, int> occ_single;  // (n, f32) -> waves per CU
    std::map<std::pair<int, int>, int> occ_batch;   // (bucket, kind) -> waves per CU
    std::unordered_map<std::string, std::shared_ptr<const HostPlan>> plans;
    // Gray tables shared between plans (host), and their device copies:
    // bump-allocated in chunks that are never moved while referenced
    TableCache tables;
    std::vector<std::unique_ptr<DevBuf>> tab_chunks;
    size_t tab_chunk = 0, tab_used = 0;  // current chunk, bytes used in it
    // device copy of each host table (keyed by the host table's address)
    std::unordered_map<const void*, DevTable> dev_tables;
    size_t plan_cap = 16384;                   // cached plans before a flush
    size_t table_entry_cap = size_t(4) << 20;  // cached table entries (16 B each) before a flush
    PlanParams params;
    std::map<std::pair<int, int>, uint64_t> batch_L;  // (n, kind) -> tuned unit length
    uint64_t plan_epoch = 0;  // bumped when unit lengths change (plans of earlier calls are stale)
    // the shapes and plans of the last perm_batch: a batch with the same shapes
    // and multiplicities reuses its plans without a lookup per item
    struct BatchMemo {
        uint64_t epoch = ~0ull;
        int f32 = -1;  // the precision argument of the batch
        std::vector<int32_t> n_rows, n_cols, mult;
        std::vector<std::shared_ptr<const HostPlan>> plans;
    } batch_memo;
    // captured batch evaluations, keyed by layout (replayed on repeats)
    std::unordered_map<uint64_t, hipGraphExec_t> graphs;
    std::unordered_set<uint64_t> graph_seen;
    hipStream_t cstream = nullptr;  // capture stream
};

// Unit length used for n-column permanents in batched launches; kind = 0
// (FP64), 1 (FP32) or BBFG_MINORS (leave-one-column-out walks, n = minor size).
constexpr uint64_t kDefaultBatchUnit = 512;
uint64_t batch_unit_length(Context& c, int n, int kind);

// Plans for a single launch (units fill the device) or for batched launches
// (fixed unit length: the split depends on the item's shape only).
enum PlanMode { PLAN_SINGLE = 0, PLAN_BATCH = 1 };

// Context of the current HIP device (created on first use).
int get_context(Context** out);
// Device address of the no-allocation entry point's scratch array on the
// current device, taken once per device (noalloc.hip).
int noalloc_setup();
hipStream_t current_stream();
void set_current_stream(hipStream_t s);

int walk_slots(Context& c, int n, int f32, uint64_t* slots);
// Resident wavefronts per CU of a batch kernel: kind = 0 (FP64), 1 (FP32) or
// kKindMinors (leave-one-column-out walks).
constexpr int kKindMinors = 2;
constexpr int kKindCols = 3;  // uniform column multiplicities
int batch_waves(Context& c, int bucket, int kind, int* waves);
// kind = 0 (FP64), 1 (FP32) or BBFG_MINORS: selects the tuned unit length of
// PLAN_BATCH plans (plans of different kinds are cached separately).
// PLAN_SINGLE plans fill the resident wavefronts of the kernel that runs them:
// the plain walk for n_cols columns, the minors kernel for n_cols + 1 columns
// (kind kKindMinors), or the column-power kernel for kernel_cols distinct
// columns (kind kKindCols).
// ryser: the plan of Eq. ryser with row multiplicities (no pivot, base 0).
int get_plan(Context& c, const int32_t* mult, int n_rows, int n_cols, int kind, int mode,
             std::shared_ptr<const HostPlan>* out, int kernel_cols = 0, bool ryser = false);
// Pool space for a device table of `bytes` bytes (resident until a flush).
int table_reserve(Context& c, size_t bytes, TabEntry** out);
// Caches are bounded (Context::plan_cap, Context::table_entry_cap): past these
// sizes plans, tables and captured graphs are dropped (after the device has
// drained) and rebuilt on demand.
constexpr size_t kTableChunkBytes = size_t(8) << 20;
int flush_plans(Context& c);
// Loads "precision n L" lines written by bbfg_autotune.
int load_autotune_file(Context& c, const char* path);

// Is p device memory (of any device)?
bool is_device_ptr(const void* p);

// ---- permanent engine ----------------------------------------------------------
// One permanent to evaluate.  Its matrix is n_rows x n: row i, column j is the
// complex element src[src_off + row(i) * ld + col(j)] of device memory, with
// row(i) = row_map[i] (or i) and col(j) = col_map[j] (or j).
struct PermItem {
    const double* src = nullptr;
    uint64_t src_off = 0;
    uint32_t ld = 0;
    int n_rows = 0;
    int n = 0;
    const int32_t* mult = nullptr;
    const int32_t* row_map = nullptr;
    const int32_t* col_map = nullptr;
    // 0: perm of the n columns.  G > 0: the matrix has n + 1 columns (col_map
    // lists n + 1) and the item yields the G permanents that each leave out one
    // of its last G columns; the plan is that of the n-column permanents.
    int targets = 0;
    // Column multiplicities: col_pow >= 2 means the matrix has arena_cols
    // distinct columns (col_map lists them when given), each with multiplicity
    // col_pow, arena_cols * col_pow = the plan's n (Eq. bbfgrepeated).
    int col_pow = 0;
    int arena_cols = 0;
    std::shared_ptr<const HostPlan> plan;
};

struct RunResult {
    double kernel_ms = 0.0;  // walk kernel (eager) or whole graph (replay)
    uint64_t units = 0;
    bool graph = false;      // evaluated by replaying a captured graph
};

// Evaluates items (all n >= 1).  The (re, im) results stay in c.results (item
// order; an item with targets = G has G consecutive results) and, when out_host
// is not null, are copied to out_host[2*i]; the diagnostics (err_est, kappa) to
// diag_host[2*i] (for minor items from the sampled magnitude sums, see
// walk_minors_unit).  The device copy of the diagnostics follows the results:
// w.results + 2 * (number of results).  With sync = false nothing is
// copied back and the stream is not synchronised (the caller queues more work
// that reads c.results).  single = true uses the one-permanent launch.
// use_graph = true captures a layout into a hipGraph the second time it is
// seen and replays the graph from then on.
// Runs in workspace w (the context's own by default); the results stay in
// w.results.
int run_perms(Context& c, Workspace& w, std::vector<PermItem>& items, int f32, bool single, double* out_host,
              double* diag_host, RunResult* rr, bool sync = true, bool use_graph = false);
inline int run_perms(Context& c, std::vector<PermItem>& items, int f32, bool single, double* out_host,
                     double* diag_host, RunResult* rr, bool sync = true, bool use_graph = false)
{
    return run_perms(c, c.ws, items, f32, single, out_host, diag_host, rr, sync, use_graph);
}

}  // namespace bbfg
