// noalloc.hip -- perm_bbfg without device allocation.
//
// The same single-permanent evaluation as perm_bbfg (same plan, kernels and
// reduction orders, hence the same bits), with every device buffer it needs
// carved out of one file-scope device array instead of hipMalloc'd
// workspaces: the binomial table, the metadata image, the Gray table, the
// staged input, the gathered rows, the unit partials and the results.  The
// array's device address is taken once per device with hipGetSymbolAddress
// (at bbfg_init, or at the first call on that device); host code only ever
// passes that address, never the array's name, to kernels and copies.
//
// Layout of the array (256-byte aligned regions):
//   binomial table | metadata | Gray table | staged A | rows and +-2a rows |
//   unit partials | results and diagnostics
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "kernels.hpp"
#include "runtime.hpp"

namespace bbfg {
namespace {

constexpr size_t kScratchBytes = size_t(2) << 20;
constexpr uint64_t kMaxUnits = 32768;  // unit partials the array holds
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// region offsets and sizes (bytes)
constexpr size_t kOffBinom = 0;
constexpr size_t kBinomBytes = sizeof(double) * kBinomDim * kBinomDim;
constexpr size_t kOffMeta = align256(kOffBinom + kBinomBytes);
constexpr size_t kMetaBytes = 8192;
constexpr size_t kOffTable = align256(kOffMeta + kMetaBytes);
constexpr size_t kTableBytes = sizeof(TabEntry) * 4096;
constexpr size_t kOffA = align256(kOffTable + kTableBytes);
constexpr int kMaxRows = 256;  // rows of A (zero multiplicities included) a host A may have
constexpr size_t kABytes = 16 * size_t(kMaxRows) * size_t(kMaxN);
constexpr size_t kOffArena = align256(kOffA + kABytes);
constexpr size_t kArenaBytes = 16 * 3 * size_t(kMaxN) * size_t(kMaxN);
constexpr size_t kOffPartials = align256(kOffArena + kArenaBytes);
constexpr size_t kPartialBytes = sizeof(double) * kPartialDoubles * kMaxUnits;
constexpr size_t kOffResults = align256(kOffPartials + kPartialBytes);
constexpr size_t kResultBytes = 256;
static_assert(kOffResults + kResultBytes <= kScratchBytes, "scratch layout exceeds the array");

std::mutex g_mu;                        // serialises no-allocation calls (they share the array)
char* g_ptr[kMaxDevices] = {};           // device address of `scratch`, per device
int g_waves[kMaxDevices][kMaxN + 1] = {};  // resident walk wavefronts per CU, per device and n
alignas(256) char g_host_meta[kMetaBytes + kTableBytes];  // host image of metadata + table

// Once per device, with that device current: the array's device address and
// the binomial table in it.  No allocation.
int setup_locked(int dev)
{
    if (g_ptr[dev]) return BBFG_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return set_error(BBFG_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    char* base = static_cast<char*>(p);
    BBFG_HIP(launch_init_binom(reinterpret_cast<double*>(base + kOffBinom), nullptr));
    BBFG_HIP(hipStreamSynchronize(nullptr));
    g_ptr[dev] = base;
    return BBFG_OK;
}

int current_device(int* dev)
{
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(BBFG_EDEVICE, "no HIP device available");
    }
    if (d < 0 || d >= kMaxDevices) return set_error(BBFG_EDEVICE, "device %d beyond the supported %d", d, kMaxDevices);
    *dev = d;
    return BBFG_OK;
}

}  // namespace

int noalloc_setup()
{
    int dev = 0;
    BBFG_TRY(current_device(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    return setup_locked(dev);
}

}  // namespace bbfg

using namespace bbfg;

extern "C" int perm_bbfg_noalloc(const bbfg_c128* A, int32_t n_rows, const int32_t* row_mult, int32_t n_cols,
                                 bbfg_c128* out, bbfg_info* info)
try {
    if (!out) return set_error(BBFG_EINVAL, "out is NULL");
    BBFG_TRY(validate_shape(row_mult, n_rows, n_cols, kMaxN));
    if (n_cols > 0 && !A) return set_error(BBFG_EINVAL, "A is NULL");
    if (info) std::memset(info, 0, sizeof *info);
    hipStream_t s = current_stream();
    const bool out_dev = is_device_ptr(out);
    if (n_cols == 0) {
        const double one[2] = {1.0, 0.0};
        if (info) {
            info->kappa = 1.0;
            info->n_addends = 1;
        }
        if (out_dev) {
            BBFG_HIP(hipMemcpyAsync(out, one, sizeof one, hipMemcpyHostToDevice, s));
            BBFG_HIP(hipStreamSynchronize(s));
        } else {
            std::memcpy(out, one, sizeof one);
        }
        return BBFG_OK;
    }
    int dev = 0;
    BBFG_TRY(current_device(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    BBFG_TRY(setup_locked(dev));
    char* base = g_ptr[dev];

    // the plan perm_bbfg makes: units fill the walk kernel's resident wavefronts
    if (!g_waves[dev][n_cols]) {
        int blocks = 0, ncu = 0;
        BBFG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, walk_single_fn(n_cols, 0), kWave, 0));
        BBFG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        g_waves[dev][n_cols] = std::max(1, blocks) * std::max(1, ncu);
    }
    const uint64_t slots = (uint64_t)g_waves[dev][n_cols];
    PlanParams pp;
    HostPlan P;
    std::string err;
    int rc = build_plan(row_mult, n_rows, n_cols, slots, pp, P, err);
    if (rc != BBFG_OK) return set_error(rc, "%s", err.c_str());
    if (P.units > kMaxUnits) {
        // longer units, so that the partials fit the array (still whole rounds of slots)
        const uint64_t total = (uint64_t)P.groups * P.span;
        const uint64_t rounds = std::max<uint64_t>(1, kMaxUnits / slots);
        pp.l_target = std::max<uint64_t>(pp.l_target, (total + slots * rounds - 1) / (slots * rounds));
        rc = build_plan(row_mult, n_rows, n_cols, slots, pp, P, err);
        if (rc != BBFG_OK) return set_error(rc, "%s", err.c_str());
        if (P.units > kMaxUnits)
            return set_error(BBFG_ERANGE, "%llu work units exceed the no-allocation maximum %llu",
                             (unsigned long long)P.units, (unsigned long long)kMaxUnits);
    }
    const int r = P.r, n = P.n;
    const size_t tab_bytes = sizeof(TabEntry) * P.table->size();
    if (tab_bytes > kTableBytes) return set_error(BBFG_ERANGE, "Gray table beyond the no-allocation maximum");

    // metadata image: descriptor | row records | gather record | source rows | result -> item
    Layout L;
    const size_t o_desc = L.add(sizeof(PermDesc));
    const size_t o_row = L.add(sizeof(RowInfo) * (size_t)r);
    const size_t o_prep = L.add(sizeof(PrepItem));
    const size_t o_src = L.add(sizeof(uint32_t) * (size_t)r);
    const size_t o_ritem = L.add(sizeof(uint32_t));
    if (L.size > kMetaBytes) return set_error(BBFG_ERANGE, "metadata beyond the no-allocation maximum");
    char* H = g_host_meta;
    std::memset(H, 0, L.size);
    char* D = base + kOffMeta;
    double* Astage = reinterpret_cast<double*>(base + kOffA);
    double* arena = reinterpret_cast<double*>(base + kOffArena);
    double* partials = reinterpret_cast<double*>(base + kOffPartials);
    double* results = reinterpret_cast<double*>(base + kOffResults);
    const TabEntry* tab = reinterpret_cast<const TabEntry*>(base + kOffTable);

    const double* src = reinterpret_cast<const double*>(A);
    if (!is_device_ptr(A)) {
        if (n_rows > kMaxRows)
            return set_error(BBFG_ERANGE, "n_rows = %d beyond the no-allocation maximum %d for a host A", n_rows,
                             kMaxRows);
        BBFG_HIP(hipMemcpyAsync(Astage, A, sizeof(bbfg_c128) * (size_t)n_rows * (size_t)n_cols,
                                hipMemcpyHostToDevice, s));
        src = Astage;
    }
    PermDesc& d = *reinterpret_cast<PermDesc*>(H + o_desc);
    d.a_off = 0;
    d.a2_off = (uint64_t)r * n;
    d.tab = tab;
    d.units = P.units;
    d.units_per_group = P.units_per_group;
    d.span = P.span;
    d.n = n;
    d.r = r;
    d.Q = P.Q;
    d.lane_product = P.lane_product;
    d.groups = P.groups;
    d.scale = std::ldexp(1.0, P.scale_log2);
    d.err_coeff = P.err_coeff * 0x1.0p-53;
    d.col_pow = 1;
    d.mag_every = 1;
    std::memcpy(H + o_row, P.rows.data(), sizeof(RowInfo) * (size_t)r);
    PrepItem& q = *reinterpret_cast<PrepItem*>(H + o_prep);
    q.src = src;
    q.ld = (uint32_t)n_cols;
    q.a2_off = d.a2_off;
    q.srcrow_off = 0;
    q.srccol_off = kIdentityCols;
    q.n = n;
    q.r = r;
    uint32_t* hs = reinterpret_cast<uint32_t*>(H + o_src);
    for (int k = 0; k < r; ++k) hs[k] = (uint32_t)P.src_row[(size_t)k];
    std::memcpy(g_host_meta + kMetaBytes, P.table->data(), tab_bytes);

    WalkArgs W;
    std::memset(&W, 0, sizeof W);
    W.descs = reinterpret_cast<const PermDesc*>(D + o_desc);
    W.rowinfo = reinterpret_cast<const RowInfo*>(D + o_row);
    W.a = arena;
    W.a2 = arena;
    W.binom = reinterpret_cast<const double*>(base + kOffBinom);
    W.partials = partials;
    W.total_units = (uint32_t)P.units;
    W.nitem = 1;

    BBFG_HIP(hipMemcpyAsync(D, H, L.size, hipMemcpyHostToDevice, s));
    BBFG_HIP(hipMemcpyAsync(base + kOffTable, g_host_meta + kMetaBytes, tab_bytes, hipMemcpyHostToDevice, s));
    BBFG_HIP(launch_prep(1, s, reinterpret_cast<const PrepItem*>(D + o_prep), reinterpret_cast<const uint32_t*>(D + o_src),
                         nullptr, arena, arena, nullptr, nullptr));
    BBFG_HIP(launch_walk_single(n, 0, (uint32_t)P.units, s, W, 0u));
    BBFG_HIP(launch_finalize(1, s, W.descs, reinterpret_cast<const uint32_t*>(D + o_ritem), partials, results,
                             results + 2));
    double host_res[4];
    BBFG_HIP(hipMemcpyAsync(host_res, results, sizeof host_res, hipMemcpyDeviceToHost, s));
    if (out_dev) BBFG_HIP(hipMemcpyAsync(out, results, 2 * sizeof(double), hipMemcpyDeviceToDevice, s));
    BBFG_HIP(hipStreamSynchronize(s));
    if (!out_dev) std::memcpy(out, host_res, 2 * sizeof(double));
    if (info) {
        info->rel_err_est = host_res[2];
        info->kappa = host_res[3];
        bool mult = false;
        for (int32_t i = 0; i < n_rows; ++i) mult = mult || row_mult[i] > 1;
        info->n_addends = P.n_addends;
        info->n_units = P.units;
        info->flops = (double)P.n_addends * walk_flops(n_cols, mult);
    }
    return BBFG_OK;
}
BBFG_API_CATCH
