// walk_emu.cpp -- CPU emulation of the permanent kernels, for tests.
//
// Runs the SAME per-lane code as the gfx950 walk kernel (walk_core.hpp, here
// compiled for the host with bounds-checked pointers), one lane at a time, on
// the work split of the host planner (plan.cpp), and then reproduces the
// kernel's wavefront butterfly and the finalize kernel's fixed-order
// double-double sum.  Built with AddressSanitizer/UBSan by the tests.  Because
// every floating-point operation is written out (no contraction), the result
// is expected to match the GPU bit for bit.
//
// stdin : n_rows n slots f32 l_batch minors / n_rows multiplicities / n_rows*n
//         complex entries (re im, hex floats), row-major.  l_batch > 0 plans the
//         item as a batched launch does (fixed unit length), 0 as a single launch.
//         minors = 1: the multiplicities sum to n - 1 and the n leave-one-column-
//         out permanents are formed as the batched minors walk does (FP64).
//         minors = 3: the Ryser formula (Eq. ryser with row multiplicities) on
//         the same walk, FP64.
//         minors = 2: column multiplicities; one more line of n column
//         multiplicities (>= 1) follows the row multiplicities (FP64).  As the
//         library does, equal multiplicities e >= 2 use (prod_j c_j)^e over the
//         distinct columns, other ones the column-expanded matrix.
// stdout: re im rel_err_est kappa units   (hex floats, then an integer), or for
//         minors n lines "re im rel_err_est kappa" (permanent without column l,
//         l = 0 .. n-1)
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "plan.hpp"
#include "walk_core.hpp"

using namespace bbfg;

namespace {

template <int NMIN, int NMAX, typename Real>
void run_unit(const WalkArgs& W, const PermDesc& d, uint32_t u, uint32_t lane, double& r, double& i, double& a)
{
    if constexpr (NMIN <= NMAX) {
        if (d.n == NMIN) walk_unit<NMIN, Real>(W, d, u, lane, r, i, a);
        else run_unit<NMIN + 1, NMAX, Real>(W, d, u, lane, r, i, a);
    }
}

int read_case(int& n_rows, int& n, long long& slots, int& f32, long long& l_batch, int& minors,
              std::vector<int32_t>& M, std::vector<int32_t>& N, std::vector<double>& A)
{
    if (std::scanf("%d %d %lld %d %lld %d", &n_rows, &n, &slots, &f32, &l_batch, &minors) != 6) return 1;
    M.resize((size_t)n_rows);
    for (int i = 0; i < n_rows; ++i)
        if (std::scanf("%d", &M[(size_t)i]) != 1) return 1;
    if (minors == 2) {
        N.resize((size_t)n);
        for (int j = 0; j < n; ++j)
            if (std::scanf("%d", &N[(size_t)j]) != 1) return 1;
    }
    A.resize(2 * (size_t)n_rows * (size_t)n);
    for (size_t i = 0; i < A.size(); ++i)
        if (std::scanf("%la", &A[i]) != 1) return 1;
    return 0;
}

template <int NMIN, int NMAX>
void run_unit_pow(const WalkArgs& W, const PermDesc& d, uint32_t u, uint32_t lane, double& r, double& i, double& a)
{
    if constexpr (NMIN <= NMAX) {
        if (d.n == NMIN) walk_unit<NMIN, double, true>(W, d, u, lane, r, i, a);
        else run_unit_pow<NMIN + 1, NMAX>(W, d, u, lane, r, i, a);
    }
}

// N (optional): the same multiplicity e = N[0] >= 2 for each of the n distinct
// columns; the plan is then that of n * e columns and the walk forms
// (prod_j c_j)^e (FP64 only).
template <typename Real>
int emulate(int n_rows, int n, long long slots, long long l_batch, const std::vector<int32_t>& M,
            const std::vector<double>& A, const std::vector<int32_t>& N = {}, bool ryser = false)
{
    const bool pow = !N.empty();
    const int n_total = pow ? n * N[0] : n;
    const int f32 = sizeof(Real) == 4 ? 1 : 0;
    HostPlan P;
    std::string err;
    PlanParams pp;
    pp.l_batch = (uint64_t)l_batch;
    pp.ryser = ryser;
    int rc = build_plan(M.data(), n_rows, n_total, (uint64_t)slots, pp, P, err);
    if (rc) {
        std::fprintf(stderr, "plan error %d: %s\n", rc, err.c_str());
        return 2;
    }
    if (n == 0) {
        std::printf("%a %a %a %a %d\n", 1.0, 0.0, 0.0, 1.0, 0);
        return 0;
    }
    const int r = P.r;
    // arena exactly as the prep kernel lays it out: r x n rows, then 2r x n +-2a rows
    std::vector<Real> arena(2 * (size_t)r * (size_t)n * 3);
    for (int k = 0; k < r; ++k)
        for (int j = 0; j < n; ++j) {
            const double xr = A[2 * ((size_t)P.src_row[(size_t)k] * n + j)];
            const double xi = A[2 * ((size_t)P.src_row[(size_t)k] * n + j) + 1];
            const size_t da = (size_t)k * n + j;
            const size_t dp = (size_t)r * n + (size_t)(2 * k) * n + j;
            const size_t dm = dp + (size_t)n;
            const Real fr = (Real)xr, fi = (Real)xi;
            arena[2 * da] = fr;
            arena[2 * da + 1] = fi;
            arena[2 * dp] = (Real)2 * fr;
            arena[2 * dp + 1] = (Real)2 * fi;
            arena[2 * dm] = (Real)-2 * fr;
            arena[2 * dm + 1] = (Real)-2 * fi;
        }
    std::vector<double> binom((size_t)kBinomDim * kBinomDim);
    for (int m = 0; m < kBinomDim; ++m)
        for (int k = 0; k < kBinomDim; ++k) {
            double v;
            if (k > m) v = 0.0;
            else if (k == 0 || k == m) v = 1.0;
            else v = binom[(size_t)(m - 1) * kBinomDim + k - 1] + binom[(size_t)(m - 1) * kBinomDim + k];
            binom[(size_t)m * kBinomDim + k] = v;
        }
    PermDesc d;
    std::memset(&d, 0, sizeof d);
    d.a_off = 0;
    d.a2_off = (uint64_t)r * n;
    d.tab = P.table->data();
    d.unit_base = 0;
    d.units = P.units;
    d.units_per_group = P.units_per_group;
    d.mag_every = mag_every_for(P.units_per_group);
    d.span = P.span;
    d.rowinfo_off = 0;
    d.n = n;
    d.r = r;
    d.Q = P.Q;
    d.lane_product = P.lane_product;
    d.groups = P.groups;
    d.scale = std::ldexp(1.0, P.scale_log2);
    d.err_coeff = P.err_coeff * (f32 ? 0x1.0p-24 : 0x1.0p-53);
    d.col_pow = pow ? (uint32_t)N[0] : 1u;

    WalkArgs W;
    std::memset(&W, 0, sizeof W);
    W.rowinfo = P.rows.data();
    W.binom = binom.data();
    if (f32) {
        W.af = reinterpret_cast<const float*>(arena.data());
        W.a2f = W.af;
    } else {
        W.a = reinterpret_cast<const double*>(arena.data());
        W.a2 = W.a;
    }
    emu_clear();
    emu_register(P.rows.data(), sizeof(RowInfo) * P.rows.size());
    emu_register(P.table->data(), sizeof(TabEntry) * P.table->size());
    emu_register(binom.data(), sizeof(double) * binom.size());
    emu_register(arena.data(), sizeof(Real) * arena.size());

    std::vector<double> part((size_t)P.units * kPartialDoubles);
    for (uint64_t u = 0; u < P.units; ++u) {
        ddv sr[kWave], si[kWave];
        double sa[kWave];
        for (uint32_t lane = 0; lane < (uint32_t)kWave; ++lane) {
            double x = 0, y = 0, z = 0;
            if constexpr (sizeof(Real) == 8) {
                if (pow) run_unit_pow<1, kMaxN>(W, d, (uint32_t)u, lane, x, y, z);
                else run_unit<1, kMaxN, Real>(W, d, (uint32_t)u, lane, x, y, z);
            } else {
                run_unit<1, kMaxN, Real>(W, d, (uint32_t)u, lane, x, y, z);
            }
            sr[lane] = {x, 0.0};
            si[lane] = {y, 0.0};
            sa[lane] = z;
        }
        for (int off = 1; off < kWave; off <<= 1) {
            ddv nr[kWave], ni[kWave];
            double na[kWave];
            for (int l = 0; l < kWave; ++l) {
                nr[l] = dd_add(sr[l], sr[l ^ off]);
                ni[l] = dd_add(si[l], si[l ^ off]);
                na[l] = sa[l] + sa[l ^ off];
            }
            for (int l = 0; l < kWave; ++l) {
                sr[l] = nr[l];
                si[l] = ni[l];
                sa[l] = na[l];
            }
        }
        double* p = part.data() + u * kPartialDoubles;
        p[0] = sr[0].hi;
        p[1] = sr[0].lo;
        p[2] = si[0].hi;
        p[3] = si[0].lo;
        p[4] = sa[0];
    }
    constexpr int T = 256;
    std::vector<double> sh(T * 5);
    for (int t = 0; t < T; ++t) {
        ddv r2 = {0.0, 0.0}, i2 = {0.0, 0.0};
        double a2 = 0.0;
        for (uint64_t u = (uint64_t)t; u < P.units; u += T) {
            const double* p = part.data() + u * kPartialDoubles;
            r2 = dd_add(r2, {p[0], p[1]});
            i2 = dd_add(i2, {p[2], p[3]});
            a2 += p[4];
        }
        sh[(size_t)t * 5 + 0] = r2.hi;
        sh[(size_t)t * 5 + 1] = r2.lo;
        sh[(size_t)t * 5 + 2] = i2.hi;
        sh[(size_t)t * 5 + 3] = i2.lo;
        sh[(size_t)t * 5 + 4] = a2;
    }
    for (int s = T / 2; s > 0; s >>= 1)
        for (int t = 0; t < s; ++t) {
            double* m = sh.data() + (size_t)t * 5;
            const double* o = sh.data() + (size_t)(t + s) * 5;
            ddv x = dd_add({m[0], m[1]}, {o[0], o[1]});
            ddv y = dd_add({m[2], m[3]}, {o[2], o[3]});
            m[0] = x.hi;
            m[1] = x.lo;
            m[2] = y.hi;
            m[3] = y.lo;
            m[4] = m[4] + o[4];
        }
    const double re = (sh[0] + sh[1]) * d.scale;
    const double im = (sh[2] + sh[3]) * d.scale;
    const double mag = std::sqrt(re * re + im * im);
    const double absum = sh[4] * d.scale;
    const double kappa = mag > 0.0 ? absum / mag : INFINITY;
    std::printf("%a %a %a %a %llu\n", re, im, kappa * d.err_coeff, kappa, (unsigned long long)P.units);
    return 0;
}

// wavefront double-double butterfly of one value per lane (as the kernel's)
void butterfly(ddv* sr, ddv* si)
{
    for (int off = 1; off < kWave; off <<= 1) {
        ddv nr[kWave], ni[kWave];
        for (int l = 0; l < kWave; ++l) {
            nr[l] = dd_add(sr[l], sr[l ^ off]);
            ni[l] = dd_add(si[l], si[l ^ off]);
        }
        for (int l = 0; l < kWave; ++l) {
            sr[l] = nr[l];
            si[l] = ni[l];
        }
    }
}

// One lane's unit results: sums and magnitude sum per target.
struct LaneSink {
    double *r, *i, *a;
    void sum(int t, double re, double im)
    {
        r[t] = re;
        i[t] = im;
    }
    void mag(int t, double v) { a[t] = v; }
    void no_mag(int t) { a[t] = 0.0; }
};

template <int KMIN, int KMAX>
void run_minor_unit(const WalkArgs& W, const PermDesc& d, uint32_t u, uint32_t lane, double* r, double* i, double* mag)
{
    if constexpr (KMIN <= KMAX) {
        if (d.n == KMIN) {
            LaneSink sink{r, i, mag};
            walk_minors_unit<KMIN, minor_group(KMIN), double>(W, d, u, lane, sink);
        }
        else run_minor_unit<KMIN + 1, KMAX>(W, d, u, lane, r, i, mag);
    }
}

// The batched minors path: targets in groups of minor_group(K), each group a
// walk over its columns reordered (others first, targets last); per target the
// unit partials are reduced as the finalize kernel does.
int emulate_minors(int n_rows, int K, long long slots, long long l_batch, const std::vector<int32_t>& M,
                   const std::vector<double>& A)
{
    HostPlan P;
    std::string err;
    PlanParams pp;
    pp.l_batch = (uint64_t)l_batch;
    int rc = build_plan(M.data(), n_rows, K - 1, (uint64_t)slots, pp, P, err);
    if (rc) {
        std::fprintf(stderr, "plan error %d: %s\n", rc, err.c_str());
        return 2;
    }
    std::vector<double> out(4 * (size_t)K, 0.0);
    if (K == 1) {
        std::printf("%a %a %a %a\n", 1.0, 0.0, 0.0, 1.0);
        return 0;
    }
    const int r = P.r;
    const int G = minor_group(K);
    const int groups = (K + G - 1) / G;
    std::vector<double> binom((size_t)kBinomDim * kBinomDim);
    for (int m = 0; m < kBinomDim; ++m)
        for (int k = 0; k < kBinomDim; ++k) {
            double v;
            if (k > m) v = 0.0;
            else if (k == 0 || k == m) v = 1.0;
            else v = binom[(size_t)(m - 1) * kBinomDim + k - 1] + binom[(size_t)(m - 1) * kBinomDim + k];
            binom[(size_t)m * kBinomDim + k] = v;
        }
    for (int gi = 0; gi < groups; ++gi) {
        const int t0 = std::min(gi * G, K - G);
        std::vector<int> cols;
        for (int l = 0; l < K; ++l)
            if (l < t0 || l >= t0 + G) cols.push_back(l);
        for (int l = t0; l < t0 + G; ++l) cols.push_back(l);
        std::vector<double> arena(2 * (size_t)r * (size_t)K * 3);
        for (int k = 0; k < r; ++k)
            for (int j = 0; j < K; ++j) {
                const size_t src = 2 * ((size_t)P.src_row[(size_t)k] * K + (size_t)cols[(size_t)j]);
                const double xr = A[src], xi = A[src + 1];
                const size_t da = (size_t)k * K + j;
                const size_t dp = (size_t)r * K + (size_t)(2 * k) * K + j;
                const size_t dm = dp + (size_t)K;
                arena[2 * da] = xr;
                arena[2 * da + 1] = xi;
                arena[2 * dp] = 2.0 * xr;
                arena[2 * dp + 1] = 2.0 * xi;
                arena[2 * dm] = -2.0 * xr;
                arena[2 * dm + 1] = -2.0 * xi;
            }
        PermDesc d;
        std::memset(&d, 0, sizeof d);
        d.a2_off = (uint64_t)r * K;
        d.tab = P.table->data();
        d.units = P.units;
        d.units_per_group = P.units_per_group;
        d.mag_every = mag_every_for(P.units_per_group);
        d.span = P.span;
        d.n = K;
        d.r = r;
        d.Q = P.Q;
        d.lane_product = P.lane_product;
        d.groups = P.groups;
        d.scale = std::ldexp(1.0, 1 - (K - 1));
        d.err_coeff = P.err_coeff * 0x1.0p-53;
        d.targets = (uint32_t)G;
        WalkArgs W;
        std::memset(&W, 0, sizeof W);
        W.rowinfo = P.rows.data();
        W.binom = binom.data();
        W.a = arena.data();
        W.a2 = arena.data();
        emu_clear();
        emu_register(P.rows.data(), sizeof(RowInfo) * P.rows.size());
        emu_register(P.table->data(), sizeof(TabEntry) * P.table->size());
        emu_register(binom.data(), sizeof(double) * binom.size());
        emu_register(arena.data(), sizeof(double) * arena.size());
        // partial (unit, target) -> (re hi, re lo, im hi, im lo, magnitude sum)
        std::vector<double> part((size_t)P.units * G * kPartialDoubles);
        for (uint64_t u = 0; u < P.units; ++u) {
            std::vector<double> lr((size_t)kWave * G), li((size_t)kWave * G), lm((size_t)kWave * G);
            for (uint32_t lane = 0; lane < (uint32_t)kWave; ++lane)
                run_minor_unit<2, kMaxN>(W, d, (uint32_t)u, lane, lr.data() + (size_t)lane * G,
                                         li.data() + (size_t)lane * G, lm.data() + (size_t)lane * G);
            for (int t = 0; t < G; ++t) {
                ddv sr[kWave], si[kWave];
                double sa[kWave];
                for (int l = 0; l < kWave; ++l) {
                    sr[l] = {lr[(size_t)l * G + t], 0.0};
                    si[l] = {li[(size_t)l * G + t], 0.0};
                    sa[l] = lm[(size_t)l * G + t];
                }
                butterfly(sr, si);
                for (int off = 1; off < kWave; off <<= 1) {
                    double na[kWave];
                    for (int l = 0; l < kWave; ++l) na[l] = sa[l] + sa[l ^ off];
                    for (int l = 0; l < kWave; ++l) sa[l] = na[l];
                }
                double* p = part.data() + ((size_t)u * G + t) * kPartialDoubles;
                p[0] = sr[0].hi;
                p[1] = sr[0].lo;
                p[2] = si[0].hi;
                p[3] = si[0].lo;
                p[4] = sa[0];
            }
        }
        constexpr int T = 256;
        for (int t = 0; t < G; ++t) {
            if (t0 + t < gi * G) continue;  // owned by the previous group
            std::vector<ddv> shr(T), shi(T);
            std::vector<double> sha(T);
            for (int th = 0; th < T; ++th) {
                ddv a = {0.0, 0.0}, b = {0.0, 0.0};
                double c = 0.0;
                for (uint64_t u = (uint64_t)th; u < P.units; u += T) {
                    const double* p = part.data() + ((size_t)u * G + t) * kPartialDoubles;
                    a = dd_add(a, {p[0], p[1]});
                    b = dd_add(b, {p[2], p[3]});
                    c += p[4];
                }
                shr[(size_t)th] = a;
                shi[(size_t)th] = b;
                sha[(size_t)th] = c;
            }
            for (int sst = T / 2; sst > 0; sst >>= 1)
                for (int th = 0; th < sst; ++th) {
                    shr[(size_t)th] = dd_add(shr[(size_t)th], shr[(size_t)(th + sst)]);
                    shi[(size_t)th] = dd_add(shi[(size_t)th], shi[(size_t)(th + sst)]);
                    sha[(size_t)th] = sha[(size_t)th] + sha[(size_t)(th + sst)];
                }
            const int l = t0 + t;
            const double re = (shr[0].hi + shr[0].lo) * d.scale;
            const double im = (shi[0].hi + shi[0].lo) * d.scale;
            const double mag = std::sqrt(re * re + im * im);
            const double kappa = mag > 0.0 ? sha[0] * d.scale / mag : INFINITY;
            out[4 * (size_t)l] = re;
            out[4 * (size_t)l + 1] = im;
            out[4 * (size_t)l + 2] = kappa * d.err_coeff;
            out[4 * (size_t)l + 3] = kappa;
        }
    }
    for (int l = 0; l < K; ++l)
        std::printf("%a %a %a %a\n", out[4 * (size_t)l], out[4 * (size_t)l + 1], out[4 * (size_t)l + 2],
                    out[4 * (size_t)l + 3]);
    return 0;
}

}  // namespace

int main()
{
    int n_rows = 0, n = 0, f32 = 0, minors = 0;
    long long slots = 0, l_batch = 0;
    std::vector<int32_t> M, N;
    std::vector<double> A;
    if (read_case(n_rows, n, slots, f32, l_batch, minors, M, N, A)) {
        std::fprintf(stderr, "bad input\n");
        return 2;
    }
    if (minors == 1) return emulate_minors(n_rows, n, slots, l_batch, M, A);
    if (minors == 3) return emulate<double>(n_rows, n, slots, l_batch, M, A, {}, true);
    if (minors == 2) {
        bool uniform = true;
        for (int32_t e : N) uniform = uniform && e == N[0];
        if (uniform && N[0] >= 2) return emulate<double>(n_rows, n, slots, l_batch, M, A, N);
        // mixed multiplicities: the column-expanded matrix
        std::vector<double> X;
        int nx = 0;
        for (int32_t e : N) nx += e;
        for (int i = 0; i < n_rows; ++i)
            for (int j = 0; j < n; ++j)
                for (int t = 0; t < N[(size_t)j]; ++t) {
                    X.push_back(A[2 * ((size_t)i * n + j)]);
                    X.push_back(A[2 * ((size_t)i * n + j) + 1]);
                }
        return emulate<double>(n_rows, nx, slots, l_batch, M, X);
    }
    return f32 ? emulate<float>(n_rows, n, slots, l_batch, M, A) : emulate<double>(n_rows, n, slots, l_batch, M, A);
}
