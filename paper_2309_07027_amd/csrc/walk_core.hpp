// walk_core.hpp -- per-lane core of the generalized BB/FG walk
// (arXiv:2309.07027, Eq. bbfgrepeated walked as in Sec. 2.1/2.2).
//
// This header is compiled twice:
//   * by hipcc for gfx950 (walk.hip): uniform tables are read through the
//     constant address space, so the compiler turns them into scalar loads and
//     SGPR operands;
//   * by a host C++ compiler for the CPU emulation used in tests: the same code
//     runs one lane at a time with bounds-checked pointers.
// Floating-point operations are spelled out (explicit fused multiply-adds, the
// sources are built with -ffp-contract=off), so both builds round identically.
#pragma once

#include <cstddef>
#include <cstdint>

#include "internal.hpp"

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define BBFG_FN __device__ __forceinline__
namespace bbfg {
template <typename T>
using kptr = const __attribute__((address_space(4))) T*;
template <typename T>
BBFG_FN kptr<T> kconst(const T* p)
{
    return (kptr<T>)p;
}
BBFG_FN uint32_t uniform_u32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
}  // namespace bbfg
#else
#define BBFG_FN inline
#include "emu_ptr.hpp"
#endif

namespace bbfg {

// ---------------------------------------------------------------------------
// double-double helpers (Knuth TwoSum, Dekker FastTwoSum)
// ---------------------------------------------------------------------------
struct ddv {
    double hi, lo;
};

BBFG_FN ddv dd_two_sum(double a, double b)
{
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}

BBFG_FN ddv dd_fast(double a, double b)
{
    double s = a + b;
    return {s, b - (s - a)};
}

BBFG_FN ddv dd_add(ddv a, ddv b)
{
    ddv s = dd_two_sum(a.hi, b.hi);
    ddv t = dd_two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = dd_fast(s.hi, s.lo);
    s.lo += t.lo;
    return dd_fast(s.hi, s.lo);
}

// fused multiply-add in the precision of the operands
BBFG_FN float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
BBFG_FN double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

// complex product (a_r + i a_i)(b_r + i b_i): two products, two fused
template <typename Real>
BBFG_FN void cmul(Real ar, Real ai, Real br, Real bi, Real& cr, Real& ci)
{
    const Real t0 = ai * bi;
    const Real t1 = ai * br;
    cr = fmar(ar, br, -t0);
    ci = fmar(ar, bi, t1);
}

// ---------------------------------------------------------------------------
// product of N complex column sums: four independent chains, then a tree
// ---------------------------------------------------------------------------
template <int N, typename Real>
BBFG_FN void cprod(const Real* re, const Real* im, Real& pr, Real& pi)
{
    constexpr int C = N >= 12 ? 4 : (N >= 4 ? 2 : 1);
    Real cr[C], ci[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        cr[c] = re[c];
        ci[c] = im[c];
    }
#pragma unroll
    for (int j = C; j < N; ++j) {
        const int c = j % C;
        const Real t0 = ci[c] * im[j];
        const Real t1 = ci[c] * re[j];
        const Real nr = fmar(cr[c], re[j], -t0);
        const Real ni = fmar(cr[c], im[j], t1);
        cr[c] = nr;
        ci[c] = ni;
    }
#pragma unroll
    for (int s = 1; s < C; s *= 2) {
#pragma unroll
        for (int c = 0; c + s < C; c += 2 * s) {
            const Real t0 = ci[c] * ci[c + s];
            const Real t1 = ci[c] * cr[c + s];
            const Real nr = fmar(cr[c], cr[c + s], -t0);
            const Real ni = fmar(cr[c], ci[c + s], t1);
            cr[c] = nr;
            ci[c] = ni;
        }
    }
    pr = cr[0];
    pi = ci[0];
}

// z^e for a uniform integer e >= 1 by binary powering (most significant bit
// first): floor(log2 e) squarings and popcount(e) - 1 multiplies.
template <typename Real>
BBFG_FN void cpow_uint(Real& zr, Real& zi, uint32_t e)
{
    const Real br = zr, bi = zi;
    int top = 31;
    while (top > 0 && !((e >> top) & 1u)) --top;
    for (int b = top - 1; b >= 0; --b) {
        const Real t0 = zi * zi;
        const Real t1 = zr * zi;
        const Real sr = fmar(zr, zr, -t0);
        const Real si = t1 + t1;
        zr = sr;
        zi = si;
        if ((e >> b) & 1u) {
            const Real u0 = zi * bi;
            const Real u1 = zi * br;
            const Real nr = fmar(zr, br, -u0);
            const Real ni = fmar(zr, bi, u1);
            zr = nr;
            zi = ni;
        }
    }
}

// (x / stride) % radix for a 64-bit x; 32-bit arithmetic when x fits.
BBFG_FN uint32_t digit_of(uint64_t x, uint32_t stride, uint32_t radix)
{
    if ((x >> 32) == 0) {
        const uint32_t x32 = (uint32_t)x;
        return (x32 / stride) % radix;
    }
    return (uint32_t)((x / stride) % radix);
}

template <typename Real>
struct RowsOf;
template <>
struct RowsOf<double> {
    static BBFG_FN const double* a(const WalkArgs& A) { return A.a; }
    static BBFG_FN const double* a2(const WalkArgs& A) { return A.a2; }
};
template <>
struct RowsOf<float> {
    static BBFG_FN const float* a(const WalkArgs& A) { return A.af; }
    static BBFG_FN const float* a2(const WalkArgs& A) { return A.a2f; }
};

// Column sums at block h, position t, for the lane with lane index lane_idx;
// also the lane's weight for its LANE and HIGH digits:
// w = prod (-1)^Delta C(M', Delta).
template <int N, typename Real>
BBFG_FN void seed(const WalkArgs& A, const PermDesc& d, uint32_t lane_idx, uint64_t h, uint32_t t, Real* re,
                  Real* im, double& w)
{
    kptr<RowInfo> ri = kconst(A.rowinfo + d.rowinfo_off);
    kptr<Real> rows = kconst(RowsOf<Real>::a(A) + 2 * d.a_off);
    kptr<double> binom = kconst(A.binom);
#pragma unroll
    for (int j = 0; j < N; ++j) {
        re[j] = Real(0);
        im[j] = Real(0);
    }
    w = 1.0;
    for (int k = 0; k < d.r; ++k) {
        RowInfo x;
        x.base = ri[k].base;
        x.kind = ri[k].kind;
        x.radix = ri[k].radix;
        x.stride = ri[k].stride;
        x.mp = ri[k].mp;
        uint32_t delta = 0;
        if (x.kind == ROW_LANE) {
            delta = (lane_idx / x.stride) % x.radix;
        } else if (x.kind == ROW_HIGH) {
            delta = digit_of(h, x.stride, x.radix);
        } else if (x.kind == ROW_LOW) {
            const uint32_t dg = (t / x.stride) % x.radix;
            const uint32_t q = t / (x.stride * x.radix);
            delta = (q & 1u) ? (x.radix - 1u - dg) : dg;
        }
        if (x.kind == ROW_LANE || x.kind == ROW_HIGH) {
            const double b = binom[x.mp * kBinomDim + (int)delta];
            w *= (delta & 1u) ? -b : b;
        }
        const Real coef = (Real)(x.base - 2 * (int)delta);
        kptr<Real> row = rows + 2 * (size_t)k * N;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            re[j] = fmar(coef, (Real)row[2 * j], re[j]);
            im[j] = fmar(coef, (Real)row[2 * j + 1], im[j]);
        }
    }
}

// One work unit of permanent d, for one lane: the lane's sum of weighted
// addends and the sum of their magnitudes (|re| + |im|).  POW: each of the N
// columns has multiplicity d.col_pow, the product is (prod_j c_j)^col_pow.
template <int N, typename Real, bool POW = false>
BBFG_FN void walk_unit(const WalkArgs& A, const PermDesc& d, uint32_t u_local, uint32_t lane, double& out_r,
                       double& out_i, double& out_a)
{
    const uint32_t upg = (uint32_t)d.units_per_group;
    const uint32_t g = u_local / upg;
    const uint32_t part = u_local - g * upg;
    const uint64_t base = d.span / upg;
    const uint32_t rem = (uint32_t)(d.span - base * upg);
    uint64_t lin = (uint64_t)part * base + (part < rem ? part : rem);
    const uint64_t lin1 = lin + base + (part < rem ? 1u : 0u);
    uint32_t lane_idx = g * kWave + lane;
    const bool valid = lane_idx < d.lane_product;
    if (!valid) lane_idx = 0;

    kptr<TabEntry> tab = kconst(d.tab);
    kptr<Real> a2 = kconst(RowsOf<Real>::a2(A) + 2 * d.a2_off);
    const uint32_t cpow = POW ? uniform_u32(d.col_pow) : 1u;
    const uint32_t Q = d.Q;

    double accr = 0.0, acci = 0.0, acca = 0.0;
    Real re[N], im[N];
    while (lin < lin1) {
        const uint64_t h = lin / Q;
        const uint32_t t0 = (uint32_t)(lin - h * Q);
        const uint64_t bend = (h + 1) * (uint64_t)Q;
        const uint32_t t1 = (uint32_t)(((lin1 < bend) ? lin1 : bend) - h * Q);
        double w;
        seed<N, Real>(A, d, lane_idx, h, t0, re, im, w);
        if (!valid) w = 0.0;
        double sr, si, sa;
        {
            Real pr, pi;
            cprod<N, Real>(re, im, pr, pi);
            if constexpr (POW) cpow_uint<Real>(pr, pi, cpow);
            const double s = tab[t0].s;
            sr = s * (double)pr;
            si = s * (double)pi;
            sa = __builtin_fabs(s) * (__builtin_fabs((double)pr) + __builtin_fabs((double)pi));
        }
        for (uint32_t t = t0 + 1; t < t1; ++t) {
            const uint32_t rowi = uniform_u32(tab[t].row);
            const double s = tab[t].s;
            kptr<Real> row = a2 + 2 * (size_t)rowi * N;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                re[j] += row[2 * j];
                im[j] += row[2 * j + 1];
            }
            Real pr, pi;
            cprod<N, Real>(re, im, pr, pi);
            if constexpr (POW) cpow_uint<Real>(pr, pi, cpow);
            sr = __builtin_fma(s, (double)pr, sr);
            si = __builtin_fma(s, (double)pi, si);
            sa = __builtin_fma(__builtin_fabs(s), __builtin_fabs((double)pr) + __builtin_fabs((double)pi), sa);
        }
        accr = __builtin_fma(w, sr, accr);
        acci = __builtin_fma(w, si, acci);
        acca = __builtin_fma(__builtin_fabs(w), sa, acca);
        lin += (uint64_t)(t1 - t0);
    }
    out_r = accr;
    out_i = acci;
    out_a = acca;
}

// Leave-one-column-out products of one addend, accumulated: with c_j the K
// column sums and T = K - G, for every target t < G
//   acc[t] += ws * prod_{j != T + t} c_j
// = ws * (prod_{j < T} c_j) * (prod_{i < t} c_{T+i}) * (prod_{t < i < G} c_{T+i}):
// one product of the leading sums, prefix products over the targets, and a
// running suffix product (about K + 2G complex products for G permanents).
// The weight ws enters the first prefix product, so each target's update is
// one complex multiply-accumulate of its prefix and suffix products: four
// fused multiply-adds instead of a complex product and a weighted add.
template <int K, int G, typename Real>
BBFG_FN void minors_accumulate(const Real* re, const Real* im, double ws, double* accr, double* acci)
{
    constexpr int T = K - G;
    Real pr[G], pim[G];
    if constexpr (T > 0) {
        Real cr, ci;
        cprod<T, Real>(re, im, cr, ci);
        pr[0] = (Real)(ws * (double)cr);
        pim[0] = (Real)(ws * (double)ci);
    } else {
        pr[0] = (Real)ws;
        pim[0] = Real(0);
    }
#pragma unroll
    for (int t = 1; t < G; ++t) cmul<Real>(pr[t - 1], pim[t - 1], re[T + t - 1], im[T + t - 1], pr[t], pim[t]);
    Real sr = Real(1), si = Real(0);
#pragma unroll
    for (int t = G - 1; t >= 0; --t) {
        if (t == G - 1) {
            accr[t] = accr[t] + (double)pr[t];
            acci[t] = acci[t] + (double)pim[t];
        } else {
            const double ar = (double)pr[t], ai = (double)pim[t], br = (double)sr, bi = (double)si;
            accr[t] = __builtin_fma(-ai, bi, __builtin_fma(ar, br, accr[t]));
            acci[t] = __builtin_fma(ai, br, __builtin_fma(ar, bi, acci[t]));
        }
        if (t > 0) {
            if (t == G - 1) {
                sr = re[T + t];
                si = im[T + t];
            } else {
                Real nr, ni;
                cmul<Real>(sr, si, re[T + t], im[T + t], nr, ni);
                sr = nr;
                si = ni;
            }
        }
    }
}

// One work unit of a leave-one-column-out walk (d.targets == G): the lane's
// sums over its addends of w(Delta) * prod_{j != K-G+t} c_j(Delta), t < G, i.e.
// of the permanents (size K - 1) that each drop one of the last G columns.
// The walk over the rows is the one of walk_unit; the signed weight w * s is
// an integer below 2^53 (a product of binomials), hence exact.
// After the walk, sink.sum(t, re_t, im_t) hands over target t's sums.  Then
// units whose index in the lane group is a multiple of d.mag_every call
// sink.mag(t, a_t) with the lane's estimate of the sum of |addend| of target t
// over its positions in this unit and the d.mag_every - 1 units after it: the
// modulus of the addend at the unit's last position,
//   |w s| prod_{j != K-G+t} |c_j|,
// times the unit's number of positions and the number of units it stands for
// (one sample per lane, from column sums seeded afresh at that position, so
// the walk loop carries no extra work or registers); the other units call
// sink.no_mag(t).  The passes over the targets are separate loops, each small
// enough to be unrolled in full.
template <int K, int G, typename Real, typename Sink>
BBFG_FN void walk_minors_unit(const WalkArgs& A, const PermDesc& d, uint32_t u_local, uint32_t lane, Sink& sink)
{
    constexpr int T = K - G;
    const uint32_t upg = (uint32_t)d.units_per_group;
    const uint32_t g = u_local / upg;
    const uint32_t part = u_local - g * upg;
    const uint64_t base = d.span / upg;
    const uint32_t rem = (uint32_t)(d.span - base * upg);
    const uint64_t lin0 = (uint64_t)part * base + (part < rem ? part : rem);
    const uint64_t lin1 = lin0 + base + (part < rem ? 1u : 0u);
    uint64_t lin = lin0;
    uint32_t lane_idx = g * kWave + lane;
    const bool valid = lane_idx < d.lane_product;
    if (!valid) lane_idx = 0;

    kptr<TabEntry> tab = kconst(d.tab);
    kptr<Real> a2 = kconst(RowsOf<Real>::a2(A) + 2 * d.a2_off);
    const uint32_t Q = d.Q;

    double out_r[G], out_i[G];
#pragma unroll
    for (int t = 0; t < G; ++t) {
        out_r[t] = 0.0;
        out_i[t] = 0.0;
    }
    Real re[K], im[K];
    while (lin < lin1) {
        const uint64_t h = lin / Q;
        const uint32_t t0 = (uint32_t)(lin - h * Q);
        const uint64_t bend = (h + 1) * (uint64_t)Q;
        const uint32_t t1 = (uint32_t)(((lin1 < bend) ? lin1 : bend) - h * Q);
        double w;
        seed<K, Real>(A, d, lane_idx, h, t0, re, im, w);
        if (!valid) w = 0.0;
        for (uint32_t t = t0; t < t1; ++t) {
            if (t > t0) {
                const uint32_t rowi = uniform_u32(tab[t].row);
                kptr<Real> row = a2 + 2 * (size_t)rowi * K;
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    re[j] += row[2 * j];
                    im[j] += row[2 * j + 1];
                }
            }
            const double ws = w * tab[t].s;
            minors_accumulate<K, G, Real>(re, im, ws, out_r, out_i);
        }
        lin += (uint64_t)(t1 - t0);
    }
#pragma unroll
    for (int t = 0; t < G; ++t) sink.sum(t, out_r[t], out_i[t]);
    const uint32_t every = d.mag_every;
    if (part % every != 0) {
#pragma unroll
        for (int t = 0; t < G; ++t) sink.no_mag(t);
        return;
    }
    // a sampled unit stands for itself and the unsampled ones after it
    const uint32_t reps = (upg - part < every) ? upg - part : every;
    // the column sums at the unit's last position, seeded afresh: keeping the
    // walk's own ones alive past the loop costs the loop registers
    const uint64_t hl = (lin1 - 1) / Q;
    const uint32_t tl = (uint32_t)(lin1 - 1 - hl * Q);
    double w;
    seed<K, Real>(A, d, lane_idx, hl, tl, re, im, w);
    if (!valid) w = 0.0;
    // moduli |c_j| in re[] (im[] is free after this), then each target's
    // leave-one-out product of moduli from prefix products (kept in im[]) and a
    // running suffix product: no division, so zero column sums are harmless
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const double x = (double)re[j], y = (double)im[j];
        re[j] = (Real)__builtin_sqrt(__builtin_fma(x, x, y * y));
    }
    double lead = (double)(lin1 - lin0) * (double)reps * __builtin_fabs(w * tab[tl].s);
#pragma unroll
    for (int j = 0; j < T; ++j) lead *= (double)re[j];
    im[T] = (Real)lead;
#pragma unroll
    for (int t = 1; t < G; ++t) im[T + t] = (Real)((double)im[T + t - 1] * (double)re[T + t - 1]);
    double suffix = 1.0;
#pragma unroll
    for (int t = G - 1; t >= 0; --t) {
        sink.mag(t, (double)im[T + t] * suffix);
        suffix *= (double)re[T + t];
    }
}

}  // namespace bbfg
