/*
 * oracle.c -- plain CPU reference evaluation of the permanent and of
 * boson-sampling probabilities, in double-double arithmetic.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke entry point and the
 * CPU-baseline leg of the benchmark may.  It shares no code, header, table or
 * helper with the GPU library (the two are independent implementations of the
 * same mathematics, so that agreement between them means something).
 *
 * Paper: "High performance Boson Sampling simulation via data-flow engines"
 * (arXiv:2309.07027).  Every routine names the passage it follows.
 *
 * Precision.  The paper's ground truth is a multiple-precision evaluation
 * (Sec. 3.2, "Numerical accuracy").  Here every sum and product is carried in
 * double-double (about 106 significant bits): Knuth's TwoSum, Dekker's
 * FastTwoSum and an FMA-based TwoProd.  Complex numbers are pairs of
 * double-doubles and are multiplied with the plain four-product formula.
 *
 * Matrices are passed as interleaved complex doubles, row-major:
 *   A[2*(i*cols + j)] = Re a_ij,  A[2*(i*cols + j) + 1] = Im a_ij.
 * Complex results are returned as out[4] = {re_hi, re_lo, im_hi, im_lo}.
 *
 * Parallel sums (OpenMP) always split the index range into a FIXED number of
 * contiguous blocks that does not depend on the thread count, and add the
 * block results in block order, so every result is bit-reproducible.
 *
 * Build:  gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared oracle.c -lm
 * (-ffp-contract=off matters: the error-free transformations below rely on
 * every product and sum being rounded exactly as written.)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_VERSION 1
#define NBLOCKS 512 /* fixed block count of every parallel sum */

/* ------------------------------------------------------------------------- */
/* double-double arithmetic                                                   */
/* ------------------------------------------------------------------------- */

typedef struct { double hi, lo; } dd;
typedef struct { dd re, im; } cdd;

static dd dd_make(double x) { dd r; r.hi = x; r.lo = 0.0; return r; }

/* Knuth's TwoSum: s + e == a + b exactly, for any a, b. */
static dd two_sum(double a, double b)
{
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    dd r; r.hi = s; r.lo = e; return r;
}

/* Dekker's FastTwoSum: exact when |a| >= |b| or a == 0. */
static dd fast_two_sum(double a, double b)
{
    double s = a + b;
    double e = b - (s - a);
    dd r; r.hi = s; r.lo = e; return r;
}

/* TwoProd: p + e == a * b exactly (the FMA computes the rounding error). */
static dd two_prod(double a, double b)
{
    double p = a * b;
    double e = fma(a, b, -p);
    dd r; r.hi = p; r.lo = e; return r;
}

static dd dd_add(dd a, dd b)
{
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}

static dd dd_neg(dd a) { a.hi = -a.hi; a.lo = -a.lo; return a; }
static dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

static dd dd_mul(dd a, dd b)
{
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return fast_two_sum(p.hi, p.lo);
}

static dd dd_mul_d(dd a, double b)
{
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return fast_two_sum(p.hi, p.lo);
}

static double dd_to_d(dd a) { return a.hi + a.lo; }

static cdd cdd_zero(void) { cdd z; z.re = dd_make(0.0); z.im = dd_make(0.0); return z; }
static cdd cdd_one(void) { cdd z; z.re = dd_make(1.0); z.im = dd_make(0.0); return z; }
static cdd cdd_from(const double *p) { cdd z; z.re = dd_make(p[0]); z.im = dd_make(p[1]); return z; }

static cdd cdd_add(cdd a, cdd b) { cdd r; r.re = dd_add(a.re, b.re); r.im = dd_add(a.im, b.im); return r; }

/* (a + ib)(c + id) = (ac - bd) + i(ad + bc) */
static cdd cdd_mul(cdd x, cdd y)
{
    cdd r;
    r.re = dd_sub(dd_mul(x.re, y.re), dd_mul(x.im, y.im));
    r.im = dd_add(dd_mul(x.re, y.im), dd_mul(x.im, y.re));
    return r;
}

static cdd cdd_scale_d(cdd a, double s) { cdd r; r.re = dd_mul_d(a.re, s); r.im = dd_mul_d(a.im, s); return r; }

/* a + s * x with s a small integer-valued double; each product is exact in dd. */
static cdd cdd_axpy_d(cdd acc, double s, const double *x)
{
    acc.re = dd_add(acc.re, two_prod(s, x[0]));
    acc.im = dd_add(acc.im, two_prod(s, x[1]));
    return acc;
}

static double cdd_abs_d(cdd a)
{
    return hypot(dd_to_d(a.re), dd_to_d(a.im));
}

static void cdd_store(cdd a, double *out)
{
    out[0] = a.re.hi; out[1] = a.re.lo; out[2] = a.im.hi; out[3] = a.im.lo;
}

/* exact power of two: 2^e */
static double pow2i(int e) { return ldexp(1.0, e); }

/* ------------------------------------------------------------------------- */
/* exported double-double primitives (so the tests can check them against     */
/* exact rational arithmetic)                                                 */
/* ------------------------------------------------------------------------- */

int oracle_version(void) { return ORACLE_VERSION; }

void oracle_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

int oracle_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_dd_add(const double *a, const double *b, double *out)
{
    dd x = {a[0], a[1]}, y = {b[0], b[1]};
    dd r = dd_add(x, y);
    out[0] = r.hi; out[1] = r.lo;
}

void oracle_dd_mul(const double *a, const double *b, double *out)
{
    dd x = {a[0], a[1]}, y = {b[0], b[1]};
    dd r = dd_mul(x, y);
    out[0] = r.hi; out[1] = r.lo;
}

/* ------------------------------------------------------------------------- */
/* block-parallel sum over an index range                                     */
/* ------------------------------------------------------------------------- */

/* Block b of [0, total) is [total*b/NBLOCKS, total*(b+1)/NBLOCKS). */
static uint64_t block_lo(uint64_t total, int b, int nb)
{
    unsigned __int128 t = (unsigned __int128)total * (unsigned)b;
    return (uint64_t)(t / (unsigned)nb);
}

/* ------------------------------------------------------------------------- */
/* Eq. (perm_def): the definition, a sum over all n! permutations.            */
/* ------------------------------------------------------------------------- */

static void brute_rec(int n, const double *A, int row, unsigned used, cdd prod, cdd *acc)
{
    if (row == n) { *acc = cdd_add(*acc, prod); return; }
    for (int j = 0; j < n; ++j) {
        if (used & (1u << j)) continue;
        brute_rec(n, A, row + 1, used | (1u << j),
                  cdd_mul(prod, cdd_from(A + 2 * (row * n + j))), acc);
    }
}

/* perm(A) = sum over sigma in S_n of prod_i a_{i,sigma(i)}  -- Sec. 1, Eq. (perm_def). */
int oracle_perm_bruteforce(int n, const double *A, double *out)
{
    if (n < 0 || n > 12) return -1;
    cdd acc = cdd_zero();
    if (n == 0) acc = cdd_one();
    else brute_rec(n, A, 0, 0u, cdd_one(), &acc);
    cdd_store(acc, out);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Eq. (ryser): perm(A) = (-1)^n sum_{S subset of columns} (-1)^{|S|}          */
/*              prod_i sum_{j in S} a_ij.                                      */
/* Subsets are visited in binary reflected Gray order (Sec. 2: the inner sums */
/* are then updated by one matrix element per step), with the row sums        */
/* recomputed from scratch at the start of every block.                       */
/* ------------------------------------------------------------------------- */

int oracle_perm_ryser(int n, const double *A, double *out)
{
    if (n < 0 || n > 40) return -1;
    if (n == 0) { cdd_store(cdd_one(), out); return 0; }
    const uint64_t total = (uint64_t)1 << n;
    const int nb = total < NBLOCKS ? (int)total : NBLOCKS;
    cdd *part = (cdd *)calloc((size_t)nb, sizeof(cdd));
    if (!part) return -2;

#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < nb; ++b) {
        uint64_t lo = block_lo(total, b, nb), hi = block_lo(total, b + 1, nb);
        cdd rowsum[64];
        cdd acc = cdd_zero();
        for (uint64_t s = lo; s < hi; ++s) {
            uint64_t g = s ^ (s >> 1); /* subset as a bit mask over columns */
            if (s == lo) {
                for (int i = 0; i < n; ++i) {
                    rowsum[i] = cdd_zero();
                    for (int j = 0; j < n; ++j)
                        if (g >> j & 1) rowsum[i] = cdd_add(rowsum[i], cdd_from(A + 2 * (i * n + j)));
                }
            } else {
                int j = __builtin_ctzll(s);       /* the one column whose membership changed */
                double sgn = (g >> j & 1) ? 1.0 : -1.0; /* joined or left S */
                for (int i = 0; i < n; ++i)
                    rowsum[i] = cdd_axpy_d(rowsum[i], sgn, A + 2 * (i * n + j));
            }
            cdd p = cdd_one();
            for (int i = 0; i < n; ++i) p = cdd_mul(p, rowsum[i]);
            int card = __builtin_popcountll(g);
            if ((card + n) & 1) p = cdd_scale_d(p, -1.0);
            acc = cdd_add(acc, p);
        }
        part[b] = acc;
    }
    cdd acc = cdd_zero();
    for (int b = 0; b < nb; ++b) acc = cdd_add(acc, part[b]);
    free(part);
    cdd_store(acc, out);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Eq. (bbfg): perm(A) = 2^{1-n} sum_delta (prod_k delta_k)                   */
/*                       prod_j sum_i delta_i a_ij,  delta_1 = +1.             */
/* Column sums over rows, as the paper chooses (Sec. 2).  Every addend is     */
/* computed from scratch (no Gray code): O(rows*cols) per addend, the most    */
/* accurate form (Sec. 3.2).  The routine accepts any rows x cols shape:      */
/*  - rows == cols: the permanent;                                            */
/*  - rows >= cols + 2: the sum cancels exactly to zero (Sec. 3.2);           */
/*  - padded shapes of App. A.1 (extra columns equal to 1 in the first row   */
/*    and 0 elsewhere) leave the value unchanged.                             */
/* abs_sum (nullable) receives 2^{1-rows} sum |addend| for the conditioning.  */
/* ------------------------------------------------------------------------- */

int oracle_perm_glynn(int rows, int cols, const double *A, double *out, double *abs_sum)
{
    if (rows < 1 || rows > 40 || cols < 0 || cols > 64) return -1;
    const uint64_t total = (uint64_t)1 << (rows - 1);
    const int nb = total < NBLOCKS ? (int)total : NBLOCKS;
    cdd *part = (cdd *)calloc((size_t)nb, sizeof(cdd));
    double *apart = (double *)calloc((size_t)nb, sizeof(double));
    if (!part || !apart) { free(part); free(apart); return -2; }

#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < nb; ++b) {
        uint64_t lo = block_lo(total, b, nb), hi = block_lo(total, b + 1, nb);
        cdd acc = cdd_zero();
        double aacc = 0.0;
        for (uint64_t d = lo; d < hi; ++d) {
            /* bit (i-1) of d set <=> delta_i = -1, for rows i = 1..rows-1 */
            int neg = __builtin_popcountll(d) & 1;
            cdd p = cdd_one();
            for (int j = 0; j < cols; ++j) {
                cdd cs = cdd_zero();
                for (int i = 0; i < rows; ++i) {
                    double di = (i > 0 && (d >> (i - 1) & 1)) ? -1.0 : 1.0;
                    cs = cdd_axpy_d(cs, di, A + 2 * (i * cols + j));
                }
                p = cdd_mul(p, cs);
            }
            if (neg) p = cdd_scale_d(p, -1.0);
            acc = cdd_add(acc, p);
            aacc += cdd_abs_d(p);
        }
        part[b] = acc;
        apart[b] = aacc;
    }
    cdd acc = cdd_zero();
    double aacc = 0.0;
    for (int b = 0; b < nb; ++b) { acc = cdd_add(acc, part[b]); aacc += apart[b]; }
    free(part); free(apart);
    double scale = pow2i(1 - rows);
    cdd_store(cdd_scale_d(acc, scale), out);
    if (abs_sum) *abs_sum = aacc * scale;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Sec. 2.1: Eq. (bbfg) walked in binary reflected Gray-code order.           */
/* Index i in [0, 2^{n-1}) has Gray code g_i = i XOR (i >> 1); bit b of g_i   */
/* is delta_{b+2} (bit 0 -> delta = +1, bit 1 -> delta = -1).  The index      */
/* range is cut into contiguous blocks; each block computes its first column  */
/* sums from scratch, then each step changes the one row given by the lowest  */
/* set bit of i, adding or subtracting twice that row.  The parity of delta   */
/* flips every step.                                                          */
/* Only the indices [first, first + count) are summed (count < 0: all), so a  */
/* bounded sample of the work can be timed.                                   */
/* ------------------------------------------------------------------------- */

int oracle_perm_glynn_gray(int n, const double *A, int64_t first, int64_t count, double *out)
{
    if (n < 1 || n > 48) return -1;
    const uint64_t total_all = (uint64_t)1 << (n - 1);
    uint64_t f = first < 0 ? 0 : (uint64_t)first;
    if (f > total_all) f = total_all;
    uint64_t total = (count < 0 || f + (uint64_t)count > total_all) ? total_all - f : (uint64_t)count;
    const int nb = total == 0 ? 1 : (total < NBLOCKS ? (int)total : NBLOCKS);
    cdd *part = (cdd *)calloc((size_t)nb, sizeof(cdd));
    if (!part) return -2;

#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < nb; ++b) {
        uint64_t lo = f + block_lo(total, b, nb), hi = f + block_lo(total, b + 1, nb);
        cdd cs[64];
        cdd acc = cdd_zero();
        for (uint64_t i = lo; i < hi; ++i) {
            uint64_t g = i ^ (i >> 1);
            if (i == lo) {
                for (int j = 0; j < n; ++j) {
                    cs[j] = cdd_zero();
                    for (int r = 0; r < n; ++r) {
                        double dr = (r > 0 && (g >> (r - 1) & 1)) ? -1.0 : 1.0;
                        cs[j] = cdd_axpy_d(cs[j], dr, A + 2 * (r * n + j));
                    }
                }
            } else {
                int bit = __builtin_ctzll(i);
                /* the bit is now 1: delta went +1 -> -1, subtract 2*row; else add */
                double s = (g >> bit & 1) ? -2.0 : 2.0;
                int r = bit + 1;
                for (int j = 0; j < n; ++j) cs[j] = cdd_axpy_d(cs[j], s, A + 2 * (r * n + j));
            }
            cdd p = cdd_one();
            for (int j = 0; j < n; ++j) p = cdd_mul(p, cs[j]);
            if (__builtin_popcountll(g) & 1) p = cdd_scale_d(p, -1.0);
            acc = cdd_add(acc, p);
        }
        part[b] = acc;
    }
    cdd acc = cdd_zero();
    for (int b = 0; b < nb; ++b) acc = cdd_add(acc, part[b]);
    free(part);
    cdd_store(cdd_scale_d(acc, pow2i(1 - n)), out);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Eq. (bbfgrepeated) with column multiplicities N_j = 1:                     */
/*                                                                           */
/*   perm(A, M) = 2^{1-n} sum_Delta prod_k (-1)^{Delta_k} C(M'_k, Delta_k)    */
/*                 prod_j ( a_pj + sum_k (M'_k - 2 Delta_k) a_kj )            */
/*                                                                           */
/* Rows k = 0..r-1 of the r x n matrix A each stand for M_k identical rows    */
/* (Eq. Deltak), n = sum M_k.  Delta_k counts the -1 signs among row k's     */
/* copies.  One copy of the pivot row p is held at delta = +1 (the first row  */
/* of Eq. bbfg is fixed, Sec. 2.2), so M'_p = M_p - 1 and M'_k = M_k          */
/* otherwise.  Delta runs over the box prod_k [0, M'_k] in plain              */
/* lexicographic (odometer) order -- deliberately not a Gray code -- and      */
/* every addend's column sums are recomputed from scratch.                    */
/*                                                                           */
/* pivot < 0 selects the first row with the smallest nonzero multiplicity.    */
/* Rows with M_k = 0 contribute nothing.  n = 0 gives 1.                      */
/* abs_sum (nullable) receives 2^{1-n} sum |addend|.                          */
/* ------------------------------------------------------------------------- */

/* Binomial coefficients from Pascal's triangle, C(m, k) = C(m-1, k-1) +
 * C(m-1, k) with C(m, 0) = C(m, m) = 1, for 0 <= k <= m <= 64.  Every entry is
 * an exact integer (the largest, C(64, 32) ~ 1.8e18, is below 2^63).  The
 * triangle is filled once when the library is loaded. */
#define PASCAL_ROWS 65
static uint64_t pascal_tri[PASCAL_ROWS][PASCAL_ROWS];

__attribute__((constructor)) static void pascal_fill(void)
{
    for (int row = 0; row < PASCAL_ROWS; ++row) {
        pascal_tri[row][0] = 1;
        for (int col = 1; col < row; ++col)
            pascal_tri[row][col] = pascal_tri[row - 1][col - 1] + pascal_tri[row - 1][col];
        pascal_tri[row][row] = 1;
    }
}

static uint64_t choose(int m, int k)
{
    if (m < 0 || m >= PASCAL_ROWS || k < 0 || k > m) return 0;
    return pascal_tri[m][k];
}

uint64_t oracle_binom(int m, int k) { return choose(m, k); }

static int choose_pivot(int r, const int *M)
{
    int p = -1;
    for (int k = 0; k < r; ++k)
        if (M[k] > 0 && (p < 0 || M[k] < M[p])) p = k;
    return p;
}

int oracle_default_pivot(int r, const int *M) { return choose_pivot(r, M); }

int oracle_perm_generalized(int r, int n, const double *A, const int *M, int pivot,
                            double *out, double *abs_sum)
{
    if (r < 0 || n < 0 || n > 64 || r > 64) return -1;
    int sum = 0;
    for (int k = 0; k < r; ++k) { if (M[k] < 0) return -1; sum += M[k]; }
    if (sum != n) return -1;
    if (n == 0) { cdd_store(cdd_one(), out); if (abs_sum) *abs_sum = 1.0; return 0; }
    if (pivot < 0) pivot = choose_pivot(r, M);
    if (pivot >= r || M[pivot] < 1) return -1;

    int Mp[64];
    uint64_t total = 1;
    for (int k = 0; k < r; ++k) {
        Mp[k] = M[k] - (k == pivot ? 1 : 0);
        total *= (uint64_t)(Mp[k] + 1);
    }
    const int nb = total < NBLOCKS ? (int)total : NBLOCKS;
    cdd *part = (cdd *)calloc((size_t)nb, sizeof(cdd));
    double *apart = (double *)calloc((size_t)nb, sizeof(double));
    if (!part || !apart) { free(part); free(apart); return -2; }

#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < nb; ++b) {
        uint64_t lo = block_lo(total, b, nb), hi = block_lo(total, b + 1, nb);
        int D[64];
        /* lexicographic decode of lo, row 0 the fastest digit */
        uint64_t x = lo;
        for (int k = 0; k < r; ++k) { D[k] = (int)(x % (uint64_t)(Mp[k] + 1)); x /= (uint64_t)(Mp[k] + 1); }
        cdd acc = cdd_zero();
        double aacc = 0.0;
        for (uint64_t idx = lo; idx < hi; ++idx) {
            /* weight prod_k (-1)^{Delta_k} C(M'_k, Delta_k): an exact integer <= 2^{n-1} */
            uint64_t w = 1;
            int parity = 0;
            for (int k = 0; k < r; ++k) { w *= choose(Mp[k], D[k]); parity += D[k]; }
            cdd p = cdd_one();
            for (int j = 0; j < n; ++j) {
                cdd cs = cdd_from(A + 2 * (pivot * n + j));
                for (int k = 0; k < r; ++k) {
                    double c = (double)(Mp[k] - 2 * D[k]);
                    if (c != 0.0) cs = cdd_axpy_d(cs, c, A + 2 * (k * n + j));
                }
                p = cdd_mul(p, cs);
            }
            p = cdd_scale_d(p, (parity & 1) ? -(double)w : (double)w);
            acc = cdd_add(acc, p);
            aacc += cdd_abs_d(p);
            /* odometer increment */
            for (int k = 0; k < r; ++k) {
                if (D[k] < Mp[k]) { D[k]++; break; }
                D[k] = 0;
            }
        }
        part[b] = acc;
        apart[b] = aacc;
    }
    cdd acc = cdd_zero();
    double aacc = 0.0;
    for (int b = 0; b < nb; ++b) { acc = cdd_add(acc, part[b]); aacc += apart[b]; }
    free(part); free(apart);
    double scale = pow2i(1 - n);
    cdd_store(cdd_scale_d(acc, scale), out);
    if (abs_sum) *abs_sum = aacc * scale;
    return 0;
}

/* The other reading of Eq. (bbfgrepeated): every row, the first included,   */
/* runs Delta_k over [0, M_k] (no copy held at +1), with prefactor 2^{-n}.    */
/* Summing over all 2^n sign vectors counts each addend of Eq. (bbfg) twice   */
/* (delta and -delta give the same addend), which the prefactor undoes; the   */
/* two readings must agree.                                                   */
int oracle_perm_generalized_full(int r, int n, const double *A, const int *M, double *out)
{
    if (r < 0 || n < 0 || n > 64 || r > 64) return -1;
    int sum = 0;
    for (int k = 0; k < r; ++k) { if (M[k] < 0) return -1; sum += M[k]; }
    if (sum != n) return -1;
    if (n == 0) { cdd_store(cdd_one(), out); return 0; }
    uint64_t total = 1;
    for (int k = 0; k < r; ++k) total *= (uint64_t)(M[k] + 1);
    int D[64] = {0};
    cdd acc = cdd_zero();
    for (uint64_t idx = 0; idx < total; ++idx) {
        uint64_t w = 1;
        int parity = 0;
        for (int k = 0; k < r; ++k) { w *= choose(M[k], D[k]); parity += D[k]; }
        cdd p = cdd_one();
        for (int j = 0; j < n; ++j) {
            cdd cs = cdd_zero();
            for (int k = 0; k < r; ++k) {
                double c = (double)(M[k] - 2 * D[k]);
                if (c != 0.0) cs = cdd_axpy_d(cs, c, A + 2 * (k * n + j));
            }
            p = cdd_mul(p, cs);
        }
        p = cdd_scale_d(p, (parity & 1) ? -(double)w : (double)w);
        acc = cdd_add(acc, p);
        for (int k = 0; k < r; ++k) {
            if (D[k] < M[k]) { D[k]++; break; }
            D[k] = 0;
        }
    }
    cdd_store(cdd_scale_d(acc, pow2i(-n)), out);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Eq. (ryser) with row multiplicities (the generalized Ryser formula that   */
/* Sec. 2.2 cites).  perm(A) = perm(A^T), so the subsets may run over rows   */
/* instead of columns.  Row k of the r x n matrix A stands for M_k identical */
/* rows; a subset that takes s_k of those copies can do so in C(M_k, s_k)    */
/* ways, all giving the same addend, hence                                   */
/*                                                                           */
/*   perm(A, M) = (-1)^n sum_{s_k in [0, M_k]} (-1)^{s_1 + ... + s_r}         */
/*                 prod_k C(M_k, s_k) prod_j ( sum_k s_k a_kj ).              */
/*                                                                           */
/* The inner sums hold a varying number of matrix elements (the reason the  */
/* paper gives, Sec. 3.2, for Ryser's weaker accuracy).  s runs over the box */
/* in lexicographic order with every inner sum recomputed from scratch.      */
/* abs_sum (nullable) receives sum |addend|.                                  */
/* ------------------------------------------------------------------------- */

int oracle_perm_ryser_generalized(int r, int n, const double *A, const int *M, double *out, double *abs_sum)
{
    if (r < 0 || n < 0 || n > 64 || r > 64) return -1;
    int sum = 0;
    for (int k = 0; k < r; ++k) { if (M[k] < 0) return -1; sum += M[k]; }
    if (sum != n) return -1;
    if (n == 0) { cdd_store(cdd_one(), out); if (abs_sum) *abs_sum = 1.0; return 0; }
    uint64_t total = 1;
    for (int k = 0; k < r; ++k) total *= (uint64_t)(M[k] + 1);
    const int nb = total < NBLOCKS ? (int)total : NBLOCKS;
    cdd *part = (cdd *)calloc((size_t)nb, sizeof(cdd));
    double *apart = (double *)calloc((size_t)nb, sizeof(double));
    if (!part || !apart) { free(part); free(apart); return -2; }

#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < nb; ++b) {
        uint64_t lo = block_lo(total, b, nb), hi = block_lo(total, b + 1, nb);
        int s_cnt[64];
        uint64_t x = lo;
        for (int k = 0; k < r; ++k) { s_cnt[k] = (int)(x % (uint64_t)(M[k] + 1)); x /= (uint64_t)(M[k] + 1); }
        cdd acc = cdd_zero();
        double aacc = 0.0;
        for (uint64_t idx = lo; idx < hi; ++idx) {
            uint64_t ways = 1;
            int picked = 0;
            for (int k = 0; k < r; ++k) { ways *= choose(M[k], s_cnt[k]); picked += s_cnt[k]; }
            cdd p = cdd_one();
            for (int j = 0; j < n; ++j) {
                cdd inner = cdd_zero();
                for (int k = 0; k < r; ++k)
                    if (s_cnt[k]) inner = cdd_axpy_d(inner, (double)s_cnt[k], A + 2 * (k * n + j));
                p = cdd_mul(p, inner);
            }
            p = cdd_scale_d(p, ((picked + n) & 1) ? -(double)ways : (double)ways);
            acc = cdd_add(acc, p);
            aacc += cdd_abs_d(p);
            for (int k = 0; k < r; ++k) {
                if (s_cnt[k] < M[k]) { s_cnt[k]++; break; }
                s_cnt[k] = 0;
            }
        }
        part[b] = acc;
        apart[b] = aacc;
    }
    cdd acc = cdd_zero();
    double aacc = 0.0;
    for (int b = 0; b < nb; ++b) { acc = cdd_add(acc, part[b]); aacc += apart[b]; }
    free(part); free(apart);
    cdd_store(acc, out);
    if (abs_sum) *abs_sum = aacc;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Sec. 4, Eq. (bs_p):  p_U(S -> T) = |perm(U_ST)|^2 / prod_i s_i! t_i!       */
/* U_S takes column i of U s_i times (m x n); U_ST then takes row j of U_S    */
/* t_j times (n x n).  The permanent is the from-scratch Eq. (bbfg) sum.      */
/* Returns -1 on invalid input (sum s != sum t gives probability 0).          */
/* ------------------------------------------------------------------------- */

static double factorial_d(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= (double)i;
    return f;
}

int oracle_bs_prob(int m, const double *U, const int *S, const int *T, double *prob)
{
    int ns = 0, nt = 0;
    for (int i = 0; i < m; ++i) { if (S[i] < 0 || T[i] < 0) return -1; ns += S[i]; nt += T[i]; }
    if (ns != nt) { *prob = 0.0; return 0; }
    int n = ns;
    if (n == 0) { *prob = 1.0; return 0; }
    if (n > 24) return -1;
    int cols[64], rows[64], c = 0, rr = 0;
    for (int i = 0; i < m; ++i) for (int k = 0; k < S[i]; ++k) cols[c++] = i;
    for (int i = 0; i < m; ++i) for (int k = 0; k < T[i]; ++k) rows[rr++] = i;
    double *B = (double *)malloc(sizeof(double) * 2 * (size_t)n * (size_t)n);
    if (!B) return -2;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            const double *u = U + 2 * (rows[a] * m + cols[b]);
            B[2 * (a * n + b)] = u[0];
            B[2 * (a * n + b) + 1] = u[1];
        }
    double out[4];
    int rc = oracle_perm_glynn(n, n, B, out, NULL);
    free(B);
    if (rc) return rc;
    cdd p; p.re.hi = out[0]; p.re.lo = out[1]; p.im.hi = out[2]; p.im.lo = out[3];
    dd a2 = dd_add(dd_mul(p.re, p.re), dd_mul(p.im, p.im));
    double den = 1.0;
    for (int i = 0; i < m; ++i) den *= factorial_d(S[i]) * factorial_d(T[i]);
    *prob = dd_to_d(a2) / den;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Counter-based random numbers: SplitMix64 (G. Steele, D. Lea, C. Flood,     */
/* "Fast splittable pseudorandom number generators", OOPSLA 2014; constants   */
/* as in S. Vigna's public-domain splitmix64).  draw(key, c) is the c-th      */
/* output of the generator seeded with key.                                   */
/* ------------------------------------------------------------------------- */

static uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static uint64_t sm64_draw(uint64_t key, uint64_t c)
{
    return sm64_mix(key + (c + 1) * 0x9E3779B97F4A7C15ULL);
}

uint64_t oracle_splitmix64_draw(uint64_t key, uint64_t c) { return sm64_draw(key, c); }

/* ------------------------------------------------------------------------- */
/* Clifford & Clifford sampling (the sampler of Sec. 4), written from its     */
/* definition.  For one sample:                                               */
/*  1. A = the columns of W picked by the input occupation (column i taken    */
/*     s_i times), in mode order: a rows x n matrix.                          */
/*  2. The columns are put in uniformly random order pi (Fisher-Yates).       */
/*  3. For k = 1..n the k-th output mode r_k is drawn with probability        */
/*     proportional to |perm A[(r_1..r_{k-1}, r), (pi_1..pi_k)]|^2 over all    */
/*     candidate rows r.  The k x k permanent is evaluated directly (rows     */
/*     with multiplicities, Eq. bbfgrepeated) for every candidate.            */
/*  4. The sample is the occupation of the output modes.                      */
/* Lossy sampling (Sec. 4, loss by doubling the modes): W is the 2m x 2m      */
/* unitary [[sqrt(eta) U, sqrt(1-eta) I], [sqrt(1-eta) U, -sqrt(eta) I]]; the */
/* photons enter the first m modes, all 2m modes are sampled and only the     */
/* first m are reported.                                                      */
/*                                                                           */
/* Random numbers for sample s of a job with seed `seed`:                     */
/*   key_s = draw(seed, s);                                                   */
/*   draws c = 0 .. n-2 : Fisher-Yates, i = n-1 down to 1, using draw c =     */
/*                        n-1-i: j = ((x >> 32) * (i+1)) >> 32, swap(pi_i, pi_j) */
/*   draw  c = n-1+(k-1): step k, u = (x >> 11) * 2^-53.                      */
/* Draw rule: weights w_r (rounded to double), total = sum in row order,     */
/* target = u * total, r_k = the first r whose running sum exceeds target;    */
/* if rounding leaves none, the last r with w_r > 0.                          */
/* ------------------------------------------------------------------------- */

static void build_dilation(int m, const double *U, double eta, double *W)
{
    int M2 = 2 * m;
    double se = sqrt(eta), sl = sqrt(1.0 - eta);
    memset(W, 0, sizeof(double) * 2 * (size_t)M2 * (size_t)M2);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            const double *u = U + 2 * (i * m + j);
            W[2 * (i * M2 + j)] = se * u[0];
            W[2 * (i * M2 + j) + 1] = se * u[1];
            W[2 * ((m + i) * M2 + j)] = sl * u[0];
            W[2 * ((m + i) * M2 + j) + 1] = sl * u[1];
        }
    for (int i = 0; i < m; ++i) {
        W[2 * (i * M2 + m + i)] = sl;
        W[2 * ((m + i) * M2 + m + i)] = -se;
    }
}

int oracle_lossy_dilation(int m, const double *U, double eta, double *W)
{
    if (m < 1 || eta < 0.0 || eta > 1.0) return -1;
    build_dilation(m, U, eta, W);
    return 0;
}

/* weights[r] for all `rows` candidates, given the prefix r_1..r_{k-1} (prefix
 * has k-1 entries) and the first k permuted columns.  A is rows x n. */
static int cc_weights(int rows, int n, const double *A, const int *prefix, int k,
                      const int *pi, double *weights)
{
    int cnt[256];
    double *B = (double *)malloc(sizeof(double) * 2 * (size_t)(k) * (size_t)k);
    if (!B) return -2;
    for (int r = 0; r < rows; ++r) {
        /* rows of the k x k matrix: distinct modes among (prefix, r) with counts */
        int modes[64], M[64], nd = 0;
        memset(cnt, 0, sizeof(int) * (size_t)rows);
        for (int t = 0; t < k - 1; ++t) cnt[prefix[t]]++;
        cnt[r]++;
        for (int q = 0; q < rows; ++q)
            if (cnt[q]) { modes[nd] = q; M[nd] = cnt[q]; nd++; }
        for (int a = 0; a < nd; ++a)
            for (int b = 0; b < k; ++b) {
                const double *x = A + 2 * (modes[a] * n + pi[b]);
                B[2 * (a * k + b)] = x[0];
                B[2 * (a * k + b) + 1] = x[1];
            }
        double out[4];
        int rc = oracle_perm_generalized(nd, k, B, M, -1, out, NULL);
        if (rc) { free(B); return rc; }
        cdd p; p.re.hi = out[0]; p.re.lo = out[1]; p.im.hi = out[2]; p.im.lo = out[3];
        weights[r] = dd_to_d(dd_add(dd_mul(p.re, p.re), dd_mul(p.im, p.im)));
    }
    free(B);
    return 0;
}

int oracle_cc_weights(int rows, int n, const double *A, const int *prefix, int k,
                      const int *pi, double *weights)
{
    if (rows < 1 || rows > 256 || n < 1 || n > 40 || k < 1 || k > n) return -1;
    return cc_weights(rows, n, A, prefix, k, pi, weights);
}

static int draw_index(int rows, const double *w, double u)
{
    double total = 0.0;
    for (int r = 0; r < rows; ++r) total += w[r];
    double target = u * total, run = 0.0;
    for (int r = 0; r < rows; ++r) {
        run += w[r];
        if (run > target) return r;
    }
    for (int r = rows - 1; r >= 0; --r) if (w[r] > 0.0) return r;
    return rows - 1;
}

/* Samples of the photons entering the input modes of `src` (rows x ld,
 * row-major; column i is input mode i, i < m): A = the columns picked by the
 * input occupation (rows x n), every one of the `rows` rows a candidate
 * output mode, the occupation of the first m rows reported.  Random numbers
 * as described above. */
static int cc_sample_rows_kept(int rows, int m, const double *src, int ld, const int *input_occ, int n,
                               int n_samples, uint64_t seed, double keep, int *out_occ);

static int cc_sample_rows(int rows, int m, const double *src, int ld, const int *input_occ, int n,
                          int n_samples, uint64_t seed, int *out_occ)
{
    return cc_sample_rows_kept(rows, m, src, ld, input_occ, n, n_samples, seed, 1.0, out_occ);
}

/* As cc_sample_rows, with the uniform part of the loss taken out at the input
 * (Sec. 4): before its steps, sample s keeps each input photon b (the b-th
 * column in input order) with probability `keep`, using draw 2n-1+b of its key
 * (u = (x >> 11) 2^-53, kept when u < keep); the kept photons, in the order pi
 * gives them, are its columns, and it draws one output row per kept photon.
 * keep = 1 draws nothing extra and is the ideal sampler. */
static int cc_sample_rows_kept(int rows, int m, const double *src, int ld, const int *input_occ, int n,
                               int n_samples, uint64_t seed, double keep, int *out_occ)
{
    double *A = (double *)malloc(sizeof(double) * 2 * (size_t)rows * (size_t)(n > 0 ? n : 1));
    double *w = (double *)malloc(sizeof(double) * (size_t)rows);
    if (!A || !w) { free(A); free(w); return -2; }
    int cols[64], c = 0;
    for (int i = 0; i < m; ++i) for (int t = 0; t < input_occ[i]; ++t) cols[c++] = i;
    for (int r = 0; r < rows; ++r)
        for (int b = 0; b < n; ++b) {
            A[2 * (r * n + b)] = src[2 * ((size_t)r * ld + cols[b])];
            A[2 * (r * n + b) + 1] = src[2 * ((size_t)r * ld + cols[b]) + 1];
        }
    int rc = 0;
    for (int s = 0; s < n_samples && rc == 0; ++s) {
        uint64_t key = sm64_draw(seed, (uint64_t)s);
        int pi[64], prefix[64];
        for (int b = 0; b < n; ++b) pi[b] = b;
        for (int i = n - 1; i >= 1; --i) {
            uint64_t x = sm64_draw(key, (uint64_t)(n - 1 - i));
            int j = (int)(((x >> 32) * (uint64_t)(i + 1)) >> 32);
            int t = pi[i]; pi[i] = pi[j]; pi[j] = t;
        }
        int steps = n;
        if (keep < 1.0) {
            int alive[64], kept[64];
            for (int b = 0; b < n; ++b) {
                uint64_t x = sm64_draw(key, (uint64_t)(2 * n - 1 + b));
                alive[b] = (double)(x >> 11) * 0x1.0p-53 < keep;
            }
            steps = 0;
            for (int l = 0; l < n; ++l) if (alive[pi[l]]) kept[steps++] = pi[l];
            for (int l = 0; l < steps; ++l) pi[l] = kept[l];
        }
        for (int k = 1; k <= steps; ++k) {
            rc = cc_weights(rows, n, A, prefix, k, pi, w);
            if (rc) break;
            uint64_t x = sm64_draw(key, (uint64_t)(n - 1 + (k - 1)));
            double u = (double)(x >> 11) * 0x1.0p-53;
            prefix[k - 1] = draw_index(rows, w, u);
        }
        int *o = out_occ + (size_t)s * (size_t)m;
        for (int i = 0; i < m; ++i) o[i] = 0;
        for (int k = 0; k < steps; ++k) if (prefix[k] < m) o[prefix[k]]++;
    }
    free(A); free(w);
    return rc;
}

static int count_photons(int m, const int *input_occ)
{
    int n = 0;
    for (int i = 0; i < m; ++i) { if (input_occ[i] < 0) return -1; n += input_occ[i]; }
    return n;
}

/* out_occ: n_samples x m occupations (int32).  loss in [0,1): 0 = ideal. */
int oracle_cc_sample(int m, const double *U, const int *input_occ, int n_samples,
                     double loss, uint64_t seed, int *out_occ)
{
    if (m < 1 || m > 128 || n_samples < 0 || !(loss >= 0.0 && loss < 1.0)) return -1;
    int n = count_photons(m, input_occ);
    if (n < 0 || n > 24) return -1;
    if (loss == 0.0) return cc_sample_rows(m, m, U, m, input_occ, n, n_samples, seed, out_occ);
    double *W = (double *)malloc(sizeof(double) * 2 * (size_t)(2 * m) * (size_t)(2 * m));
    if (!W) return -2;
    build_dilation(m, U, 1.0 - loss, W);
    int rc = cc_sample_rows(2 * m, m, W, 2 * m, input_occ, n, n_samples, seed, out_occ);
    free(W);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Uniform loss taken out of the interferometer (Sec. 4): a loss that acts   */
/* alike on every mode commutes with U, so it can be applied as a pure-loss  */
/* channel on the input photons before an ideal simulation with U: each     */
/* photon survives with probability 1 - loss, and the survivors are sampled  */
/* on the m modes of U (no doubled modes).  Same law as oracle_cc_sample     */
/* with the same loss; other random numbers.                                 */
int oracle_cc_sample_extracted(int m, const double *U, const int *input_occ, int n_samples,
                               double loss, uint64_t seed, int *out_occ)
{
    if (m < 1 || m > 128 || n_samples < 0 || !(loss >= 0.0 && loss < 1.0)) return -1;
    int n = count_photons(m, input_occ);
    if (n < 0 || n > 24) return -1;
    return cc_sample_rows_kept(m, m, U, m, input_occ, n, n_samples, seed, 1.0 - loss, out_occ);
}

/* Non-uniform loss (Sec. 4): a lossy interferometer is described by a       */
/* matrix T that is no longer unitary, a contraction (T^H T <= I).  With     */
/* the photons entering the first m of 2m modes, the sampled law depends     */
/* only on the first m columns of a 2m x 2m unitary dilation of T, i.e. on   */
/* an isometry V = [T; B] with B^H B = I - T^H T; every such B gives the     */
/* same law on the first m output modes (two choices differ by a unitary    */
/* acting on the unmeasured modes only).  B is taken here as the upper       */
/* triangular Cholesky factor R of I - T^H T (R^H R = I - T^H T, real        */
/* non-negative diagonal; a pivot that rounding leaves in [-1e-10, 0] is     */
/* set to zero together with the rest of its row).  Returns -3 when a pivot  */
/* is below -1e-10, i.e. T is not a contraction.                             */
/* ------------------------------------------------------------------------- */

#define CONTRACTION_TOL 1e-10

static int contraction_isometry(int m, const double *T, double *V)
{
    /* G = I - T^H T, accumulated in double-double */
    double *G = (double *)malloc(sizeof(double) * 2 * (size_t)m * (size_t)m);
    if (!G) return -2;
    for (int j = 0; j < m; ++j)
        for (int k = 0; k < m; ++k) {
            cdd acc = cdd_zero();
            for (int i = 0; i < m; ++i) {
                const double *a = T + 2 * (i * m + j), *b = T + 2 * (i * m + k);
                cdd ca; ca.re = dd_make(a[0]); ca.im = dd_make(-a[1]);
                acc = cdd_add(acc, cdd_mul(ca, cdd_from(b)));
            }
            double re = (j == k ? 1.0 : 0.0) - dd_to_d(acc.re);
            double im = -dd_to_d(acc.im);
            G[2 * (j * m + k)] = re;
            G[2 * (j * m + k) + 1] = im;
        }
    double *R = V + 2 * (size_t)m * (size_t)m; /* rows m .. 2m-1 of V */
    memset(R, 0, sizeof(double) * 2 * (size_t)m * (size_t)m);
    int rc = 0;
    /* Cholesky-Crout, one row of R at a time:
     *   R_jj = sqrt(G_jj - sum_{i<j} |R_ij|^2),
     *   R_jk = (G_jk - sum_{i<j} conj(R_ij) R_ik) / R_jj   (k > j). */
    for (int j = 0; j < m && rc == 0; ++j) {
        double d = G[2 * (j * m + j)];
        for (int i = 0; i < j; ++i) {
            const double *x = R + 2 * (i * m + j);
            d -= x[0] * x[0] + x[1] * x[1];
        }
        if (d < -CONTRACTION_TOL) { rc = -3; break; }
        if (d <= 0.0) continue;
        double rjj = sqrt(d);
        R[2 * (j * m + j)] = rjj;
        for (int k = j + 1; k < m; ++k) {
            double re = G[2 * (j * m + k)], im = G[2 * (j * m + k) + 1];
            for (int i = 0; i < j; ++i) {
                const double *x = R + 2 * (i * m + j), *y = R + 2 * (i * m + k);
                /* conj(x) * y */
                re -= x[0] * y[0] + x[1] * y[1];
                im -= x[0] * y[1] - x[1] * y[0];
            }
            R[2 * (j * m + k)] = re / rjj;
            R[2 * (j * m + k) + 1] = im / rjj;
        }
    }
    free(G);
    if (rc == 0) memcpy(V, T, sizeof(double) * 2 * (size_t)m * (size_t)m);
    return rc;
}

/* V: 2m x m isometry [T; R] (row-major). */
int oracle_contraction_isometry(int m, const double *T, double *V)
{
    if (m < 1 || m > 128) return -1;
    return contraction_isometry(m, T, V);
}

/* The uniform part of the loss of T (Sec. 4): the transmission eta_u such
 * that T = sqrt(eta_u) T' leaves T' a contraction, taken as the Gershgorin
 * bound max_j sum_k |(T^H T)_jk| of the largest eigenvalue of T^H T (exact
 * for T^H T diagonal, as for losses at the inputs or a uniform loss; an upper
 * bound otherwise, so T' is a contraction whenever T is); 1 when the bound
 * reaches 1 (nothing is taken out). */
static double uniform_transmission(int m, const double *T)
{
    double bound = 0.0;
    for (int j = 0; j < m; ++j) {
        double row = 0.0;
        for (int k = 0; k < m; ++k) {
            double re = 0.0, im = 0.0;
            for (int i = 0; i < m; ++i) {
                const double *a = T + 2 * (i * m + j), *b = T + 2 * (i * m + k);
                re += a[0] * b[0] + a[1] * b[1]; /* conj(a) b */
                im += a[0] * b[1] - a[1] * b[0];
            }
            row += sqrt(re * re + im * im);
        }
        if (row > bound) bound = row;
    }
    return bound < 1.0 ? bound : 1.0;
}

/* Clifford & Clifford samples through the lossy interferometer T (m x m
 * contraction).  Its uniform part eta_u (uniform_transmission) is taken out
 * at the input (Sec. 4): each photon survives with probability eta_u, as in
 * oracle_cc_sample_extracted, and the survivors are sampled through
 * T' = T / sqrt(eta_u): the 2m rows of V = [T'; R'] are the candidate output
 * modes, the first m are reported.  Random numbers as in oracle_cc_sample,
 * plus the survival draws of oracle_cc_sample_extracted when eta_u < 1. */
int oracle_cc_sample_lossy(int m, const double *T, const int *input_occ, int n_samples, uint64_t seed,
                           int *out_occ)
{
    if (m < 1 || m > 128 || n_samples < 0) return -1;
    int n = count_photons(m, input_occ);
    if (n < 0 || n > 24) return -1;
    double *V = (double *)malloc(sizeof(double) * 2 * (size_t)(2 * m) * (size_t)m);
    double *Ts = (double *)malloc(sizeof(double) * 2 * (size_t)m * (size_t)m);
    if (!V || !Ts) { free(V); free(Ts); return -2; }
    const double keep = uniform_transmission(m, T);
    const double scale = keep > 0.0 ? 1.0 / sqrt(keep) : 1.0;
    for (size_t i = 0; i < 2 * (size_t)m * (size_t)m; ++i) Ts[i] = T[i] * scale;
    int rc = contraction_isometry(m, Ts, V);
    if (rc == 0) rc = cc_sample_rows_kept(2 * m, m, V, m, input_occ, n, n_samples, seed, keep, out_occ);
    free(V);
    free(Ts);
    return rc;
}

/* eta_u of T, for the tests. */
double oracle_uniform_transmission(int m, const double *T)
{
    if (m < 1 || m > 128) return -1.0;
    return uniform_transmission(m, T);
}
