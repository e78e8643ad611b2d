/*
 * bbfg.h -- C ABI of the MI355X (gfx950) generalized BB/FG permanent library.
 *
 * Method: G. Morse et al., "High performance Boson Sampling simulation via
 * data-flow engines" (arXiv:2309.07027).
 *   - Eq. (bbfg): the Balasubramanian-Bax-Franklin-Glynn formula with column
 *     sums over rows (Sec. 2).
 *   - Eq. (Deltak) / Eq. (bbfgrepeated): rows repeated M_k times collapse to
 *     one row whose sign vector is summarised by Delta_k = number of -1 signs,
 *     weighted by C(M_k, Delta_k) (Sec. 2.2).
 *   - Sec. 2.1 / 2.2: the addends are walked in (n-ary) reflected Gray-code
 *     order, one row changing per step, in independent contiguous chunks whose
 *     column sums are recomputed at the chunk start.
 *   - Sec. 4 / Eq. (bs_p): boson-sampling probabilities are squared permanents;
 *     the Clifford & Clifford sampler and loss by mode doubling sit on top.
 *
 * Conventions shared by every entry point
 *   - Complex numbers are bbfg_c128 (two doubles, real then imaginary), the
 *     memory layout of std::complex<double>, numpy complex128 and
 *     torch.complex128.
 *   - A matrix argument is ROW-MAJOR: element (i, j) of an R x C matrix is at
 *     index i*C + j.  Rows are output modes, columns are input modes (Sec. 2).
 *   - Pointers documented "host or device" may point to host memory or to
 *     device memory of the current HIP device; the library finds out which
 *     with hipPointerGetAttributes and copies what it needs.  All other
 *     pointers are host memory.
 *   - The caller owns every buffer passed in, including outputs.  The library
 *     keeps no reference to them after the call returns.
 *   - Every call is synchronous: results are in place when it returns.  The
 *     library's device work runs on the stream set with bbfg_set_stream (the
 *     null stream by default), so it is ordered after earlier work the caller
 *     queued on that stream.
 *   - Every function returns 0 (BBFG_OK) or a negative bbfg_status; on error
 *     bbfg_last_error() describes the failure (thread-local string).  Argument
 *     errors are detected on the host before any device work.
 *   - Calls from several host threads are serialised per device by the
 *     library; server handles are not re-entrant.
 */
#ifndef BBFG_H
#define BBFG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BBFG_VERSION 1
/* Largest number of columns (photons) accepted by the FP64 path. */
#define BBFG_MAX_N 48
/* Largest number of columns accepted by the FP32 path. */
#define BBFG_MAX_N_FP32 24

typedef enum {
    BBFG_OK = 0,
    BBFG_EINVAL = -1,   /* bad argument: null pointer, sum(row_mult) != n_cols, negative count ... */
    BBFG_ERANGE = -2,   /* size beyond the supported maximum */
    BBFG_ENOMEM = -3,   /* device or pinned host allocation failed */
    BBFG_EDEVICE = -4,  /* HIP runtime error (no device, launch failure, ...) */
    BBFG_EBUSY = -5,     /* server job not finished yet */
    BBFG_ENOTFOUND = -6, /* unknown server job id */
    BBFG_ECANCELED = -7  /* server job cancelled before it finished */
} bbfg_status;

/* BBFG_MINORS names the batched leave-one-column-out walks (FP64) in the
 * autotuner calls and bbfg_walk_occupancy; BBFG_COLS names the column-power
 * kernel in bbfg_walk_occupancy only; BBFG_RYSER selects, in perm_batch, the
 * FP64 Ryser formula over the same walk (the accuracy comparison of Sec. 3.2). */
typedef enum { BBFG_FP64 = 0, BBFG_FP32 = 1, BBFG_MINORS = 2, BBFG_COLS = 3, BBFG_RYSER = 4 } bbfg_precision;

typedef struct {
    double re, im;
} bbfg_c128;

/* Per-result diagnostics. */
typedef struct {
    double rel_err_est;  /* estimated relative error of the result: kappa * u * (n + sqrt(Q)) */
    double kappa;        /* (sum |addend|) / |sum of addends|: conditioning of the sum */
    uint64_t n_addends;  /* number of distinct addends C' = prod_k (M'_k + 1) (Sec. 2.2) */
    uint64_t n_units;    /* independent work units (one wavefront each) */
    double kernel_ms;    /* device time of the walk kernel, from HIP events on the library stream */
    double flops;        /* algorithmic FP64 flops of the call's walks (an FMA counts 2): C' F per
                          * permanent with F = 8n - 4 (all M = 1) or 8n - 2; per leave-one-column-out
                          * addend over K columns F = 22K - 36 (all M = 1) or 22K - 32 */
} bbfg_info;

/* Thread-local description of the last error (never NULL). */
const char *bbfg_last_error(void);

/* Library version (BBFG_VERSION). */
int bbfg_version(void);

/* Initialise the library on the current HIP device (optional: every entry
 * point initialises lazily).  Errors: BBFG_EDEVICE. */
int bbfg_init(void);

/* Bounds of the per-device caches: plans (work splits, keyed by multiplicities
 * and unit length) and Gray tables (16 bytes per entry, resident in device
 * memory).  Past either bound the caches and the captured batch graphs are
 * dropped, after the device has finished all queued work, and rebuilt on
 * demand; results do not depend on the bounds.  0 restores a default (16384
 * plans, 4 Mi entries = 64 MiB of tables). */
int bbfg_set_cache_limits(uint64_t max_plans, uint64_t max_table_entries);

/* Stream for the calling thread's subsequent calls (a hipStream_t, NULL = the
 * null stream).  The stream must stay valid while it is set. */
int bbfg_set_stream(void *hip_stream);

/*
 * perm_bbfg -- generalized BB/FG permanent, Eq. (bbfgrepeated) with column
 * multiplicities N_j = 1, in FP64.
 *
 *   perm(A, M) = 2^{1-n} sum_Delta prod_k (-1)^{Delta_k} C(M'_k, Delta_k)
 *                         prod_j sum_k (M'_k - 2 Delta_k) a_kj   (+ the fixed row)
 *
 * i.e. the permanent of the n x n matrix obtained by repeating row k of A
 * row_mult[k] times.  One copy of a row with the smallest multiplicity is held
 * at sign +1 (the fixed first row of Eq. bbfg, Sec. 2.2).
 *
 *   A        [in]  n_rows x n_cols complex matrix, row-major, host or device.
 *                  One row per distinct output mode.
 *   n_rows   [in]  number of rows of A, >= 0.
 *   row_mult [in]  n_rows int32 multiplicities M_k >= 0 (host).  Rows with
 *                  M_k = 0 are ignored.  sum_k M_k must equal n_cols.
 *   n_cols   [in]  n (number of photons), 0 <= n <= BBFG_MAX_N.  n = 0 gives 1.
 *   out      [out] one bbfg_c128, host or device.
 *   info     [out] nullable, host.
 *
 * Result: column sums and products in FP64, re-seeded at every work-unit and
 * Gray-block start; per-unit partials reduced across the wavefront and across
 * units in double-double, then scaled by 2^{1-n} exactly.
 * Errors: BBFG_EINVAL (null A/out with n > 0, negative multiplicity, sum
 * mismatch), BBFG_ERANGE (n_cols > BBFG_MAX_N), BBFG_ENOMEM, BBFG_EDEVICE.
 */
int perm_bbfg(const bbfg_c128 *A, int32_t n_rows, const int32_t *row_mult, int32_t n_cols,
              bbfg_c128 *out, bbfg_info *info);

/*
 * perm_ryser -- the same permanent by Eq. (ryser) with row multiplicities, in
 * FP64 over the same walk, for the accuracy comparison of Sec. 3.2 (Ryser's
 * inner sums hold a varying number of matrix elements, so its addends span a
 * wider range of magnitudes than those of Eq. bbfg):
 *
 *   perm(A, M) = (-1)^n sum_{s_k in [0, M_k]} (-1)^{sum s} prod_k C(M_k, s_k)
 *                          prod_j sum_k s_k a_kj
 *
 * (subsets of the row copies; perm(A) = perm(A^T), so rows serve as well as
 * the columns of Eq. ryser).  The walk has no pivot row: prod_k (M_k + 1)
 * addends, 2^n for M = 1, twice those of perm_bbfg.  Every addend's column
 * sums are walked as -2 sum_k s_k a_kj (an exact power-of-two scaling), the
 * result is 2^{-n} times the walk's sum, and info->rel_err_est is the same
 * estimate kappa * u * (n + sqrt(Q)) with Ryser's own kappa.
 * Arguments and errors as perm_bbfg; BBFG_ERANGE also when the sum needs more
 * than 2^32 work units (n = 48 with all M = 1).
 */
int perm_ryser(const bbfg_c128 *A, int32_t n_rows, const int32_t *row_mult, int32_t n_cols,
               bbfg_c128 *out, bbfg_info *info);

/*
 * perm_bbfg_noalloc -- perm_bbfg for callers that cannot allocate device
 * memory (tight serving loops, code that must not call hipMalloc).  Same
 * arguments, plan, kernels and result bits as perm_bbfg; every device buffer
 * it uses (binomial table, metadata, Gray table, staged host A, gathered rows,
 * unit partials, results) lives in one file-scope device array of 2 MiB per
 * device, which stays allocated until the process ends.  It calls no
 * hipMalloc/hipFree or other device-allocating routine (host planning uses
 * ordinary heap memory).  bbfg_init takes the array's address on the current
 * device; a first call on a device without it does so itself.
 *
 * Limits: n_cols <= BBFG_MAX_N (else BBFG_ERANGE); a host A has at most 256
 * rows (BBFG_ERANGE beyond); the walk is split into at most 32768 units
 * (longer units for the largest sums).  info->kernel_ms is not measured (0).
 * Calls are serialised inside the process (they share the array); the call is
 * synchronous, so nothing of it overlaps the next call.
 * Errors: as perm_bbfg.
 */
int perm_bbfg_noalloc(const bbfg_c128 *A, int32_t n_rows, const int32_t *row_mult, int32_t n_cols,
                      bbfg_c128 *out, bbfg_info *info);

/*
 * perm_batch -- many generalized permanents of uneven sizes in one persistent
 * launch (the batched evaluation of App. A.4, generalised to unequal shapes and
 * multiplicities).
 *
 *   batch            number of permanents, >= 0.
 *   A_packed         all matrices, host or device; matrix b (n_rows[b] x
 *                    n_cols[b], row-major) starts at element A_offset[b].
 *   A_offset         batch int64 element offsets (host).
 *   n_rows, n_cols   batch int32 shapes (host).
 *   row_mult_packed  int32 multiplicities (host); those of matrix b start at
 *                    row_mult_offset[b] (batch int64 offsets, host).
 *   precision        BBFG_FP64, BBFG_FP32 (column sums and products in
 *                    FP32, accumulation in FP64/double-double; every n_cols[b]
 *                    <= BBFG_MAX_N_FP32), or BBFG_RYSER (FP64, the Ryser
 *                    formula as perm_ryser evaluates it).
 *   out              batch bbfg_c128 results, host or device.
 *   rel_err_est      nullable, batch doubles (host): per-result error estimate.
 *
 * Each item's result depends only on that item (its work split is a function of
 * its shape and the tuned unit length), so it is bitwise identical whatever
 * else is in the batch; it agrees with perm_bbfg to the stated error, not
 * necessarily bit for bit (perm_bbfg splits a lone permanent to fill the
 * device).
 * Errors: as perm_bbfg, per item.
 */
int perm_batch(int32_t batch, const bbfg_c128 *A_packed, const int64_t *A_offset,
               const int32_t *n_rows, const int32_t *row_mult_packed, const int64_t *row_mult_offset,
               const int32_t *n_cols, int32_t precision, bbfg_c128 *out, double *rel_err_est);

/*
 * perm_bbfg_cols -- the generalized permanent with row AND column
 * multiplicities (Eq. bbfgrepeated): the permanent of the n x n matrix in which
 * row i of A appears row_mult[i] times and column j col_mult[j] times,
 *   2^{1-n} sum_Delta w(Delta) prod_j (column sum j)^{N_j}.
 * A repeated column's sum is formed and updated once per addend and enters the
 * product N_j times, instead of N_j identical sums of the expanded matrix.
 *
 *   A         n_rows x n_cols complex (distinct columns), row-major, host or device.
 *   row_mult  n_rows int32 (host), >= 0.
 *   col_mult  n_cols int32 (host), >= 0; sum(col_mult) = sum(row_mult) = n
 *             <= BBFG_MAX_N.  Zero rows and columns are dropped.
 *   out, info as perm_bbfg (FP64, double-double reduction, error estimate).
 *
 * n = 0 gives 1.  Errors: EINVAL (NULL pointer, negative multiplicity, sums
 * differ), ERANGE (n > BBFG_MAX_N), ENOMEM/EDEVICE.
 */
int perm_bbfg_cols(const bbfg_c128 *A, int32_t n_rows, const int32_t *row_mult, int32_t n_cols,
                   const int32_t *col_mult, bbfg_c128 *out, bbfg_info *info);

/*
 * perm_minors -- every leave-one-column-out permanent of one matrix, from one
 * joint walk: the minors of the Laplace expansion that the Clifford & Clifford
 * step of Sec. 4 needs for all candidate output modes at once.  All minors
 * share the rows, so one walk over the Delta box of Eq. bbfgrepeated (rows
 * with multiplicities) forms the n_cols column sums once per addend and every
 * product that leaves one column out (prefix and suffix products).
 *
 *   A         n_rows x n_cols complex, row-major, host or device.
 *   row_mult  n_rows int32 multiplicities (host), sum = n_cols - 1.
 *   n_cols    1 <= n_cols <= BBFG_MAX_N.
 *   out       n_cols bbfg_c128, host or device:
 *             out[l] = perm(A without column l, row_mult).
 *   rel_err_est  nullable, n_cols doubles (host): estimated relative error of
 *             out[l], kappa_l * u * (n + sqrt(Q)) with kappa_l the sum of
 *             |addend| of minor l over |out[l]|.  The sum of |addend| is
 *             estimated from one sample per lane in about 32 work units per
 *             group of 64 lanes (the addend's modulus at the unit's last
 *             position times the positions it stands for): within a factor of
 *             8 of the exact kappa_l in the cases tested.
 *
 * FP64 with double-double reduction.  n_cols = 1 gives the empty permanent 1.
 * The walk is split to fill the device (as perm_bbfg splits a lone permanent),
 * so values may differ in the last bits from the minors the sampler forms.
 * Errors: EINVAL (NULL pointer, negative multiplicity, sum != n_cols - 1),
 * ERANGE (n_cols > BBFG_MAX_N), ENOMEM/EDEVICE.
 */
int perm_minors(const bbfg_c128 *A, int32_t n_rows, const int32_t *row_mult, int32_t n_cols, bbfg_c128 *out,
                double *rel_err_est);

/* Device time (ms) of the last perm_batch or perm_minors on this thread: the
 * walk kernel when launched directly, the whole replayed graph otherwise. */
double perm_batch_last_kernel_ms(void);

/* 1 when the last perm_batch on this thread replayed a captured hipGraph.  A
 * launch layout (metadata sizes, launch shapes, buffer addresses) seen for the
 * second time is captured into a graph -- upload, gather, persistent walk, finalize,
 * download -- and replayed whenever it recurs. */
int perm_batch_last_was_graph(void);

/*
 * Batched launches (perm_batch, and the minors of bs_sample and the server)
 * split each permanent into work units of L Gray positions per lane, with L a
 * function of the column count only, so an item's result does not depend on the
 * other items of the batch.  L is chosen by an autotuner that times synthetic
 * batches of n-photon permanents (photons at random on 60 modes) for
 * L in {64, ..., 4096} on the current device and keeps the longest L within 2 %
 * of the best rate (the shortest for BBFG_MINORS); untuned n use L = 512.  The
 * leave-one-column-out walks of the sampler (precision BBFG_MINORS; n = the
 * size of the minors, n + 1 columns) are tuned separately: a unit of theirs
 * ends with one reduction per target column.
 *
 * bbfg_autotune        tunes n in [n_lo, n_hi] for the given precision; when
 *                      cache_path is not NULL, writes every tuned entry to it as
 *                      text lines "precision n L".  Takes ~0.1-1 s per n.
 *                      Samples drawn before and after tuning may differ in the
 *                      last bits of their weights (the split changes).
 * bbfg_autotune_load   loads such a file (also done at initialisation when the
 *                      environment variable BBFG_AUTOTUNE_CACHE names one).
 * bbfg_batch_unit_length  the L currently used for n_cols columns.
 * Errors: BBFG_EINVAL, BBFG_ERANGE, BBFG_EDEVICE.
 */
int bbfg_autotune(int32_t n_lo, int32_t n_hi, int32_t precision, const char *cache_path);
int bbfg_autotune_load(const char *cache_path);
int bbfg_batch_unit_length(int32_t n_cols, int32_t precision, uint64_t *unit_length);

/*
 * bs_sample -- Clifford & Clifford boson sampling (Sec. 4), ideal or lossy.
 *
 *   U                 m x m interferometer unitary (row-major), host or device.
 *   m                 number of modes, 1 <= m <= 256 (lossy: m <= 128).
 *   input_occupation  m int32 photon counts s_i >= 0 (host); n = sum s_i <=
 *                     BBFG_MAX_N.  A count > 1 repeats that column (U_S of
 *                     Eq. bs_p).
 *   n_samples         number of samples, >= 0.
 *   loss              uniform loss 1 - eta in [0, 1); 0 = ideal.  Lossy
 *                     sampling uses the 2m x 2m dilation
 *                     [[sqrt(eta) U, sqrt(1-eta) I], [sqrt(1-eta) U, -sqrt(eta) I]],
 *                     photons entering the first m modes, and reports the first
 *                     m output modes.
 *   seed              64-bit seed.  Sample s uses key_s = SplitMix64(seed, s);
 *                     draws 0..n-2 shuffle the columns (Fisher-Yates), draw
 *                     n-1+(k-1) picks the k-th output mode by inverse CDF.
 *   out_occupation    n_samples x m int32 output occupations (host).
 *   info              nullable: kernel_ms = total walk time, n_addends = total.
 *
 * Errors: BBFG_EINVAL, BBFG_ERANGE, BBFG_ENOMEM, BBFG_EDEVICE.
 */
int bs_sample(const bbfg_c128 *U, int32_t m, const int32_t *input_occupation, int32_t n_samples,
              double loss, uint64_t seed, int32_t *out_occupation, bbfg_info *info);

/*
 * bs_sample_lossy -- Clifford & Clifford sampling through a lossy
 * interferometer with non-uniform losses (Sec. 4: the losses stay in the
 * interferometer matrix, which is then no longer unitary, and the sampler runs
 * on twice the modes, sampling only the first half).
 *
 *   T                 m x m matrix of the lossy interferometer (row-major),
 *                     host or device: a contraction, T^H T <= I (singular
 *                     values at most 1).  Per-mode transmissions eta_i at the
 *                     inputs are T = U diag(sqrt(eta)); at the outputs
 *                     T = diag(sqrt(eta)) U; uniform loss is sqrt(eta) U.
 *   m, input_occupation, n_samples, seed, out_occupation, info
 *                     as bs_sample (1 <= m <= 128); info->rel_err_est as
 *                     bs_sample.
 *
 * The uniform part of the loss, eta_u = min(1, max_j sum_k |(T^H T)_jk|) (a
 * bound of T^H T's largest eigenvalue, exact for uniform and input losses), is
 * taken out at the input as in bs_sample_extracted (each photon survives with
 * probability eta_u, same random numbers); the survivors enter the first m of
 * 2m modes of the isometry [T'; R], T' = T / sqrt(eta_u) (R the
 * upper-triangular Cholesky factor of I - T'^H T', built on the host); all 2m
 * rows are candidate outputs and the first m are reported.  Every R with
 * R^H R = I - T'^H T' gives the same law on the first m modes, so for T =
 * sqrt(eta) U the law is that of bs_sample with loss 1 - eta, though not the
 * same samples.
 * Errors: as bs_sample; BBFG_EINVAL also when T is not a contraction (a pivot
 * of I - T^H T below -1e-10).
 */
int bs_sample_lossy(const bbfg_c128 *T, int32_t m, const int32_t *input_occupation, int32_t n_samples,
                    uint64_t seed, int32_t *out_occupation, bbfg_info *info);

/*
 * bs_sample_extracted -- boson sampling with uniform loss taken out of the
 * interferometer (Sec. 4: a loss that acts alike on every mode commutes with
 * U, so it can be applied as a pure-loss channel on the input photons, and
 * the simulation then runs on fewer photons and on U's own m modes instead of
 * 2m).  Each input photon survives with probability 1 - loss; the survivors
 * are sampled by Clifford & Clifford with U.  Same law as bs_sample with the
 * same loss, not the same samples; orders of magnitude cheaper at large loss.
 *
 *   U, m, input_occupation, n_samples, loss, seed, out_occupation, info
 *                     as bs_sample (loss in [0, 1); loss = 0 gives exactly the
 *                     samples of bs_sample with loss 0).
 *
 * Random numbers: those of bs_sample, plus draw 2n-1+b of each sample's key
 * deciding whether input photon b (the b-th column in input order) survives
 * (u = (x >> 11) 2^-53 < 1 - loss); the survivors keep the sample's column
 * order and take one step each.
 * Errors: as bs_sample.
 */
int bs_sample_extracted(const bbfg_c128 *U, int32_t m, const int32_t *input_occupation, int32_t n_samples,
                        double loss, uint64_t seed, int32_t *out_occupation, bbfg_info *info);

/* ---------------------------------------------------------------------------
 * Sampling server: continuous batching of Clifford & Clifford jobs.  Sec. 4
 * scales the sampler by running independent samplers side by side (one MPI
 * process per accelerator) and gathering their samples; on one GPU the
 * samplers share the device instead.  A background host thread admits queued
 * jobs while the device-memory budget and the active-job limit allow, keeps
 * each admitted job's matrix and partial samples resident on the device, and
 * in every iteration evaluates the current step's permanents of ALL active
 * jobs in one batched launch.  A job's samples are identical to bs_sample (or
 * bs_sample_lossy) with the same arguments.
 * ------------------------------------------------------------------------- */
typedef struct bbfg_server bbfg_server;

/* hbm_budget_bytes: device bytes the active jobs may hold (0 = 1/4 of the
 * device).  max_active_jobs >= 1.  Errors: BBFG_EINVAL, BBFG_EDEVICE. */
int bs_server_create(size_t hbm_budget_bytes, int32_t max_active_jobs, bbfg_server **srv);

/* Queue a job (arguments as bs_sample; U is copied before the call returns).
 * job_id receives an id > 0.  Errors: BBFG_EINVAL, BBFG_ERANGE. */
int bs_server_submit(bbfg_server *srv, const bbfg_c128 *U, int32_t m, const int32_t *input_occupation,
                     int32_t n_samples, double loss, uint64_t seed, uint64_t *job_id);

/* Queue a job through the lossy interferometer matrix T (arguments and
 * samples as bs_sample_lossy; T is copied and validated before the call
 * returns).  Errors: BBFG_EINVAL (also a T that is not a contraction),
 * BBFG_ERANGE. */
int bs_server_submit_lossy(bbfg_server *srv, const bbfg_c128 *T, int32_t m, const int32_t *input_occupation,
                           int32_t n_samples, uint64_t seed, uint64_t *job_id);

/* Queue a job whose uniform loss is applied to the input photons (arguments
 * and samples as bs_sample_extracted; U is copied before the call returns).
 * Errors: BBFG_EINVAL, BBFG_ERANGE. */
int bs_server_submit_extracted(bbfg_server *srv, const bbfg_c128 *U, int32_t m, const int32_t *input_occupation,
                               int32_t n_samples, double loss, uint64_t seed, uint64_t *job_id);

/* Non-blocking: BBFG_EBUSY while the job runs; on completion copies
 * n_samples x m occupations to out_occupation (host), the job's latency
 * (completion - submission, seconds) to latency_s (nullable) and its error
 * estimate to err_est (nullable; as bbfg_info.rel_err_est of bs_sample), then
 * forgets the job.  Errors: BBFG_ENOTFOUND, BBFG_ECANCELED (the job was
 * cancelled; it is forgotten), BBFG_EDEVICE (the job failed). */
int bs_server_poll(bbfg_server *srv, uint64_t job_id, int32_t *out_occupation, double *latency_s,
                   double *err_est);

/* Cancels a job.  A queued job is dropped at once; an active one leaves the
 * device at the end of its current step (its memory and slot are freed for
 * other jobs then); in both cases a later poll returns BBFG_ECANCELED.  A
 * finished job that was not polled yet is forgotten with its samples.
 * Non-blocking.  Errors: BBFG_EINVAL, BBFG_ENOTFOUND. */
int bs_server_cancel(bbfg_server *srv, uint64_t job_id);

/* Blocks until all submitted jobs are finished (polled or not). */
int bs_server_drain(bbfg_server *srv);

/* Stops the worker thread and frees the server's device memory. */
int bs_server_destroy(bbfg_server *srv);

/* Server counters (host). */
typedef struct {
    uint64_t jobs_submitted, jobs_done, iterations, samples_done;
    uint64_t max_active, max_queued;
    uint64_t jobs_cancelled;
    double busy_s; /* worker time spent advancing samples (host preparation + device) */
    double host_s; /* part of busy_s spent preparing steps on the host (plans, metadata, launches) */
    double wait_s; /* part of busy_s spent waiting for the device to finish a step */
    double flops;   /* algorithmic FP64 flops of the finished steps' walks (as bbfg_info.flops) */
    double walk_ms; /* device time of those walks (HIP events around each step's walk kernel) */
} bbfg_server_stats;
int bs_server_stats(bbfg_server *srv, bbfg_server_stats *out);

/* ---------------------------------------------------------------------------
 * Host-only planning diagnostics (no device needed).
 * ------------------------------------------------------------------------- */

/* Work decomposition of one permanent (Sec. 2.1/2.2): how the sum over
 * C' addends is split into per-lane prefix digits, per-unit high digits and
 * the Gray-walked low digits. */
typedef struct {
    int32_t n_cols;
    int32_t n_rows_kept;     /* rows with M_k > 0 */
    int32_t pivot_row;       /* user row index of the row held at +1 */
    int32_t n_lane_digits, n_high_digits, n_low_digits;
    uint32_t lane_product;   /* prod of lane-digit radices (<= 64 * lane_groups) */
    uint32_t lane_groups;    /* wavefronts needed to cover the lane digits */
    uint32_t low_count;      /* Q: length of one Gray-walked block */
    uint32_t pad;
    uint64_t high_count;     /* H: number of high-digit combinations */
    uint64_t n_addends;      /* C' = lane_product * high_count * low_count */
    uint64_t n_units;        /* work units */
} bbfg_plan_summary;

/* slots: resident wavefronts assumed for the split (0 = query the device's
 * FP64 walk occupancy).  Errors: BBFG_EINVAL, BBFG_ERANGE. */
int bbfg_plan_query(const int32_t *row_mult, int32_t n_rows, int32_t n_cols, int32_t slots,
                    bbfg_plan_summary *out);

/* Reflected mixed-radix Gray code over `n_digits` digits with the given radices
 * (digit 0 fastest), as walked inside a block: for t = 1 .. len-1,
 * changed_digit[t] is the digit that moves between positions t-1 and t and
 * direction[t] = +1 or -1 its step; entry 0 is -1 / 0.  len = prod(radices)
 * must be <= max_len.  Errors: BBFG_EINVAL, BBFG_ERANGE. */
int bbfg_gray_table(const int32_t *radices, int32_t n_digits, int32_t max_len,
                    int32_t *changed_digit, int32_t *direction);

/* Measured FP64 fused multiply-add throughput of the device (TFLOP/s, an FMA
 * counted as 2 flops): independent FMA chains in 32 wavefronts per compute unit,
 * about 10 ms of warm-up then about 40 ms timed; *ms (nullable) is the timed
 * kernel's duration.  The walk
 * kernels' rates are quoted against the published peak and against this.
 * Errors: BBFG_EINVAL, BBFG_EDEVICE. */
int bbfg_fp64_fma_peak(double *tflops, double *ms);

/* Resident wavefronts per compute unit of the walk kernel for n_cols columns
 * and the number of compute units (device query).  precision BBFG_MINORS: the
 * leave-one-column-out kernel for n_cols >= 2 columns (perm_minors splits its
 * walk into whole rounds of those wavefronts); precision BBFG_COLS (accepted
 * only here): the column-power kernel for n_cols distinct columns, which runs
 * perm_bbfg_cols when every column multiplicity is the same e >= 2.  Errors:
 * BBFG_ERANGE, BBFG_EDEVICE. */
int bbfg_walk_occupancy(int32_t n_cols, int32_t precision, int32_t *waves_per_cu, int32_t *n_cu);

#ifdef __cplusplus
}
#endif
#endif /* BBFG_H */
