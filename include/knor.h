/*
 * knor.h -- C ABI of the MI355X (gfx950) k-means library.
 *
 * The library implements the Lloyd iteration of Mhembere et al., "knor: A
 * NUMA-Optimized In-Memory, Distributed and Semi-External-Memory k-means
 * Library" (HPDC'17, arXiv 1606.08905): the nearest-centroid assignment
 * (Algorithm 1), optionally pruned by the minimal triangle inequality (MTI,
 * Section "Minimal Triangle Inequality (MTI) Pruning"), followed by the
 * centroid update (Phase II / the merge of per-thread partial centroids of
 * Algorithm 1).  All compute runs in HIP kernels on one GPU.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Points X are n x d, row-major, contiguous, in DEVICE memory, of the
 *    element type given by knor_dtype (BF16 as raw 16-bit patterns).
 *  - Centroids are k x d row-major FP64 in DEVICE memory.  Labels are int32
 *    in DEVICE memory.  The caller owns every array passed in.
 *  - Distances are squared Euclidean, D(x, c) = sum_i (x_i - c_i)^2 (Section
 *    "Nomenclature"); the assigned centroid is the lowest index among those
 *    whose D, evaluated in FP64 in index order without fused multiply-add,
 *    is smallest (Algorithm 1's strict "<" scan).  Lower-precision arithmetic
 *    is used only where a rounding-error bound proves it picks that same
 *    centroid; every other point is recomputed in that FP64 form.
 *  - A centroid is the mean of its members (Phase II), summed in FP64 in a
 *    fixed order: members by increasing point index, leaves of 64
 *    consecutive members summed left to right starting from the first
 *    member, leaf sums combined pairwise with the split at the largest power
 *    of two below the leaf count, then one correctly rounded division by the
 *    member count.  A cluster without members keeps its previous centroid.
 *  - Work is stream-ordered on opts->stream (a hipStream_t; NULL = the null
 *    stream).  knor_assign and knor_update return before the work finishes;
 *    knor_fit returns after it finishes, because it observes convergence.
 *  - Argument errors are detected before any device work is enqueued; on
 *    every error return, the output arrays are left untouched.
 *  - knor_assign and knor_update accept n = 0 (X and the label array may
 *    then be NULL): assign does nothing; update copies C_prev to C_out and
 *    writes zero counts.
 *  - Limits: 1 <= d <= 256, 1 <= k <= 16384, 1 <= n < 2^31, k <= n (fit).
 *  - Process-wide state: one table of FP32 tile schedules per (padded d,
 *    padded k) class, filled by the timing-based tuner (opts->autotune,
 *    knor_fit_batched) and read by later calls, behind a mutex.  A schedule
 *    changes speed only, never a result, so concurrent calls on different
 *    streams give the same results as the same calls made one at a time;
 *    which schedule the tuner keeps can depend on concurrent load.
 *    opts->tile_blocks / tile_resident force a schedule and bypass the table.
 */
#ifndef KNOR_H
#define KNOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KNOR_OK = 0,
  KNOR_ERR_INVALID_ARG = 1,   /* a size, pointer or option is out of range  */
  KNOR_ERR_OUT_OF_MEMORY = 2, /* device workspace could not be allocated, or
                                 exceeds opts->workspace_cap               */
  KNOR_ERR_HIP = 3,           /* a HIP runtime call failed                  */
  KNOR_ERR_NUMERIC = 4,       /* NaN or Inf in X or in the centroids        */
  KNOR_ERR_UNSUPPORTED = 5,   /* valid request this build does not handle   */
  KNOR_ERR_SCRATCH = 6        /* knor_assign_noalloc: the request needs more
                                 than its fixed scratch                      */
} knor_status;

typedef enum { KNOR_F64 = 0, KNOR_F32 = 1, KNOR_BF16 = 2 } knor_dtype;

/* Initial centroids.  The paper does not specify initialisation. */
/* Every mode other than GIVEN is a deterministic function of opts->seed and
 * the values of X (SplitMix64, Steele, Lea and Flood 2014, seeded with
 * opts->seed; next() is its next 64-bit output); C_init is then ignored. */
typedef enum {
  KNOR_INIT_GIVEN = 0, /* C_init holds the k x d FP64 initial centroids      */
  KNOR_INIT_FORGY = 1, /* k distinct rows of X: a Fisher-Yates pass over
                          slots i = n-1 down to n-k, j = next() % (i + 1),
                          swap slots i and j; centroid r is the row that
                          lands in slot n-1-r                                */
  KNOR_INIT_SHUFFLE_FIRSTK = 2, /* the first k entries of a front-to-back
                          Fisher-Yates shuffle of 0..n-1: for i = 0..k-1,
                          j = i + next() % (n - i), swap slots i and j;
                          centroid i is the row in slot i                    */
  KNOR_INIT_KMEANSPP = 3 /* k-means++ (D^2) seeding on the device: centroid 0
                          is row floor(r_0 n / 2^64); draw t >= 1 weights
                          every point p by w(p) = floor(D(p) 2^(B - e)),
                          D(p) the canonical FP64 squared distance to the
                          nearest centroid so far, e the exponent with
                          max_p D(p) < 2^e, B = 63 - ceil(log2 n), and takes
                          the point whose weight interval contains
                          floor(r_t W / 2^64), W = sum of the weights
                          (integers, so no summation order matters); W = 0
                          takes row floor(r_t n / 2^64).  r_t = the t-th
                          output of next().  Costs k - 1 passes over X   */
} knor_init;

typedef struct {
  uint32_t struct_size; /* sizeof(knor_opts); 0 selects all defaults        */
  int32_t prune;        /* 0: every point scans every centroid;
                           1: MTI pruning (default)                          */
  int32_t recheck;      /* 1: FP64 recheck of near-tie points only (default);
                           2: FP64 recheck of every point (validation mode)  */
  int32_t check_numeric;/* 1: reject NaN/Inf in X and C (default 1)         */
  uint64_t seed;        /* seed of the non-GIVEN init modes                  */
  void* stream;         /* hipStream_t; NULL = null stream                   */
  size_t workspace_cap; /* bytes of device workspace allowed; 0 = unlimited  */
  int32_t* label_history; /* DEVICE, optional: max_iters x n; row t receives
                             the labels produced by iteration t's assignment */
  int64_t* iter_counters; /* HOST, optional: max_iters x KNOR_NCOUNTERS; row
                             t receives that iteration's counters (below)    */
  int32_t poll_every;   /* knor_fit checks convergence on the host every this
                           many iterations (default 8); iterations enqueued
                           after convergence do no work                       */
  double* profile_ms;   /* HOST, optional: KNOR_NPROF entries.  knor_fit adds
                           the GPU time (HIP events on opts->stream) of every
                           launch of each kernel group (below)               */
  int64_t* profile_launches; /* HOST, optional: KNOR_NPROF launch counts     */
  int32_t profile_mask; /* bit g set: time kernel group g; 0 = every group.
                           Each timed launch adds two event records          */
  int32_t tile_blocks;  /* FP32 tile: blocks of 16 points per wave (1, 2 or
                           4); 0 = tuned or default.  A value the row width
                           does not allow gives KNOR_ERR_UNSUPPORTED         */
  int32_t tile_resident;/* FP32 tile: 1 = all centroids resident in LDS
                           (KNOR_ERR_UNSUPPORTED if they do not fit),
                           2 = centroids streamed in chunks, 0 = tuned or
                           default.  The schedule never changes results      */
  int32_t autotune;     /* 1: knor_fit times the FP32 tile schedules of its
                           (d, k) class on a sample of X once per process
                           and keeps the fastest; 0: use the table or the
                           default (knor_fit_batched always tunes unless a
                           schedule is forced)                               */
  int32_t learned;      /* 1: learned candidate proposal on MTI survivors
                           (needs prune = 1): an MLP d -> 256 -> 256 -> k,
                           trained with train_batches minibatches of 4096
                           (x, label) pairs after each of iterations
                           1..train_iters, proposes 16 candidates per
                           survivor from iteration train_iters + 1 on; a
                           survivor takes its nearest candidate c* only if
                           d(x, c*) (1 + eta) < s(c*), else it is scanned
                           as usual.  Labels do not depend on this option  */
  int32_t train_iters;  /* default 5 (when 0)                               */
  int32_t train_batches;/* default 16 (when 0)                              */
  int32_t profile_every;/* time the groups of profile_mask only in iterations
                           t with t % profile_every == 0 (fewer event
                           records); 0 or 1 = every iteration               */
  int32_t update;       /* centroid update of knor_fit, knor_fit_batched and
                           knor_update.  0 (default): the member sum in the
                           canonical order (members by point index, leaves
                           of 64 summed left to right, pairwise tree over
                           the leaves), then one division.  1: the exact
                           mean of the members, rounded once to nearest
                           (ties to even), which no summation order changes;
                           inside a fit only the points whose label changed
                           move between the clusters' exact sums when few
                           do.  1 needs FP32 or BF16 points (FP64:
                           KNOR_ERR_UNSUPPORTED).  The two readings may
                           differ in the last bit of a centroid and so,
                           rarely, in a later label                          */
  double* centroid_history; /* DEVICE, optional: max_iters x k x d FP64; row
                               t receives the centroids that iteration t's
                               assignment used (row 0: the initial ones)    */
  int32_t clause2;      /* MTI Clause 2 (skip centroid j for a point of
                           cluster a when u (1 + eta) < 1/2 d(c_a, c_j))
                           applied per block of 64 survivors of one cluster,
                           sorted by bound: each block scans only its
                           candidate centroids.  0: on for FP32 points with
                           1024 <= k <= 8192 (default); 1: off; 2: on for
                           any k <= 8192 (FP32 points with prune = 1, else
                           KNOR_ERR_UNSUPPORTED).  Needs k x k FP32 of
                           workspace.  Labels do not depend on this option */
  int32_t batch_graph;  /* knor_fit_batched: 1 = set every problem up, record
                           all their iterations (max_iters each) on four
                           parallel chains into one HIP graph and launch it
                           once (iterations after a problem converges do no
                           work); 0 (default) = host worker threads, each
                           with its own stream, polling convergence.  Same
                           results either way; learned = 1 always uses 0   */
  double* objective_history; /* HOST, optional (knor_fit only): max_iters
                           entries; entry t receives J_t, the sum over points
                           of the canonical FP64 D(x, c) to the centroid of
                           x's label from iteration t's assignment, under the
                           centroids that assignment used, summed in the
                           canonical order (leaves of 64, pairwise tree).
                           Costs one extra pass over X per iteration        */
} knor_opts;

/* Kernel groups timed by opts->profile_ms. */
enum {
  KNOR_PROF_ASSIGN_DENSE = 0, /* distance tile + argmin over all points      */
  KNOR_PROF_ASSIGN_LIST = 1,  /* distance tile + argmin over MTI survivors   */
  KNOR_PROF_RECHECK = 2,      /* FP64 recheck of near-tie points             */
  KNOR_PROF_FILTER = 3,       /* MTI bound update, Clause 1 and tightening   */
  KNOR_PROF_SORT = 4,         /* update pass 1: stable counting sort          */
  KNOR_PROF_LEAF = 5,         /* update pass 2: leaf sums (gathers X)         */
  KNOR_PROF_TREE = 6,         /* update pass 2: tree, division, operands      */
  KNOR_PROF_CC = 7,           /* MTI centroid-pair bounds s(c)                */
  KNOR_PROF_LEARNED = 8,      /* proposal MLP: training and forward pass   */
  KNOR_PROF_CERTIFY = 9,      /* proposal certificate and its neighbour lists */
  KNOR_NPROF = 10
};

/* Per-iteration counters (columns of opts->iter_counters). */
enum {
  KNOR_CNT_CHANGED = 0,   /* labels that differ from the previous iteration  */
  KNOR_CNT_SCANNED = 1,   /* points whose distances to all k were evaluated  */
  KNOR_CNT_PRUNED_A = 2,  /* MTI: decided by the drift-updated bound          */
  KNOR_CNT_PRUNED_B = 3,  /* MTI: decided after tightening the bound          */
  KNOR_CNT_RECHECKED = 4, /* points recomputed in FP64                        */
  KNOR_CNT_CERTIFIED = 5, /* survivors decided by a certified proposal        */
  KNOR_CNT_QUERIED = 6,   /* survivors that took a proposal (from the network
                             or from their cached candidates)                */
  KNOR_CNT_DISTS = 7,     /* point-centroid distances evaluated (tiles, FP64
                             rechecks, Clause-3 tightening)                   */
  KNOR_CNT_FORWARD = 8,   /* survivors whose proposal was computed: a point
                             goes through the network at most once per fit */
  KNOR_NCOUNTERS = 9
};

typedef struct {
  int32_t iters;          /* iterations performed                            */
  int32_t converged;      /* 1 if #changed <= tol * n was reached            */
  int64_t changed_last;   /* #changed in the last iteration                  */
  int64_t dists_computed; /* point-centroid distances evaluated (all iters)  */
  int64_t scanned;        /* sum of KNOR_CNT_SCANNED                         */
  int64_t pruned_a;       /* sum of KNOR_CNT_PRUNED_A                        */
  int64_t pruned_b;       /* sum of KNOR_CNT_PRUNED_B                        */
  int64_t rechecked;      /* sum of KNOR_CNT_RECHECKED                       */
  double objective;       /* sum over points of D(x, c_label) for the final
                             labels and the centroids they were assigned to  */
  double seconds;         /* wall time of the call                           */
  int64_t certified;      /* sum of KNOR_CNT_CERTIFIED                       */
  int64_t mlp_queries;    /* sum of KNOR_CNT_QUERIED                         */
  int64_t mlp_forward_rows; /* sum of KNOR_CNT_FORWARD                       */
} knor_stats;

/* knor_fit: Lloyd's algorithm (Sections "Introduction", "Parallel Lloyd's
 * Algorithm"; MTI per Section "Minimal Triangle Inequality (MTI) Pruning"
 * when opts->prune = 1).  Iteration t assigns every point to its nearest
 * centroid, counts changed labels (all n at t = 0), replaces each centroid
 * by the mean of its members, and stops once #changed <= tol * n or after
 * max_iters iterations.  The returned centroids are the means of the
 * returned labels.
 *   X          DEVICE n x d, dtype dt.
 *   C_init     DEVICE k x d FP64 when init == KNOR_INIT_GIVEN, else NULL.
 *   max_iters  >= 1.       tol  in [0, 1).
 *   opts       may be NULL (defaults).
 *   C_out      DEVICE k x d FP64, written on success.
 *   labels_out DEVICE n int32, written on success.
 *   st         HOST, may be NULL.
 * Blocks until the fit is complete.  Labels do not depend on prune or on
 * the storage dtype beyond the values X holds. */
knor_status knor_fit(const void* X, knor_dtype dt, int64_t n, int32_t d,
                     int32_t k, knor_init init, const double* C_init,
                     int32_t max_iters, double tol, const knor_opts* opts,
                     double* C_out, int32_t* labels_out, knor_stats* st);

/* Host-link counters of knor_fit_streamed, per iteration. */
enum {
  KNOR_IO_COPIED = 0,   /* rows copied from host memory in whole batches (full
                           passes: iteration 0, every iteration without MTI,
                           and the objective)                               */
  KNOR_IO_GATHERED = 1, /* rows read from host memory one by one: points
                           that fail MTI Clause 1 and are not in the cache  */
  KNOR_IO_CACHED = 2,   /* rows of such points served by the row cache      */
  KNOR_IO_ADMITTED = 3, /* rows written into the row cache (refresh)        */
  KNOR_NIO = 4
};

typedef struct {
  uint32_t struct_size;   /* sizeof(knor_stream_opts); 0 selects defaults    */
  int64_t batch_rows;     /* rows per batch, rounded up to a multiple of
                             4096; 0 = min(n, 2^22) rounded up.  The device
                             holds two batches of rows for staging          */
  int64_t cache_rows;     /* row cache capacity in rows (0 = no cache).  The
                             device holds two regions of this many rows     */
  int32_t cache_interval; /* I: the cache refreshes at iterations I, 3I, 7I,
                             15I, ... (each gap twice the previous); 0 = 5   */
  int32_t skip_objective; /* 1: leave st->objective at 0 (saves the final
                             pass over X); 0 (default): compute it          */
  int64_t* io_counters;   /* HOST, optional: max_iters x KNOR_NIO; row t
                             receives iteration t's counters; the objective
                             pass adds to the last iteration's row          */
} knor_stream_opts;

/* knor_fit_streamed: knor_fit for data that stays in host memory (the
 * paper's semi-external-memory mode, Section "Semi-External Memory": I/O
 * minimization and the partitioned row cache).  Same iteration, same
 * results as knor_fit with opts->update = 1 on the same values.  Each
 * iteration runs over batches of batch_rows consecutive rows; a batch's
 * rows reach the device whole (a DMA copy) when every point needs its
 * distances (iteration 0, or prune = 0), and otherwise only for the points
 * that fail MTI Clause 1: a point that Clause 1 keeps has no row read.  A
 * needed row comes from the device row cache if the cache holds it (the
 * rows active at the last refresh iteration, lowest point indices first up
 * to cache_rows), else from host memory, read by the kernel over the host
 * link.
 *   X          HOST n x d, dtype KNOR_F32 or KNOR_BF16, in page-locked
 *              memory the device can read (hipHostMalloc, or a pinned
 *              torch tensor); anything else gives KNOR_ERR_INVALID_ARG.
 *              Must not change during the call.
 *   opts       as for knor_fit, with update = 1 required (the exact mean,
 *              which no order of the passes changes; 0 gives
 *              KNOR_ERR_UNSUPPORTED); learned = 1, clause2 = 2, init =
 *              KNOR_INIT_KMEANSPP, autotune, objective_history,
 *              profile_ms and profile_launches give KNOR_ERR_UNSUPPORTED.  Convergence is
 *              polled after every iteration (poll_every is ignored).
 *   sopts      may be NULL (defaults).
 *   C_init, C_out, labels_out, st: as for knor_fit (C_init, C_out and
 *              labels_out in DEVICE memory).
 * With opts->check_numeric the initial centroids are checked before the
 * first iteration and the rows of X as they arrive in iteration 0 (there is
 * no pass over the link for the check alone): a NaN or Inf then gives
 * KNOR_ERR_NUMERIC after that iteration, with C_out holding the initial
 * centroids and labels_out those of the batches before the first bad one;
 * no kernel reads a batch from the first bad one on.
 * Uses one extra stream (default priority) for the transfers.  Blocks
 * until the fit is complete. */
knor_status knor_fit_streamed(const void* X, knor_dtype dt, int64_t n, int32_t d,
                              int32_t k, knor_init init, const double* C_init,
                              int32_t max_iters, double tol, const knor_opts* opts,
                              const knor_stream_opts* sopts, double* C_out,
                              int32_t* labels_out, knor_stats* st);

/* knor_assign: one assignment step (Algorithm 1, nearest-centroid loop).
 *   C          DEVICE k x d FP64.
 *   labels_out DEVICE n int32: the nearest centroid of every point.
 *   dist2_out  DEVICE n FP64 or NULL: D(x, c_label) evaluated in FP64 in
 *              index order (the same value the definition above compares).
 * Asynchronous on opts->stream. */
knor_status knor_assign(const void* X, knor_dtype dt, int64_t n, int32_t d,
                        const double* C, int32_t k, const knor_opts* opts,
                        int32_t* labels_out, double* dist2_out);

/* knor_assign_noalloc: knor_assign (same arguments, results and stream
 * order) for callers that cannot allocate device memory -- code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  It
 * calls no hipMalloc, hipFree or memset: its workspace is a fixed array of
 * 32 MiB of device memory per GPU, held from the library's load until the
 * process ends, and its counters are cleared by kernels.  The workspace is
 * about 4 n + 4 kpad dp + 8 k d + 80 KiB bytes (kpad = k rounded up to 16,
 * dp = d rounded up to a power of two >= 8; FP32 points), so n up to about
 * 7.5 million at d = 32, k = 4096; a larger request returns
 * KNOR_ERR_SCRATCH before any device work.  Every call on one GPU uses
 * that GPU's single array: calls that overlap in time on the same GPU (on
 * different streams or host threads) race and must be serialized by the
 * caller; consecutive calls on one stream are ordered and safe. */
knor_status knor_assign_noalloc(const void* X, knor_dtype dt, int64_t n, int32_t d,
                                const double* C, int32_t k, const knor_opts* opts,
                                int32_t* labels_out, double* dist2_out);

/* knor_tile_values: the matrix-core tile's working values, for checking its
 * rounding bound.  The assignment step (Algorithm 1's nearest-centroid
 * loop) evaluates y_j = |c_j|^2 - 2 x.c_j for FP32 points on FP32 matrix
 * cores and for BF16 points on BF16 matrix cores (centroid operand -2c as
 * two BF16 terms), and trusts a point's smallest value only when the gap to
 * the next exceeds twice a bound E(x) on |y~_j - y_j|; every other point is
 * recomputed in FP64.  This entry point returns those values and bounds:
 *   Y  DEVICE n x k FP32: Y[p][j] = the tile's value for point p and
 *      centroid j (the same operands and accumulation order as every
 *      assignment pass);
 *   E  DEVICE n FP64: E(x_p) as the decision uses it, with R^2 over all k.
 * FP32 and BF16 points (FP64: KNOR_ERR_UNSUPPORTED).  Asynchronous. */
knor_status knor_tile_values(const void* X, knor_dtype dt, int64_t n, int32_t d,
                             const double* C, int32_t k, const knor_opts* opts, float* Y,
                             double* E);

/* knor_update: one centroid update (Phase II; the merge of Algorithm 1).
 * With opts->update = 0 (default) each centroid is the canonical-order
 * member sum divided once by the count; with opts->update = 1 it is the
 * exact member mean rounded once (FP32 / BF16 points only, else
 * KNOR_ERR_UNSUPPORTED before any device work).
 *   labels     DEVICE n int32, each in [0, k).  A label outside that range
 *              is not detected on the device; the caller guarantees range.
 *   C_prev     DEVICE k x d FP64: kept for clusters without members.
 *   C_out      DEVICE k x d FP64 (may equal C_prev).
 *   counts_out DEVICE k int64 or NULL: members per cluster.
 * Asynchronous on opts->stream. */
knor_status knor_update(const void* X, knor_dtype dt, int64_t n, int32_t d,
                        const int32_t* labels, int32_t k,
                        const double* C_prev, const knor_opts* opts,
                        double* C_out, int64_t* counts_out);

/* One problem of a batch.  All pointers are DEVICE pointers owned by the
 * caller; C_init NULL selects KNOR_INIT_FORGY with seed opts->seed + the
 * problem's index. */
typedef struct {
  const void* X;          /* n x d, dtype dt                                 */
  knor_dtype dt;
  int64_t n;
  int32_t d, k;
  const double* C_init;   /* k x d FP64 or NULL                              */
  int32_t max_iters;
  double tol;
  double* C_out;          /* k x d FP64                                      */
  int32_t* labels_out;    /* n int32                                         */
} knor_problem;

/* knor_fit_batched: knor_fit on each of `count` independent problems
 * (restarts, or unrelated data sets), each with exactly the results knor_fit
 * gives it alone.  The problems run concurrently on the device's hardware
 * queues, largest work (n k d) first; each FP32 (d, k) class is tuned once
 * per process unless opts forces a tile schedule.  Work is ordered after
 * everything already enqueued on opts->stream; the call returns when every
 * problem is done.
 *   probs   HOST array of count problems (count >= 0).
 *   opts    as for knor_fit, except that label_history, iter_counters,
 *           centroid_history, objective_history and profile_ms /
 *           profile_launches must be NULL.
 *   st      HOST array of count stats, or NULL.
 * Every problem is validated before any work starts (an invalid one gives
 * KNOR_ERR_INVALID_ARG and no output is touched).  A runtime error in one
 * problem leaves the others' results valid; the first error in problem
 * order is returned. */
knor_status knor_fit_batched(const knor_problem* probs, int32_t count,
                             const knor_opts* opts, knor_stats* st);

/* The proposal MLP on its own (used by knor_fit with opts->learned).  The
 * network d -> h -> h -> k has ReLU hidden layers; its FP32 parameters are
 * one DEVICE vector of knor_mlp_param_count(d, h, k) floats: W1 (d x h,
 * row-major, W1[i][j] joins input i to unit j), b1 (h), W2 (h x h), b2 (h),
 * W3 (h x k), b3 (k).  Every matrix product rounds its operands to BF16
 * (nearest even) and sums in FP32.  Limits: 1 <= d <= 256, h in {32, 64,
 * 128, 256}, 1 <= k <= 16384.  The paper has no such network; it serves
 * only to choose which survivors of the MTI filter skip the k-way scan. */

/* Number of parameters, or -1 if the sizes are out of range. */
int64_t knor_mlp_param_count(int32_t d, int32_t h, int32_t k);

/* He-uniform initialisation: W[i][j] = (2u - 1) sqrt(6 / fan_in) with u the
 * next output z of SplitMix64(seed) as (z >> 11) 2^-53, drawn in parameter
 * order, computed in FP64 and rounded to FP32; biases zero.  Synchronous. */
knor_status knor_mlp_init(float* params, int32_t d, int32_t h, int32_t k,
                          uint64_t seed, const knor_opts* opts);

/* One training step on a minibatch: Xs (DEVICE B x d, standardized inputs),
 * y (DEVICE B labels in [0, k), not checked on the device).  Computes the
 * mean softmax cross-entropy and its gradient; if grad_out (DEVICE, param
 * count floats) is given the gradient is written there; with lr > 0 an Adam
 * step (beta 0.9 / 0.999, eps 1e-8, bias-corrected at step number `step` >= 1)
 * updates params, adam_m and adam_v (DEVICE, param count floats each).
 * loss_out (HOST) receives the loss; the call then returns after the step
 * completes, otherwise it is asynchronous on opts->stream. */
knor_status knor_mlp_train_step(float* params, float* adam_m, float* adam_v,
                                int64_t step, int32_t d, int32_t h, int32_t k,
                                const float* Xs, const int32_t* y, int32_t B,
                                float lr, float* grad_out, double* loss_out,
                                const knor_opts* opts);

/* Candidates of m standardized points Xs (DEVICE m x d): cand_out (DEVICE
 * m x 16 int32) row p holds the 16 classes with the largest keys, in
 * decreasing key order.  The key of class j is its FP32 logit with the low
 * B mantissa bits replaced by 2^B - 1 - j, where 2^B >= k rounded up to a
 * multiple of 64 (so value and class share one float; among logits that
 * agree in their leading bits the code decides).  When k < 16 the entries
 * past the k real classes are -1.  Asynchronous on opts->stream. */
knor_status knor_mlp_propose(const float* params, int32_t d, int32_t h,
                             int32_t k, const float* Xs, int64_t m,
                             int32_t* cand_out, const knor_opts* opts);

/* Human-readable name of a status code (static storage). */
const char* knor_status_string(knor_status s);

/* Library version as major*10000 + minor*100 + patch.  0.2.0 added
 * knor_opts.update, 0.3.0 knor_opts.centroid_history, the init modes
 * SHUFFLE_FIRSTK and KMEANSPP and the kernel group KNOR_PROF_CERTIFY (so
 * profile arrays hold KNOR_NPROF = 10 entries; each new field changed
 * sizeof(knor_opts), which struct_size must equal); 0.4.0 added
 * knor_fit_streamed, knor_stream_opts, knor_opts.batch_graph and
 * knor_opts.objective_history. */
int32_t knor_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KNOR_H */
