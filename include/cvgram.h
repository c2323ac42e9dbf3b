/*
 * cvgram.h -- fold-independent cross-validation Gram products on AMD MI355X
 * (gfx950).
 *
 * Given X (N x K), Y (N x M) and a fold label per row, the library returns,
 * for every fold p, the training-partition products X_T^T X_T and X_T^T Y_T
 * (T = rows whose label is not p), with X and Y centred and/or scaled by
 * statistics of the training rows only.  This is the problem of Engstrom &
 * Jensen, "Fast Partition-Based Cross-Validation With Centering and Scaling
 * for X^T X and X^T Y": Definition 1 (partitions), Definitions 2-5
 * (means, centering, Bessel-corrected deviations, scaling), Section 6 and
 * Table 1 (the 16 centering/scaling combinations, 12 of them distinct).
 * The computation follows the paper's fast method (Algorithm 7, generalised
 * to all combinations): full-data products once, validation-block products
 * and column sums/sums of squares per fold, then subtraction (Lemmas 2-3),
 * mean downdate (Lemma 7), rank-one centering (Propositions 7-8), deviation
 * from sums (Lemmas 12-14) and Hadamard division (Propositions 15-16).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All matrix arguments are DEVICE pointers (memory of the current HIP
 *    device), dense row-major with no padding: X[n*K + k], Y[n*M + m],
 *    out_XtX[i*K + j], out_XtY[i*M + j].
 *  - Fold labels are int32, 0-based: label p is the paper's partition p+1.
 *    The number of folds is P = max(label) + 1.  Definition 1 requires
 *    2 <= P <= N, every label in [0, P) and every fold non-empty.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Device work is enqueued on it; calls return without waiting for it
 *    except where stated.  Outputs are complete once the stream reaches the
 *    point where the call enqueued its work.
 *  - Every entry point returns a cvgram_status (except the queries
 *    cvgram_num_folds, cvgram_version and the two string getters); nothing
 *    is thrown across the ABI.  On an error the output arguments are left untouched (a handle
 *    out-parameter is set to NULL) and nothing leaks;
 *    cvgram_last_error_message() gives details for the calling thread.
 *  - NaN or Inf inputs are not checked; they propagate into the outputs.
 *  - Calls on one handle must not overlap from several host threads.
 */
#ifndef CVGRAM_H
#define CVGRAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cvgram_handle* cvgram_t;

typedef enum {
  CVGRAM_OK = 0,
  CVGRAM_EINVAL = 1,        /* null pointer, bad size, bad flag or mode      */
  CVGRAM_EFOLDS = 2,        /* partitioning violates Definition 1            */
  CVGRAM_ENOTSCALABLE = 3,  /* scaling asked for but some |T_p| - ddof < 1
                               (Definition 6, generalised to ddof)           */
  CVGRAM_ENOMEM = 4,        /* device or pinned-host allocation failed       */
  CVGRAM_EDEVICE = 5,       /* a HIP runtime call or kernel launch failed    */
  CVGRAM_ERANGE = 6,        /* fold index out of range                       */
  CVGRAM_ESINGULAR = 7      /* cvgram_ridge: a system not positive definite  */
} cvgram_status;

/* element type of X and Y */
typedef enum { CVGRAM_F32 = 0, CVGRAM_F64 = 1 } cvgram_dtype;

/* arithmetic of the Gram contractions (statistics and corrections are
   always FP64):
     CVGRAM_MODE_FP64    FP64 MFMA on FP64 pivot-shifted data; outputs FP64.
     CVGRAM_MODE_BF16X3  each pivot-shifted value split as hi + lo in bf16;
                         hi*hi + hi*lo + lo*hi on bf16 MFMA with FP32
                         accumulation, row blocks combined in FP64 (64- and
                         128-wide tiles) or in FP32 running totals every
                         512 rows (256 x 128 tiles); outputs FP32.
     CVGRAM_MODE_FP32    FP32 MFMA, FP32 accumulation over row blocks that
                         are combined in FP64; outputs FP32.
   The paper computes in FP64 only (Section 7); the two mixed modes are this
   library's.  Their error against FP64, per fold and class as a relative
   Frobenius norm, is held to 1e-6 (FP32) and 2e-5 (BF16X3) on sums over
   many rows.  Over a few rows the split's rounding does not average out:
   per entry it is at most (3 * 2^-18 + |T| * 2^-24) * sum over the training
   rows T of |z_i z_j|, z the pivot-shifted values. */
typedef enum {
  CVGRAM_MODE_FP64 = 0,
  CVGRAM_MODE_BF16X3 = 1,
  CVGRAM_MODE_FP32 = 2
} cvgram_mode;

/* Class numbering of the distinct products (Section 6, Table 1).
   X^T X depends only on X's preprocessing:
     xtx class = 2*center_x + scale_x   (0 raw, 1 scaled, 2 centred,
                                          3 centred and scaled)
   X^T Y depends on whether X or Y (or both) is centred (Lemma 9) and on
   each scaling:
     xty class = 4*(center_x | center_y) + 2*scale_x + scale_y            */
#define CVGRAM_XTX_CLASSES 4
#define CVGRAM_XTY_CLASSES 8

/*
 * cvgram_create -- plan and run the per-fold statistics and Gram pass.
 *
 * Inputs: X (N x K) and Y (N x M) of element type `dtype`, fold_id[N]
 * (int32); all device pointers.  Y may be NULL only when M == 0.
 * N >= 2, K >= 1, M >= 0.  center_x/scale_x/center_y/scale_y (0 or 1)
 * select the combination returned by cvgram_fold(); ddof is 0 or 1 (1 is
 * the paper's Bessel correction, Definition 4); deviations divide by
 * |T_p| - ddof.
 *
 * What it does (Algorithm 1; Algorithm 7 steps 3-4, 8, 10, 17, 19): sorts
 * the rows by fold label on the device (stable: rows ascending within a
 * fold), validates the partitioning, computes per-column pivots, the FP64
 * column sums, sums of squares, minima and maxima of every validation
 * block, and the validation-block Gram products of all folds in one grouped
 * MFMA launch.  It waits on `stream` once for the validation data and the
 * fold sizes (twice when P > 4096); everything after that is only enqueued.
 *
 * Fold path: with many small folds (P >= 64 and no fold above 24 rows,
 * e.g. leave-one-out), or when one FP64 K x (K + M) slab per fold would
 * exceed 16 GB, the rows are packed without per-fold padding, only the full
 * Gram is contracted, and each fold's validation Gram is formed from its
 * rows inside the per-fold corrections (it never reaches memory).  The
 * environment variable CVGRAM_FOLD_PATH=grouped or =fused, read at each
 * create, forces either path; results agree to rounding.
 *
 * Ownership: X, Y and fold_id are borrowed; they must stay valid and
 * unchanged until the work this call enqueued has completed.  The handle
 * owns all its device workspace and is freed by cvgram_destroy().
 *
 * Errors: CVGRAM_EINVAL (bad argument), CVGRAM_EFOLDS (Definition 1),
 * CVGRAM_ENOTSCALABLE (a scale flag is set and some |T_p| - ddof < 1),
 * CVGRAM_ENOMEM, CVGRAM_EDEVICE.  *out is NULL on any error.
 */
cvgram_status cvgram_create(const void* X, const void* Y, const int32_t* fold_id,
                            int64_t N, int64_t K, int64_t M, cvgram_dtype dtype,
                            int center_x, int scale_x, int center_y, int scale_y,
                            int ddof, cvgram_mode mode, void* stream, cvgram_t* out);

/* Number of folds P of the handle's partitioning (Definition 1: the
 * largest label plus one), known on the host once cvgram_create returned.
 * Returns -1 for a NULL handle (and sets cvgram_last_error_message). */
int32_t cvgram_num_folds(cvgram_t h);

/* Copy of the fold bookkeeping of Algorithm 1 as a stable counting sort:
 * perm[N] (int32) lists the rows of fold 0, then fold 1, ..., each in
 * ascending row order; offsets[P+1] (int64) delimits fold p as
 * perm[offsets[p] .. offsets[p+1]).  Device pointers, caller-allocated; either
 * may be NULL.  Enqueued on the handle's stream. */
cvgram_status cvgram_partition(cvgram_t h, int32_t* perm, int64_t* offsets);

/*
 * cvgram_fold -- training products of fold p (0 <= p < P) for the
 * combination given at create time (Algorithm 7 steps 9, 11-16, 18, 20-27,
 * with Table 1 for the other combinations).
 * out_XtX: K x K, the full symmetric matrix (lower triangle mirrored from the
 * upper, so it is bit-symmetric).  out_XtY: K x M.  Element type: double in
 * CVGRAM_MODE_FP64, float in the mixed modes.  Either output may be NULL to
 * skip it.  Caller-allocated device memory; enqueued on the handle's stream.
 * Errors: CVGRAM_ERANGE for a bad p.
 */
cvgram_status cvgram_fold(cvgram_t h, int32_t p, void* out_XtX, void* out_XtY);

/* Leakage comparison -- NOT training-partition preprocessing, never the
 * default; for demonstrating numerically what Section 4.1 shows (a
 * validation fold's rows leak into the training products):
 *   CVGRAM_LEAK_GLOBAL    the handle's combination, but X and Y centred and
 *                         scaled with the means and deviations of ALL N rows
 *                         (divisor N - ddof; a column constant over all rows
 *                         gets deviation 1), then fold p's training rows
 *                         multiplied.  Centering X and Y are independent here.
 *   CVGRAM_LEAK_LINDGREN  Lindgren et al.'s centred products, Equation (20)
 *                         as restated in the proof of Lemma 11:
 *                         (X^T X)_ij - (X_V^T X_V)_ij - xbar_i sum_V X_nj
 *                         - xbar_j sum_V X_ni + (N/P) xbar_i xbar_j, with
 *                         xbar over all rows; X^T Y the same with Y on the
 *                         right.  Needs the handle's combination
 *                         center_x = center_y = 1, no scaling (else EINVAL).
 * Outputs as for cvgram_fold (out_XtY ignored when M == 0).  Returns
 * CVGRAM_ERANGE for a fold out of range, CVGRAM_EINVAL for an unknown kind. */
typedef enum { CVGRAM_LEAK_GLOBAL = 1, CVGRAM_LEAK_LINDGREN = 2 } cvgram_leak;
cvgram_status cvgram_fold_leaky(cvgram_t h, int32_t p, int kind, void* out_XtX, void* out_XtY);

/* Per-fold ridge regression on the device -- a consumer of the training
 * products (the paper names RR and OLS among their models, Section 1): for
 * folds [p0, p1) and the n_lambda >= 1 penalties lambdas[] (HOST array,
 * each >= 0; 0 is ordinary least squares) writes
 *     B[f][l] = (X^T X_T + lambda_l I)^{-1} X^T Y_T
 * for the handle's combination of centering and scaling, into out_B
 * (device, FP64, [p1 - p0][n_lambda][K][M], row-major).  The products are
 * formed in FP64 from the handle's Gram (mixed modes: from their Gram) and
 * solved by a blocked Cholesky factorisation and two triangular solves, all
 * on the device.  Needs M > 0.  Waits on the handle's stream for the
 * positive-definiteness flags: CVGRAM_ESINGULAR when some X^T X_T + lambda I
 * is not positive definite (its B is NaN; the others are written).
 * Errors: CVGRAM_ERANGE for a bad fold range, CVGRAM_EINVAL for M == 0, a
 * negative or non-finite lambda, n_lambda < 1 or NULL pointers,
 * CVGRAM_ENOTSCALABLE when the combination scales and the partitioning is
 * not scalable, CVGRAM_ENOMEM for the workspace. */
cvgram_status cvgram_ridge(cvgram_t h, int32_t p0, int32_t p1, const double* lambdas,
                           int32_t n_lambda, double* out_B);

/* As cvgram_fold, for any of the 16 combinations (flags 0 or 1).  Returns
 * CVGRAM_ENOTSCALABLE if a scale flag is set on a partitioning that is not
 * scalable for the handle's ddof.  Equivalent combinations (Lemma 9) return
 * identical bits. */
cvgram_status cvgram_fold_combo(cvgram_t h, int32_t p, int center_x, int scale_x,
                                int center_y, int scale_y, void* out_XtX, void* out_XtY);

/* All distinct products of folds p_begin <= p < p_end in one launch:
 * out_XtX[(p - p_begin)][c][K][K] for the 4 X^T X classes and
 * out_XtY[(p - p_begin)][c][K][M] for the 8 X^T Y classes (class numbering
 * above).  Either pointer may be NULL.  Every class is written.  With a
 * partitioning that is not scalable (Definition 6), a fold whose
 * |T_p| - ddof < 1 has no training deviation: its scaled classes (1 and 3
 * of X^T X; 1, 2, 3, 5, 6, 7 of X^T Y) are NaN; the other folds' are
 * computed as usual.  Element type as in cvgram_fold. */
cvgram_status cvgram_folds_all(cvgram_t h, int32_t p_begin, int32_t p_end,
                               void* out_XtX, void* out_XtY);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): cvgram_create + cvgram_folds_all(h, 0, P)
 * + cvgram_destroy in one call whose workspace is a fixed scratch array of
 * CVGRAM_NOALLOC_SCRATCH_BYTES that every device the library runs on holds
 * from module load until the process ends; host staging (label counts, the
 * launch plan) is a fixed 16 MiB host buffer.  It calls no hipMalloc,
 * hipHostMalloc, hipFree and creates no event.
 *   X, Y, fold_id, N, K, M, dtype, ddof, mode: as cvgram_create (every class
 *            is computed, so there are no centering/scaling flags).
 *   P        the number of folds the labels give (largest label + 1);
 *            CVGRAM_EFOLDS if they give another (or violate Definition 1).
 *   out_XtX  device [P][4][K][K], out_XtY device [P][8][K][M] (either may be
 *            NULL): every fold's classes as cvgram_folds_all(h, 0, P) writes
 *            them, bit-identical to it.
 * Waits once for the label counts (as cvgram_create does), then returns with
 * the pipeline queued on `stream`.  A problem whose workspace does not fit
 * the scratch (or whose plan exceeds the host staging) returns
 * CVGRAM_EINVAL, with the sizes in cvgram_last_error_message(), before any
 * Gram work is queued.  Every call on a device shares that device's scratch:
 * calls are serialised on the host, and calls on one device whose device
 * work may overlap (different streams without ordering between them) race;
 * calls on one stream are ordered.  The pipeline initialises every scratch
 * location it reads, so nothing has to start at zero. */
#define CVGRAM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
cvgram_status cvgram_folds_all_noalloc(const void* X, const void* Y, const int32_t* fold_id,
                                       int64_t N, int64_t K, int64_t M, cvgram_dtype dtype,
                                       int ddof, cvgram_mode mode, int32_t P, void* stream,
                                       void* out_XtX, void* out_XtY);

/* Training-partition statistics of fold p in FP64: column means
 * (Definition 2) and deviations with divisor |T_p| - ddof (Definition 4);
 * a column constant over T_p reports deviation 1 (Algorithm 7 step 24).
 * Device pointers of length K, K, M, M; any may be NULL.  If the partition is
 * not scalable, deviations of folds with |T_p| - ddof < 1 are NaN. */
cvgram_status cvgram_fold_stats(cvgram_t h, int32_t p, double* mean_x, double* std_x,
                                double* mean_y, double* std_y);

/* Per-stage device timing.  When enabled (process-wide; off by default),
 * cvgram_create records HIP events on its stream around its stages and
 * cvgram_stage_times() returns their durations in milliseconds, waiting for
 * them if needed: ms[0] fold bookkeeping (includes the host's wait for the
 * label counts and its planning), ms[1] column statistics (packing),
 * ms[2] grouped Gram launch, ms[3] slab reduction.
 * n is the capacity of ms (at most 4 entries are written).  Returns
 * CVGRAM_EINVAL if the handle was created with timing off. */
cvgram_status cvgram_set_stage_timing(int on);
cvgram_status cvgram_stage_times(cvgram_t h, double* ms, int32_t n);

/* Device workspace released by cvgram_destroy() is kept in a per-device
 * cache and reused by later handles of similar size (bounded per device to
 * half of its memory, at least 32 GiB).  cvgram_trim_cache() waits for the work still using cached blocks
 * of the current device, then frees them. */
cvgram_status cvgram_trim_cache(void);

/* ---------------------------------------------------------------------------
 * Batched form: many independent cross-validation problems (different N, K,
 * M and P) computed together.  Every stage runs as one launch over all
 * problems (one grouped MFMA Gram launch for every fold of every problem),
 * and the whole pipeline -- pivots, pack pass with validation-block
 * statistics, training statistics, grouped Gram, slab reduction and the 12
 * distinct training products of every fold (Algorithm 7 generalised as in
 * Table 1) -- is captured once in a HIP graph and replayed by
 * cvgram_batch_run().
 * ------------------------------------------------------------------------- */
typedef struct cvgram_batch* cvgram_batch_t;

typedef struct {
  const void* X;            /* device, N x K row-major, element type of the batch */
  const void* Y;            /* device, N x M row-major; NULL only when M == 0      */
  const int32_t* fold_id;   /* device, N labels (Definition 1, 0-based)            */
  int64_t N, K, M;
  void* out_XtX;            /* device, [P][4][K][K] (class order above), or NULL   */
  void* out_XtY;            /* device, [P][8][K][M], or NULL                       */
} cvgram_problem;

/* Validate and plan a batch of n problems (n >= 1), all of element type
 * `dtype`, arithmetic `mode` and deviation divisor |T_p| - ddof.  Runs the
 * fold bookkeeping of every problem (Algorithm 1; waits on `stream`), checks
 * Definition 1 (CVGRAM_EFOLDS, with the failing problem's index in the error
 * message), allocates one workspace for the batch and captures the pipeline
 * into a HIP graph on `stream`.  Every class is written; in a problem whose
 * partitioning is not scalable for ddof (Definition 6), the scaled classes
 * of the folds with |T_p| - ddof < 1 are NaN (as in cvgram_folds_all).
 * Problem arrays and outputs are borrowed: they must stay valid until
 * cvgram_batch_destroy(); their contents may change between runs (the fold
 * labels must not).  Output element type: double in CVGRAM_MODE_FP64, float
 * otherwise.  Gram tile shapes come from the autotuning table
 * (cvgram_autotune), else from a built-in rule. */
cvgram_status cvgram_batch_create(const cvgram_problem* problems, int32_t n, cvgram_dtype dtype,
                                  int ddof, cvgram_mode mode, void* stream, cvgram_batch_t* out);

/* Replay the captured pipeline on the batch's stream (asynchronous): every
 * problem's outputs are recomputed from the current contents of X and Y. */
cvgram_status cvgram_batch_run(cvgram_batch_t b);

/* Run the same pipeline eagerly (kernel by kernel, no graph) -- identical
 * results; for comparison and debugging. */
cvgram_status cvgram_batch_run_eager(cvgram_batch_t b);

/* Number of folds of problem i, and whether it is scalable (host outputs;
 * either may be NULL). */
cvgram_status cvgram_batch_problem_info(cvgram_batch_t b, int32_t i, int32_t* P,
                                        int32_t* scalable);

/* Wait for the batch's outstanding work, then free it (NULL is a no-op). */
cvgram_status cvgram_batch_destroy(cvgram_batch_t b);

/* ---------------------------------------------------------------------------
 * Autotuner of the grouped Gram launch.  Times the candidate tile widths (64,
 * 128, and in CVGRAM_MODE_BF16X3 the 256 x 128 tiles when K > 128) and
 * work-list sizes on the given problem (device data as in
 * cvgram_create), records the fastest in a process-wide table keyed by the
 * device (architecture name and compute-unit count), mode, dtype and K,
 * M + 1, N and the mean fold size N / P rounded up to powers of two, and
 * returns it.  Later cvgram_create / cvgram_batch_create calls on the same
 * kind of device whose problem falls in a tuned bucket use the recorded
 * choice.  With the environment variable CVGRAM_TUNE_FILE set, the table is
 * loaded from that file at first use (one entry per line: device key, the
 * six bucket numbers, tile, work-list size; entries of other devices are
 * kept and ignored) and rewritten after each tuning.  Waits on `stream`.
 * ------------------------------------------------------------------------- */
cvgram_status cvgram_autotune(const void* X, const void* Y, const int32_t* fold_id, int64_t N,
                              int64_t K, int64_t M, cvgram_dtype dtype, cvgram_mode mode,
                              void* stream, int32_t* tile, int32_t* target_items);

/* Autotuner of a batch's Gram launches, in the batch itself: times the
 * batch's problems (as cvgram_batch_create would plan them, pack through
 * slab reduction, eager) under each candidate widest tile (64, 128, and in
 * CVGRAM_MODE_BF16X3 256 x 128 tiles, for every problem the built-in rule
 * gives them or only for K >= 512; every problem's tile is capped by its own
 * widest under the built-in rule) and work-list size (512 .. 16384 items),
 * and records the fastest for
 * every problem's bucket of the table above, so that a following
 * cvgram_batch_create of these problems uses it.  Tuning each problem alone
 * (cvgram_autotune) can choose narrow tiles that give a lone small problem
 * enough work items but lose inside a batch, where the problems share the
 * launch.  problems[i]: as for cvgram_batch_create (outputs are not
 * touched); ddof does not change the timing and is taken as 1.  Outputs
 * (host, each may be NULL): the widest tile chosen, the smallest K that
 * takes 256 x 128 tiles under it (0: every problem the built-in rule gives
 * them), the work-list size, and their Gram-stage time in ms.  Waits on
 * `stream`. */
cvgram_status cvgram_batch_autotune(const cvgram_problem* problems, int32_t n,
                                    cvgram_dtype dtype, cvgram_mode mode, void* stream,
                                    int32_t* max_tile, int32_t* wide_min_k,
                                    int32_t* target_items, double* gram_ms);

/* The plan cvgram_create chose for this handle (host values):
 *   info[0] tile width of the Gram launch (64, 128, or 256: 256 x 128 tiles)
 *   info[1] Gram work items (output tile x fold row range)
 *   info[2] slabs (per-fold row splits whose partial products are summed)
 *   info[3] 1 for the fused fold path (many small folds), else 0
 *   info[4] bytes per element of the packed panels the Gram launch reads
 *           (FP64 mode: 8, or 4 when FP32 input is kept in FP32 panels; FP32
 *           mode: 4; BF16X3: 2 per panel, hi and lo)
 * n is the capacity of info (at most 5 entries are written). */
cvgram_status cvgram_plan_info(cvgram_t h, int64_t* info, int32_t n);

/* Host-side preview of the plan cvgram_create would make for a problem of
 * this shape whose fold p has fold_sizes[p] rows (Definition 1: each >= 1,
 * summing to N), with no device work and no device allocation; the tuned
 * choice of the current device applies (none on a host without a device).
 *   info[0..4] as cvgram_plan_info
 *   info[5] bytes of device workspace cvgram_create would allocate (packed
 *           panels, statistics, slabs, the full Gram; not the plan upload of
 *           a few MB or the caller's outputs)
 *   info[6], info[7] the most and the fewest Gram work items one XCD runs in
 *           the Gram launch with the most items
 * n is the capacity of info (at most 8 entries are written).  Errors:
 * CVGRAM_EINVAL for a bad shape, dtype or mode, or sizes not summing to N;
 * CVGRAM_EFOLDS for an empty fold. */
cvgram_status cvgram_plan_query(int64_t N, int64_t K, int64_t M, const int64_t* fold_sizes,
                                int32_t P, cvgram_dtype dtype, cvgram_mode mode, int64_t* info,
                                int32_t n);

/* Change the stream used by later calls on this handle.  Work queued on the
 * new stream from then on runs after everything already queued on the old
 * one (an event recorded there is waited for on the device, not the host). */
cvgram_status cvgram_set_stream(cvgram_t h, void* stream);

/* Free the handle (NULL is a no-op) without waiting for its queued work:
 * its workspace goes back to the per-device cache in stream order, tagged
 * with an event recorded on the handle's stream now.  Later work on the same
 * stream reuses it at once (stream order puts that work behind this
 * handle's); other streams, and the host for pinned blocks, reuse it only
 * once that event has completed.  Outputs of the handle's calls are complete
 * when the stream reaches this point; device errors of that work surface at
 * the caller's next synchronisation. */
cvgram_status cvgram_destroy(cvgram_t h);

/* Static description of a status code. */
const char* cvgram_status_string(cvgram_status s);

/* Details of the last error raised on the calling thread ("" if none). */
const char* cvgram_last_error_message(void);

/* Library version as major*10000 + minor*100 + patch. */
int32_t cvgram_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CVGRAM_H */
