/*
 * oica.h -- C ABI of the MI355X (gfx950) hot path of matrix-form ordering ICA.
 *
 * Paper: Y. Matsuda and K. Yamaguchi, "Efficient Estimation of Unique Components
 * in Independent Component Analysis by Matrix Representation", arXiv 2408.17118.
 * The paper states the problem as: given whitened observations X and the
 * hyper-parameters (number of random starts, iteration cap, threshold), return
 * the separating rows in the order of the ordering criterion.  The calls below
 * follow that statement: whitening (done "in advance" in the paper), the batched
 * fixed point over many random starts, and the selection of unique components.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Layout is row-major.  X and Xw are N x T (T samples, contiguous per row).
 *    W0, W and U hold one vector per row (K x N or n x N).
 *  - Every array argument is a caller-owned DEVICE pointer unless its comment
 *    says "host".  The library never frees caller memory and keeps no pointer
 *    to it after a call returns.  The library owns its context and an internal
 *    workspace that grows on demand and is freed by oica_destroy.
 *  - All work is enqueued on the context's HIP stream.  A call returns after
 *    enqueueing unless its comment says it synchronises (calls that report a
 *    count or a data-dependent error to the host do).  The batched fixed point
 *    also runs per-dataset work on four streams of its own (default priority,
 *    created on first use, destroyed with the context), and the batched
 *    whitening the last steps of its problems with N <= 64 on the first of
 *    them, ordered against the context's stream by events, so that the
 *    context's stream is still the only one the caller orders against; both
 *    synchronise before returning.
 *  - Return value: OICA_OK (0) or a negative OICA_E_* code.  Argument errors
 *    are detected on the host before any device work, so they can be tested
 *    without a GPU.  After an error, oica_last_error() gives a readable detail.
 *    Per-row outcomes of the fixed point go in the status array, never in the
 *    return code.
 *  - A context may be used by one host thread at a time.
 */
#ifndef OICA_H
#define OICA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oica_ctx oica_ctx;

typedef enum { OICA_F64 = 0, OICA_F32 = 1, OICA_BF16 = 2 } oica_dtype;

enum {
  OICA_OK = 0,
  OICA_E_ARG = -1,         /* null pointer, bad size, bad parameter          */
  OICA_E_SHAPE = -2,       /* output capacity too small                      */
  OICA_E_RANK = -3,        /* covariance singular: data cannot be whitened   */
  OICA_E_NONFINITE = -4,   /* NaN or Inf in the input                        */
  OICA_E_DEVICE = -5,      /* HIP runtime error                              */
  OICA_E_NOMEM = -6,       /* workspace allocation failed                    */
  OICA_E_UNSUPPORTED = -7, /* size or dtype outside what the kernels handle  */
  OICA_E_NOCONV = -8       /* an eigensolver did not converge within its
                              sweep limit (the Jacobi solves of oica_whiten
                              and oica_deflation)                          */
};

/* Per-row outcome of the fixed point (status array). */
enum {
  OICA_ROW_NOTCONV = 0,    /* still moving after max_iter passes             */
  OICA_ROW_CONV = 1,       /* step fell below the threshold                  */
  OICA_ROW_PRUNED = 2,     /* dropped by the learned pruner (state kept)     */
  OICA_ROW_DEGENERATE = 3  /* update had zero or non-finite norm             */
};

/* Largest number of components (dimension N) the kernels handle. */
#define OICA_MAX_N 128

/* Version of this ABI: major * 10000 + minor * 100 + patch. */
int oica_version(void);

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the legacy default stream).  *out (host) receives the
 * handle.  device == OICA_NO_DEVICE makes a context without a device, which
 * makes no HIP call: every call on it returns its argument errors as on a
 * device and OICA_E_DEVICE where device work would begin (input validation on
 * a host without a GPU).  Errors: OICA_E_ARG (out == NULL, device out of
 * range), OICA_E_DEVICE. */
#define OICA_NO_DEVICE (-1)
int oica_create(oica_ctx **out, int device, void *hip_stream);

/* Destroy a context and free its workspace (synchronises its stream). NULL is a no-op. */
void oica_destroy(oica_ctx *ctx);

/* Static name of a return code. Never NULL. */
const char *oica_status_string(int status);

/* Detail of the last error on ctx (valid until the next call on ctx); "" if none. */
const char *oica_last_error(const oica_ctx *ctx);

/* Change the stream later calls enqueue on. */
int oica_set_stream(oica_ctx *ctx, void *hip_stream);

/* Process-wide switches for tests of failure handling (every kernel still
 * ends normally), and a counter:
 *   OICA_OPT_COOP_GIVE_UP: value 1 makes every later all-rounds clustering
 *     launch start with its give-up flag set, so it ends at its first
 *     exchange and the round-by-round form redoes the clustering from the
 *     start (the path taken when the work-groups are not all resident and the
 *     bounded wait gives up).  0 restores normal launches.
 *   OICA_OPT_JACOBI_MAX_SWEEPS: cap on the Jacobi sweeps of later solves,
 *     1..30 (0 = 30); a solve still rotating at the cap fails with
 *     OICA_E_NOCONV.
 *   OICA_OPT_COOP_FALLBACKS (read only): how many all-rounds clustering
 *     launches ended in the give-up flag and were redone round by round.
 *   OICA_OPT_COOP_LAUNCH_API: 1 (default) launches the all-rounds clustering
 *     with hipLaunchCooperativeKernel (refused when its work-groups cannot
 *     all be resident: the round-by-round form runs instead); 0 uses a plain
 *     launch after the same occupancy check (for tools that do not follow
 *     cooperative launches; the bounded wait still covers residency).
 * Errors: OICA_E_ARG (unknown option or value out of range). */
enum { OICA_OPT_COOP_GIVE_UP = 1, OICA_OPT_JACOBI_MAX_SWEEPS = 2, OICA_OPT_COOP_FALLBACKS = 3,
       OICA_OPT_COOP_LAUNCH_API = 4 };
int oica_set_option(int option, int value);
int oica_get_option(int option, int *value);

/* ---------------------------------------------------------------------------
 * Whitening (Sec. 2.2: the observations are whitened before the method runs,
 * so that every unit row w gives a component with zero mean and unit variance,
 * the constraints of Theorem 1).
 *
 *   mean = X 1 / T;  C = (X - mean)(X - mean)^T / T   (FP64, divided by T)
 *   C = E D E^T, eigenvalues descending, each eigenvector's largest-magnitude
 *   entry positive;  V = D^(-1/2) E^T;  Xw = V (X - mean).
 *
 * N in [1, OICA_MAX_N], T > N.  X_raw: N x T of raw_t (OICA_F64 or OICA_F32),
 *   row n starting at element n * ld_raw (ld_raw >= T, in elements; ld_raw == T
 *   for a contiguous array), so that a window of a longer recording is read in
 *   place.  Only the first T elements of each row are read.
 * Xw: N x T of out_t (OICA_F32 or OICA_BF16, round to nearest even).
 * Xw_f32: optional extra FP32 copy (N x T) written when out_t == OICA_BF16,
 *   needed later by the FP32 refinement and by the final kurtosis; NULL to skip.
 * V (N x N), mean (N), eigval (N): FP64 outputs; any may be NULL.
 * Synchronises.  Errors: OICA_E_ARG, OICA_E_SHAPE (ld_raw < T),
 * OICA_E_UNSUPPORTED (N > OICA_MAX_N), OICA_E_NONFINITE (NaN/Inf in X_raw),
 * OICA_E_RANK (smallest eigenvalue <= 1e-12 x largest), OICA_E_NOCONV (the
 * Jacobi solve of the covariance still rotating at its sweep limit),
 * OICA_E_NOMEM, OICA_E_DEVICE.
 * ------------------------------------------------------------------------- */
int oica_whiten(oica_ctx *ctx, int N, int64_t T, const void *X_raw, oica_dtype raw_t,
                int64_t ld_raw, void *Xw, oica_dtype out_t, float *Xw_f32,
                double *V, double *mean, double *eigval);

/* Batched whitening: D problems, each exactly as in oica_whiten (same outputs,
 * same arithmetic).  Every pass covers all problems in one launch: the
 * statistics passes (in groups when their partial sums would exceed a fixed
 * scratch cap), the covariance eigenproblems (one work-group per problem) and
 * the apply pass.
 *
 * problems: host array of D (1..1024) descriptors; every pointer in it is a
 * device pointer as in oica_whiten.  out_t applies to every problem.  status
 * is written for every problem: OICA_OK, OICA_E_NONFINITE or OICA_E_RANK.
 * Synchronises.  Returns OICA_OK if every problem succeeded, else the first
 * failing problem's code (argument errors before any device work, naming the
 * problem index in oica_last_error). */
typedef struct {
  int N;
  int64_t T;
  const void *X_raw;
  oica_dtype raw_t;
  int64_t ld_raw;       /* row stride of X_raw in elements, >= T */
  void *Xw;
  float *Xw_f32;        /* nullable */
  double *V, *mean, *eigval;  /* nullable */
  int status;           /* out */
} oica_whiten_problem;

int oica_whiten_batched(oica_ctx *ctx, int D, oica_whiten_problem *problems, oica_dtype out_t);

/* ---------------------------------------------------------------------------
 * The batched kurtosis fixed point with removal of converged rows (Sec. 3.1,
 * eqs. 4-5 in the order of Algorithm 2, and Sec. 3.2), followed by the
 * kurtosis of every final row (eq. 2).
 *
 *   B = rows of W0 normalised (FP64, stored FP32);  every row active.
 *   repeat (at least once, at most max_iter passes):
 *     for the active rows P:  Z = P Xw;  G = (Z o Z o Z) Xw^T / T - 3 P
 *     b = g / ||g||;  d = min(||b - b_prev||, ||b + b_prev||)
 *     d < tol -> CONV (row leaves the active set);  ||g|| == 0 or non-finite
 *     -> DEGENERATE (row keeps b_prev and leaves the active set)
 *   kurt[l] = sum_m (b_l . x_m)^4 / T - 3 over the FP32 data, FP64 sums.
 *
 * precision = OICA_F32: the passes run on FP32 data (Xw of xw_t = OICA_F32).
 * precision = OICA_BF16: the passes run on BF16 data (Xw of xw_t = OICA_BF16;
 *   by default each row carried as BF16 hi + lo parts, see bf16_row_terms;
 *   z^3 rounded to BF16, FP32 sums) with threshold tol_bf16 (1e-3 leaves the
 *   rest to the grouped FP32 passes), until every row has stopped, at most K/64 rows
 *   are left, or the active count has not shrunk over two polls.  Then every
 *   row that converged on BF16 data or was still moving continues on the FP32
 *   copy Xw_f32 (FP32 kernels, threshold tol) for up to
 *   max(refine_iters, max_iter - BF16 passes) passes; only the FP32 test
 *   makes a row CONV.
 * traj: optional K x traj_iters x 2 FP32 record of (kurtosis of the row
 *   before pass t+1, step d of pass t+1); NaN once a row has stopped.
 * ------------------------------------------------------------------------- */
typedef struct oica_pruner oica_pruner;

typedef struct {
  int max_iter;          /* >= 1                                           */
  double tol;            /* > 0, FP32 threshold (1e-6 is the paper's)      */
  oica_dtype precision;  /* OICA_F32 or OICA_BF16                          */
  double tol_bf16;       /* > 0, used when precision == OICA_BF16          */
  int refine_iters;      /* FP32 passes after the BF16 loop (>= 0)         */
  int traj_iters;        /* 0..16: passes recorded into traj               */
  int check_every;       /* host polls the active count every this many
                            passes (>= 1; 0 = default 4)                   */
  int profile;           /* 1: time every fused update launch with HIP
                            events on the context's stream (stats below)   */
  int refine_groups;     /* BF16 only.  0: every row that converged on BF16
                            data takes the FP32 passes.  1: those rows are
                            first grouped (greedy, 1 - |cos| <= 1e-6, i.e.
                            numerically the same BF16 fixed point); only the
                            lowest-index row of each group takes the FP32
                            passes and the kurtosis pass, and the other
                            members receive its row (with their own sign),
                            status and kurtosis.                           */
  const oica_pruner *pruner; /* NULL: plain run.  Else, after pass
                            prune_pass the active rows whose predicted
                            probability of ending in a top-ranked component
                            is below the pruner's threshold become PRUNED
                            (row and counts kept); after the run, if one of
                            the checked components has fewer than guard_min
                            rows, every pruned row is resumed from its saved
                            state and finished.  Checked: with guard_top 0,
                            every accepted component and the cluster where
                            the eq. 3 walk stopped; with guard_top > 0, the
                            first guard_top accepted ones and those whose
                            criterion is within a relative 1e-3 of the
                            guard_top-th.                                  */
  int prune_pass;        /* pass after which to prune (8..16; 0 = 8)       */
  int guard_top;         /* see pruner (0 = every accepted component)      */
  int guard_min;         /* rows each of them must keep (0 = 4)            */
  int bf16_row_terms;    /* BF16 only: how the passes carry each row.
                            2: BF16 hi + lo parts (z to about 2^-17
                            relative; two GEMM1 products per pass), the
                            linear term -3P on the FP32 row.  1: the row
                            rounded once to BF16 (one product), the linear
                            term on the same rounded row, so each pass is
                            the exact update of the rounded row.  3: form 1
                            while a row's last step is >= bf16_switch_step
                            (every row at the first pass; such a row never
                            converges), then form 2.  4: form 2 while the
                            row's last step is >= bf16_switch_step (every
                            row at the first pass), then form 1.  0: the
                            default (2).  Forms 1 and 3 move each row by
                            about 2^-9 of itself per early one-term pass,
                            so a start near the boundary of a basin can
                            end at another fixed point than on FP32 or FP64
                            data; forms 2 and 4 do not in the tests.  The
                            batched entry point has forms 1 and 2 (3 and 4
                            run as 2).                                     */
  double bf16_switch_step; /* forms 3 and 4: switch step (0 = 3e-2)       */
} oica_fp_params;

typedef struct {         /* host */
  int64_t thread_iters;  /* sum over passes of the active rows             */
  int passes;            /* passes that had at least one active row        */
  int64_t refine_thread_iters; /* FP32 refinement row updates (BF16 mode)  */
  double ms;             /* wall time of the call (stream-synchronised)    */
  double update_ms;      /* profile = 1: summed duration of every fused
                            update launch (launches issued after the last
                            row stopped, before the next poll, exit at once) */
  int update_launches;   /* profile = 1: number of those launches          */
  int pruned;            /* rows pruned (pruner set)                       */
  int guard_tripped;     /* 1: the guard resumed the pruned rows           */
} oica_fp_stats;

/* N in [1, OICA_MAX_N], T > N, K >= 1.
 * Xw: N x T of xw_t; Xw_f32: N x T FP32 (may equal Xw when xw_t == F32; required).
 * W0: K x N FP32 (rows need not be normalised; a zero row ends DEGENERATE).
 * Outputs, all K rows in the original row order: W_out K x N FP32 unit rows,
 * kurt K FP64, iters K int32 (updates applied to the row), status K uint8.
 * In BF16 mode with refine_groups, rows left PRUNED take no kurtosis pass:
 * their kurt is NaN (they are never candidates of oica_unique).
 * traj may be NULL when traj_iters == 0; stats (host) may be NULL.
 * Synchronises (the active count is polled on the host).
 * Errors: OICA_E_ARG, OICA_E_UNSUPPORTED, OICA_E_NOMEM, OICA_E_DEVICE. */
int oica_fixed_point(oica_ctx *ctx, int N, int64_t T, const void *Xw, oica_dtype xw_t,
                     const float *Xw_f32, int K, const float *W0, const oica_fp_params *params,
                     float *W_out, double *kurt, int32_t *iters, uint8_t *status,
                     float *traj, oica_fp_stats *stats);

/* One unnormalised update for K given rows (eqs. 4-5, Algorithm 2 order):
 * G = (Z o Z o Z) Xw^T / T - 3 B with Z = B Xw, and s4 = sum_m z^4 / T per row.
 * B: K x N FP32 (used as given, not normalised).  G: K x N FP64, s4: K FP64.
 * xw_t = OICA_F32 or OICA_BF16 selects the kernel family of oica_fixed_point's
 * passes (BF16: each row carried as a BF16 pair hi + lo with lo = b - hi, z^3
 * rounded to BF16, FP32 sums).  Does not synchronise. */
int oica_update(oica_ctx *ctx, int N, int64_t T, const void *Xw, oica_dtype xw_t, int K,
                const float *B, double *G, double *s4);

/* Kurtosis of eq. (2) for K rows: kurt[l] = sum_m (b_l . x_m)^4 / T - 3,
 * FP32 products of FP32 data with FP64 sums over samples.  Does not synchronise. */
int oica_kurtosis(oica_ctx *ctx, int N, int64_t T, const float *Xw_f32, int K,
                  const float *W, double *kurt);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kurtosis as oica_kurtosis (same kernels, bitwise the same result), with its
 * per-split partial sums in a fixed library-owned device array of
 * OICA_NOALLOC_SCRATCH_BYTES per device (held from library load until the
 * process ends) instead of the context's workspace.  Allocates nothing and
 * does not synchronise.  Every call on a device shares that device's array
 * and overwrites it; calls that overlap on one device (other streams, other
 * contexts, other host threads) race and must be serialised by the caller.
 * Nothing needs clearing between calls.  Errors: as oica_kurtosis, plus
 * OICA_E_UNSUPPORTED when K needs more partial sums than the array holds
 * (above about two million rows). */
#define OICA_NOALLOC_SCRATCH_BYTES (16 * 1024 * 1024)
int oica_kurtosis_noalloc(oica_ctx *ctx, int N, int64_t T, const float *Xw_f32, int K,
                          const float *W, double *kurt);

/* ---------------------------------------------------------------------------
 * Learned pruner (an extension beyond the paper, built on its trajectories):
 * a 16 -> 64 -> 64 -> 1 network (ReLU, sigmoid) reads, for the first eight
 * passes of a start vector, the kurtosis before the pass and log10 of the step
 * (features interleaved per pass, standardised with fixed statistics) and
 * predicts whether the vector ends in one of the top-ranked components.  The
 * forward pass uses FP16 weights with FP32 arithmetic; training keeps FP32
 * master weights and Adam moments.  Parameters are packed W1 (64 x 16, row
 * major), b1 (64), W2 (64 x 64), b2 (64), w3 (64), b3 (1).
 * ------------------------------------------------------------------------- */
#define OICA_PRUNER_PARAMS 5313

/* init_w: host, OICA_PRUNER_PARAMS FP32; feat_mean, feat_std: host, 16 each
 * (std > 0).  The pruner lives on ctx's device.  Synchronises. */
int oica_pruner_create(oica_ctx *ctx, const float *init_w, const float *feat_mean,
                       const float *feat_std, oica_pruner **out);
void oica_pruner_destroy(oica_pruner *p);
/* FP32 master weights to host (OICA_PRUNER_PARAMS floats).  Synchronises. */
int oica_pruner_get_weights(oica_ctx *ctx, const oica_pruner *p, float *host_w);
int oica_pruner_set_threshold(oica_pruner *p, float theta);
/* prob[r] = network output for traj rows r = 0..R-1 (traj: R x 8 x 2 FP32). */
int oica_pruner_predict(oica_ctx *ctx, const oica_pruner *p, const float *traj, int64_t R,
                        float *prob);
/* Mean loss (host) and its gradient (device, OICA_PRUNER_PARAMS FP32) over R
 * rows: binary cross-entropy with positive-class weight w_pos.  Synchronises. */
int oica_pruner_grad(oica_ctx *ctx, const oica_pruner *p, const float *traj,
                     const uint8_t *labels, int64_t R, float w_pos, float *grad, double *loss);
/* One Adam step (lr; betas 0.9, 0.999; eps 1e-8) on the gradient of the rows
 * given; the loss before the step goes to *loss (host, may be NULL). */
int oica_pruner_train_step(oica_ctx *ctx, oica_pruner *p, const float *traj,
                           const uint8_t *labels, int64_t R, float w_pos, float lr, double *loss);
/* Training run: epochs passes over the R rows (traj: R x 8 x 2 FP32, labels:
 * R, device), each in a fresh pseudo-random order drawn from seed and the
 * epoch number (a keyed permutation evaluated on the device, so the same seed
 * gives the same weights), cut into consecutive steps of batch rows (the last
 * one shorter); every step is oica_pruner_train_step on its rows.  w_pos: the
 * positive-class weight, or 0 for n_negative / n_positive of the labels.
 * epoch_loss: host, epochs doubles (may be NULL): the mean over the epoch's
 * steps of each step's loss before its update.  Synchronises when it counts
 * the labels or reports losses.  Errors: OICA_E_ARG (null pointers, R < 1,
 * epochs outside [1, 100000], batch < 1, lr <= 0, w_pos < 0, all labels
 * positive with w_pos 0), OICA_E_NOMEM, OICA_E_DEVICE. */
int oica_pruner_train(oica_ctx *ctx, oica_pruner *p, const float *traj, const uint8_t *labels,
                      int64_t R, int epochs, int batch, float w_pos, float lr, uint64_t seed,
                      double *epoch_loss);

/* ---------------------------------------------------------------------------
 * Batched form: D independent problems of uneven N, T and K run the passes of
 * oica_fixed_point together, one persistent kernel launch per pass for the
 * whole batch (a work queue of (problem, row block, sample split) items).
 * Each problem's sample partition depends on its own T only and the tuned tile
 * shape only regroups independent rows, so every problem's results are the
 * same alone (D = 1) or in any batch and under any tuner choice.
 * ------------------------------------------------------------------------- */
typedef struct {          /* host array of D entries; all pointers DEVICE   */
  int N;                  /* [1, OICA_MAX_N]                                */
  int64_t T;              /* > N                                            */
  int K;                  /* >= 1                                           */
  const void *Xw;         /* N x T of xw_t                                  */
  const float *Xw_f32;    /* N x T FP32 (may equal Xw for FP32 data)        */
  const float *W0;        /* K x N                                          */
  float *W_out;           /* K x N unit rows, original row order            */
  double *kurt;           /* K                                              */
  int32_t *iters;         /* K                                              */
  uint8_t *status;        /* K                                              */
} oica_problem;

typedef struct {
  int autotune;           /* 1: time the candidate tile shapes (rows per wave
                             per padded-N bucket, persistent grid size) on
                             the first pass unless the choice is cached     */
  const char *cache_path; /* host string: JSON-lines file of tuned choices,
                             read and appended (NULL: context memory only)  */
  int force_wk;           /* 0: tuned or default; 1 or 2: rows per wave of
                             32-row blocks for padded N <= 64              */
  int force_grid;         /* 0: tuned or default; else work-groups          */
} oica_batch_params;

typedef struct {          /* host */
  int64_t thread_iters;   /* all problems, main loop                        */
  int64_t refine_thread_iters; /* all problems, FP32 passes after BF16      */
  int passes;             /* batched passes with at least one active row    */
  double ms;              /* wall time of the call                          */
  double update_ms;       /* params->profile = 1: persistent-kernel time    */
  int update_launches;
  int grid;               /* work-groups of the persistent kernel           */
  int wk32, wk64;         /* rows-per-wave choice for padded N 32 and 64    */
  int tuned;              /* 1: chosen by timing in this call; 2: from cache */
  double update_flops;    /* algorithmic flops of the main-loop passes:
                             sum over problems of 4 N T thread_iters        */
} oica_batch_stats;

/* D in [1, 1024].  params as for oica_fixed_point (traj_iters must be 0; the
 * pruner is not used).  BF16 mode with refine_groups = 1: per problem, the rows
 * that converged on BF16 data are grouped as in oica_fixed_point and one row
 * per group takes the FP32 passes with the rows still moving (one batched
 * launch per pass for all problems); with refine_groups = 0 every such row
 * does.  bparams and stats may be NULL.
 * Synchronises.  Errors: OICA_E_ARG (naming the problem index),
 * OICA_E_UNSUPPORTED, OICA_E_NOMEM, OICA_E_DEVICE. */
int oica_fixed_point_batched(oica_ctx *ctx, int D, const oica_problem *problems, oica_dtype xw_t,
                             const oica_fp_params *params, const oica_batch_params *bparams,
                             oica_batch_stats *stats);

/* ---------------------------------------------------------------------------
 * Unique components (generalises Algorithm 2's argmax over the random starts
 * and its Gaussianity test, eq. 3, to the whole ordered set):
 *   candidates = rows with status CONV (if none: every non-degenerate row),
 *   with finite kurtosis;  order = upsilon(kurt) descending, then row index,
 *   upsilon(a) = a - 2 log(1 + a/2) (eq. 1, +inf for a <= -2);
 *   greedy leader clustering up to sign in that order: a row joins the first
 *   representative r with 1 - |b . b_r| <= tau, else starts a new cluster;
 *   representatives are output in that order with the sign that makes their
 *   largest-magnitude entry positive;  the Gaussianity walk accepts ranks
 *   r = 1, 2, ... while upsilon_r >= 2 (N - r + 2)(N - r + 1) / T.
 * ------------------------------------------------------------------------- */
typedef struct {
  double tau;            /* clustering threshold on 1 - |cos|, in (0, 1)  */
  int gaussianity_test;  /* 0: accept every cluster                        */
  int n_top;             /* > 0: cap the accepted count                    */
} oica_unique_params;

/* W: K x N FP32 unit rows; kurt: K FP64; status: K uint8 (as from oica_fixed_point).
 * Outputs (device) for the first min(n_unique, cap) clusters: U cap x N FP64,
 * kurt_u, ups_u (cap FP64), rep_thread, cluster_size (cap int32).
 * row_cluster: optional K int32, the rank (0-based, output order) of the
 * cluster each row joined, -1 for rows that were not candidates.
 * n_unique, n_accepted: host.  Synchronises.
 * Errors: OICA_E_ARG; OICA_E_SHAPE if cap < n_unique (the counts are still
 * written, and the first cap clusters). */
int oica_unique(oica_ctx *ctx, int N, int64_t T, int K, const float *W, const double *kurt,
                const uint8_t *status, const oica_unique_params *params, int cap,
                double *U, double *kurt_u, double *ups_u, int32_t *rep_thread,
                int32_t *cluster_size, int32_t *row_cluster, int *n_unique, int *n_accepted);

/* Many problems in one call, each exactly as in oica_unique (the same
 * partition, order, outputs and counts): the per-row passes cover every
 * problem in one launch, and the clustering rounds of all problems with
 * K <= 16384 and K N <= 2^19 run in one launch (one work-group per problem).
 * problems: host array of D (1..1024) descriptors whose pointers are device
 * pointers as in oica_unique; n_unique and n_accepted are written back.
 * Synchronises.  Errors: OICA_E_ARG (argument errors before any device work,
 * naming the problem); OICA_E_SHAPE for the first problem with cap < n_unique
 * (every problem's counts and first cap clusters are still written). */
typedef struct {
  int N;
  int64_t T;
  int K;
  const float *W;
  const double *kurt;
  const uint8_t *status;
  int cap;
  double *U, *kurt_u, *ups_u;
  int32_t *rep_thread, *cluster_size;
  int32_t *row_cluster;   /* nullable */
  int n_unique, n_accepted;  /* out */
} oica_unique_problem;

int oica_unique_batched(oica_ctx *ctx, int D, oica_unique_problem *problems,
                        const oica_unique_params *params);

/* ---------------------------------------------------------------------------
 * The deflation driver: Algorithm 2's outer loop (Sec. 3.3, eqs. 6-8), one
 * component per step on data reduced to the complement of the components
 * found so far.
 *
 *   for i = 1, 2, ..., N:
 *     F = I_N - W^T W with its bottom i-1 rows deleted (F~, (N-i+1) x N);
 *     G = (F~ F~^T)^(-1/2) F~ (at i = 1, G = I);  X~ = G Xw;
 *     the batched fixed point (as oica_fixed_point, with params) on X~ from
 *       step i's start rows;  p = the converged row of largest criterion
 *       (eq. 1; lowest row on ties);
 *     stop if upsilon_p < 2 (N-i+2)(N-i+1) / T (eq. 3; only with
 *       gaussianity_test != 0, else all N steps run);
 *     W <- [W; b_p G], the new row normalised in FP64.
 *
 * Xw: N x T FP32 whitened data (row stride T).  With params->precision ==
 * OICA_BF16 every step's X~ is also rounded to BF16 for the BF16 passes.
 * L: start rows per step.  W0: device FP32, the start rows of every step one
 * block after the other: step i's block is L x (N - i + 1), row-major, at
 * element offset L * sum_{k < i} (N - k + 1) (L N (N + 1) / 2 values in all).
 * tau: the clustering threshold of oica_unique (0 < tau < 1), which picks p.
 * W_out: device N x N FP64; its first *n_found rows are the components in the
 * order found (unit rows, orthonormal).  n_found: host.  steps: host array of
 * N records, nullable; entries past the last step taken are left untouched.
 * params->pruner must be NULL and traj_iters 0.  Synchronises.
 * Errors: as oica_fixed_point; OICA_E_RANK when a step's F~ F~^T is singular
 * (smallest eigenvalue <= 1e-12 x largest). */
typedef struct {
  int dim;               /* N - i + 1                                      */
  int rep;               /* p: the chosen start row of the step            */
  int accepted;          /* 1: b_p G was appended; 0: eq. 3 ended the loop */
  int passes;            /* fixed-point passes of the step                 */
  int64_t thread_iters;  /* row updates of the step (BF16 or FP32)         */
  int64_t refine_thread_iters; /* FP32 finish row updates (BF16 mode)      */
  double alpha;          /* kurtosis of row p on X~                        */
  double upsilon;        /* eq. 1 at alpha                                 */
  double threshold;      /* eq. 3's right-hand side for step i             */
} oica_deflation_step;

int oica_deflation(oica_ctx *ctx, int N, int64_t T, const float *Xw, int L, const float *W0,
                   const oica_fp_params *params, double tau, int gaussianity_test, double *W_out,
                   int *n_found, oica_deflation_step *steps);

/* ---------------------------------------------------------------------------
 * The original ordering ICA (Algorithm 1, Sec. 2.2) as a batched variant:
 * the L runs of a step are the rows of one fixed point on the full data, with
 * Algorithm 1's projection.
 *
 *   for i = 1, 2, ..., N:  E = W^T W (E = 0 at i = 1);
 *     every start row w <- w - E w, normalised; every pass
 *       w <- Xw (y o y o y)^T / T - 3 w,  w <- w - E w,  normalised,
 *     with the step test and removal of converged rows of oica_fixed_point;
 *     p = the run of largest criterion (eq. 1) over every run, converged or
 *       not (lowest row on ties);
 *     stop if upsilon_p < 2 (N-i+2)(N-i+1) / T (eq. 3; only with
 *       gaussianity_test != 0);  W <- [W; w_p] (normalised in FP64).
 *
 * Arguments as oica_deflation, except: W0 holds N blocks of L x N start rows
 * (step i's block at element offset (i - 1) L N); params->precision must be
 * OICA_F32; the steps' dim is N.  Synchronises.  Errors: as oica_fixed_point. */
int oica_ordering_original(oica_ctx *ctx, int N, int64_t T, const float *Xw, int L,
                           const float *W0, const oica_fp_params *params, double tau,
                           int gaussianity_test, double *W_out, int *n_found,
                           oica_deflation_step *steps);

#ifdef __cplusplus
}
#endif
#endif /* OICA_H */
