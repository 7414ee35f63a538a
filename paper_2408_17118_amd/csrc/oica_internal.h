// Internal declarations shared by the host runtime and the kernel translation
// units of liboica.  Nothing here is part of the public ABI (include/oica.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/oica.h"
#include "row_perm.h"

namespace oica {

constexpr int WAVES_PER_WG = 4;      // waves per work-group of the fused kernels
// Waves per work-group of the single-problem BF16 pass kernel at padded
// dimension np: for the widest tiles eight waves share one staged X tile,
// which halves the staging work per row; below that (two 32-row blocks per
// wave already) four waves measured faster.
__host__ __device__ constexpr int bf16_waves(int np) { return np >= 96 ? 8 : 4; }
constexpr int SPLIT_GROUP_HOST = 16; // splits per first-stage reduction item

// Device-side bookkeeping of one fixed-point run.  Written by single lanes of
// the fixed-point kernels; read back by the host when it polls.
struct FpControl {
  int kact[2];            // active-row count, double buffered by pass parity
  int passes;             // passes that had at least one active row
  int pad;
  long long thread_iters; // sum over passes of the active-row count
  int kc[2];              // BF16 switched form: the first kc rows of a pass's
                          // active list take the one-term (coarse) form; the
                          // first pass of a run takes it for every row
  int kf;                 // rows entering the hi + lo (fine) form, staged by
                          // the epilogue before they join the list's tail
  int pad2;
};
// How BF16 passes carry a row (the BF16 kernel's row form).  BF_SWITCH: one
// term while the row's step is large, then hi + lo; BF_LATE: hi + lo while the
// step is large, then one term.  Both keep the active list as a head (the
// first form) and a tail (the second).
enum BfRowForm { BF_ONE = 1, BF_HILO = 2, BF_SWITCH = 3, BF_LATE = 4 };

// Launch plan of the fused update kernel.  The grid is fixed for a whole run;
// each work-group derives its (row block, sample split) from the active count
// it reads on the device, so no host round trip is needed between passes.
struct FusedPlan {
  int grid;         // work-groups launched (multiple of 8)
  int max_splits;   // cap on sample splits (each split >= a minimum length)
  int kwg;          // rows per work-group
  int n_sub;        // 32-sample sub-tiles covering T
  long long ld;     // row stride of X in elements (T, or T rounded up for 16-byte rows)
  int thin = 0;     // FP32 only: one 32-row block per item, each wave of a
                    // work-group on its own split (WAVES_PER_WG times the splits)
};

// Row stride that makes every row of X start on a 16-byte boundary.
inline long long aligned_ld(long long T, int esize) {
  const long long per = 16 / esize;
  return (T + per - 1) / per * per;
}
// Copy of an N x T matrix into rows of stride ld (ld >= T); esize 2 or 4.
hipError_t launch_pad_rows(hipStream_t st, const void *src, int esize, int N, long long T,
                           void *dst, long long ld);

// Number of sample splits used when n_kb row blocks are active.  Host and
// device evaluate the same expression.
__host__ __device__ inline int plan_splits(const FusedPlan &p, int n_kb) {
  if (n_kb <= 0) return 0;
  int s = (p.thin ? WAVES_PER_WG * p.grid : p.grid) / n_kb;
  if (s > p.max_splits) s = p.max_splits;
  if (s < 1) s = 1;
  return s;
}

// The learned pruner's device state.
struct PrunerState {
  float *w32 = nullptr;   // FP32 master weights
  void *w16 = nullptr;    // FP16 copy used by every forward pass
  float *m = nullptr;     // Adam moments
  float *v = nullptr;
  float mean[16];         // feature standardisation
  float stdv[16];
  float theta = 0.f;      // prune threshold on the predicted probability
  int step = 0;           // Adam steps taken
};

// One dataset of the batched form (device array, one entry per dataset).
struct BatchDesc {
  const void *X;       // pass data, FP32 or BF16 (N x T)
  const float *X32;    // FP32 copy
  float *B;            // K x N rows (the caller's W_out)
  int *act0;           // active list read on even passes
  int *act1;           // active list read on odd passes
  FpControl *ctl;
  float *gpart;        // n_sp x (K + 256) x np partial G
  float *s4part;       // n_sp x (K + 256) partial sum z^4
  double *red;         // first-stage reduction sums
  int32_t *iters;
  uint8_t *status;
  long long T;
  long long ld, ld32;  // row strides of X and X32 (elements)
  int N, K, np, wk, kwg, n_sp, n_sub, variant;
  int bf_one;          // BF16 passes on the BF16-rounded rows (one-term form)
};

// Batched FP32 variants from THIN_VARIANT on (+ np / 32 - 1), for problems
// with few active rows: one 32-row block per work item, THIN_SPLITS
// times the problem's usual splits, each wave of the work-group on its own
// split (an item covers THIN_SPLITS consecutive splits).
constexpr int THIN_VARIANT = 16;
constexpr int THIN_SPLITS = WAVES_PER_WG;

// Batch-wide counters of one pass.
struct BatchCtl {
  int counter[2];      // work-queue heads, by pass parity
  int total_items;
  int total_epi;
  long long total_red;
};

// ---- launchers (defined next to their kernels) ----------------------------

// unique.hip: greedy leader clustering of one problem in one work-group
struct ClusterJob {
  int K, N;
  const float *W;      // K x N rows
  const float *Wt;     // N x K: the same rows transposed
  const double *key;   // K: rank key (descending, then row index)
  int *cluster;        // K: -2 not a candidate, -1 candidate; out: cluster id
  int *reps;           // out: representative row of each cluster
  int *ctl;            // out: ctl[1] = number of clusters, ctl[2] = 1
};
constexpr int CW_MAX_K = 4096;
// One problem alone: the one-work-group form only for small K (its row loads
// are latency-bound; larger problems use the all-rounds multi-work-group
// kernel); many problems: whenever K fits, since they run side by side.
inline bool cluster_in_one_wg(int K, bool many) { return K <= (many ? CW_MAX_K : 256); }
hipError_t launch_cluster_wg(hipStream_t st, int D, const ClusterJob *jobs_dev,
                             const ClusterJob &one, double tau, int k_max);

// Appends `item` to list[] for every lane with `take`, with one atomic on
// *counter per wave (lanes in lane order).  Every lane of the wave must call it.
__device__ inline void wave_append(bool take, int item, int *list, int *counter) {
  const unsigned long long mask = __ballot(take);
  if (mask == 0ull) return;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)mask) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, __popcll(mask));
  base = __shfl(base, leader);
  if (take) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = item;
}

// whiten.hip
struct JacJob {        // one symmetric eigenproblem of the Jacobi solver
  int N;
  const double *C;     // N x N, symmetric
  double *E;           // out: N x N eigenvectors (column j = vector j), then N eigenvalues
  double2 *rot;        // rotation log (c, s), jacobi_log_entries(N)
  int *pq;             // rotation log p | q << 16 (q = 0xFFFF: padding index)
  int *sweeps;         // out: sweeps that rotated
  int *flags;          // nullable: |= 4 when the solve is still rotating at its sweep limit
  int max_sweeps;      // sweep limit (<= 30)
};
// Process-wide test switches (oica_set_option).
int jacobi_max_sweeps();
void set_jacobi_max_sweeps(int s);
void set_coop_give_up(bool on);
void set_coop_launch_api(bool on);
int coop_launch_api();
int coop_fallbacks();
size_t jacobi_log_entries(int N);
struct WhitenJob {     // one problem of the batched whitening
  int N;
  int64_t T;
  const void *X;
  oica_dtype raw_t;
  int64_t ld;              // row stride of X in elements, >= T
  void *Xw;
  oica_dtype out_t;
  float *Xw_f32;
  double *V, *mean, *eig;  // nullable outputs
};
size_t whiten_batched_workspace_bytes(int D, const WhitenJob *jobs);
// aux: nullable; with it, the problems with N <= 64 finish (eigen-solve,
// canon, apply) on `aux` between `fork` (recorded on st) and `join` (waited
// for by st), beside the others on st.
hipError_t launch_whiten_batched(hipStream_t st, int D, const WhitenJob *jobs, void *ws,
                                 int *flags_dev, hipStream_t aux, hipEvent_t fork,
                                 hipEvent_t join);
hipError_t launch_jacobi(hipStream_t st, int D, const JacJob *jobs_dev, const JacJob &one,
                         int n_max);
hipError_t launch_apply_rows(hipStream_t st, int N, int n_out, int64_t T, const float *X,
                             int64_t ld, const double *Wh, const double *mean, float *o32,
                             uint16_t *obf);

// deflation.hip
// Reduced basis of the deflation driver for n_prev found components W
// (n_prev x N FP64): Ft = first N - n_prev rows of I - W^T W and C = Ft Ft^T.
hipError_t launch_defl_gram(hipStream_t st, int N, int n_prev, const double *W, double *Ft,
                            double *C);
// From the eigenpairs E of C (n x n, then n eigenvalues): G = E D^(-1/2) E^T Ft
// (n x N) and Wh = G padded to N x N with zero rows; flag |= 1 when the
// smallest eigenvalue is <= rank_tol x the largest.
hipError_t launch_defl_basis(hipStream_t st, int N, int n_prev, const double *Ft, const double *E,
                             double rank_tol, double *G, double *Wh, int *flag);
// Algorithm 1: every row that did not degenerate becomes a selection candidate;
// W[n_prev] = B[rep[0]] normalised in FP64 (B: K x N FP32).
hipError_t launch_mark_runs(hipStream_t st, int K, uint8_t *status);
hipError_t launch_append_row(hipStream_t st, int N, int n_prev, const float *B, const int32_t *rep,
                             double *W);
// W[n_prev] = normalised B[rep[0]] G (B: rows of n = N - n_prev FP32 entries).
hipError_t launch_defl_append(hipStream_t st, int N, int n_prev, const double *G, const float *B,
                              const int32_t *rep, double *W);
hipError_t launch_whiten(hipStream_t st, int N, int64_t T, const void *X, oica_dtype raw_t, int64_t ld,
                         void *Xw, oica_dtype out_t, float *Xw_f32, double *V_out,
                         double *mean_out, double *eig_out, void *ws, size_t ws_bytes,
                         int *flags_dev);
size_t whiten_workspace_bytes(int N, int64_t T);

// fixed_point.hip
int fused_np(int N);  // padded feature count used by the kernels for N
FusedPlan narrow_plan(const FusedPlan &p, int np);
FusedPlan thin_plan(const FusedPlan &p);
// Most active rows for the thin FP32 plan (rows padded to 32 instead of the
// plan's 128 or 256).
constexpr int THIN_PLAN_ROWS = 2 * WAVES_PER_WG * 32;
FusedPlan make_plan(int N, int64_t T, int kmax, bool bf16);
size_t fp_workspace_floats(const FusedPlan &p, int N, int kmax);

hipError_t launch_init_rows(hipStream_t st, int K, int N, const float *W0, float *B,
                            int32_t *iters, uint8_t *status, int *act0, FpControl *ctl,
                            float *traj, int traj_iters, const double *proj = nullptr,
                            int n_proj = 0);
hipError_t launch_fused_update(hipStream_t st, const FusedPlan &p, int N, int64_t T,
                               const void *X, bool bf16, const float *B, const int *act,
                               const int *kact_dev, int kact_host, float *gpart, float *s4part,
                               FpControl *ctl, int pass, int bf_form = BF_HILO);
size_t fp_reduce_doubles(const FusedPlan &p, int N, int kmax);
hipError_t launch_epilogue(hipStream_t st, const FusedPlan &p, int N, int64_t T, int kmax,
                           float *B, const int *act_cur, int *act_next, FpControl *ctl, int pass,
                           const float *gpart, const float *s4part, double *red, double tol,
                           int32_t *iters, uint8_t *status, float *traj, int traj_iters,
                           const double *proj = nullptr, int n_proj = 0, int bf_form = 0,
                           double switch_step = 0.0, int *fine_list = nullptr);
hipError_t launch_update_out(hipStream_t st, const FusedPlan &p, int N, int64_t T, int K,
                             const float *B, const float *gpart, const float *s4part, double *G,
                             double *s4);
hipError_t launch_kurtosis(hipStream_t st, const FusedPlan &p, int N, int64_t T,
                           const float *X, int K, const float *W, double *s4part64,
                           double *kurt, const int *act = nullptr, const int *kact_dev = nullptr);
// kurt: rows left PRUNED get NaN (they take no kurtosis pass)
hipError_t launch_group_lists(hipStream_t st, int K, const int *cluster, const int *reps,
                              const int *n_groups_dev, uint8_t *status, double *kurt,
                              int *refine_list, FpControl *ctl_refine, const int *left_list,
                              int left, int *kurt_list, FpControl *ctl_kurt);
hipError_t launch_propagate(hipStream_t st, int K, int N, const int *cluster, const int *reps,
                            float *W, uint8_t *status, double *kurt);
hipError_t launch_refine_select(hipStream_t st, int K, uint8_t *status, int *dst, FpControl *ctl,
                                const int *left_list, int left);

// batched.hip
int batch_splits(int64_t T);
int batch_max_datasets();
hipError_t launch_batch_plan(hipStream_t st, const BatchDesc *descs, int D, BatchCtl *bctl,
                             int *item_start, long long *red_start, int *epi_start, int pass,
                             bool dry);
hipError_t launch_fused_batched(hipStream_t st, const BatchDesc *descs, int D, BatchCtl *bctl,
                                const int *item_start, int pass, int grid, bool bf16);
hipError_t launch_epilogue_batched(hipStream_t st, const BatchDesc *descs, int D,
                                   const BatchCtl *bctl, const long long *red_start,
                                   const int *epi_start, int pass, double tol, int kmax_total);

// pruner.hip
hipError_t pruner_alloc(PrunerState *p, const float *init_w, const float *mean, const float *stdv);
void pruner_free(PrunerState *p);
hipError_t launch_pruner_predict(hipStream_t st, const PrunerState *p, const float *traj, long long R,
                                 const int *list, const int *count_dev, float *prob);
size_t pruner_grad_workspace_bytes(long long R);
// Loss and gradient over the R rows base .. base + R - 1 of the order perm.
hipError_t launch_pruner_grad(hipStream_t st, const PrunerState *p, const float *traj,
                              const uint8_t *labels, long long R, const RowPerm &perm,
                              long long base, float w_pos, void *ws, float *grad,
                              double *loss_dev);
hipError_t launch_count_pos(hipStream_t st, const uint8_t *labels, long long R,
                            unsigned long long *count_dev);
hipError_t launch_pruner_adam(hipStream_t st, PrunerState *p, const float *grad, float lr);
hipError_t launch_prune(hipStream_t st, const PrunerState *p, const float *traj, int traj_stride,
                        int *list, int *count_dev, int kmax, uint8_t *status, int *keep,
                        int *keep_count, int *pruned_count);
hipError_t launch_unprune(hipStream_t st, int K, uint8_t *status, int *list, FpControl *ctl);

// unique.hip
struct CoopSlot {      // one work-group's arg-max in the all-rounds clustering
  unsigned long long word;  // (round + 1) << 32 | row index (0xFFFFFFFF: none)
  unsigned long long spare;
};
struct UJob {          // one unique-components problem
  int K, N;
  long long T;
  const float *W;
  const double *kurt;
  const uint8_t *status;
  double tau;
  int gtest, n_top, cap;
  double *U, *kurt_u, *ups_u;
  int32_t *rep_thread, *csize, *row_cluster;
  // workspace (carved by the launcher)
  double *key;
  int *cluster, *part_idx, *reps, *sizes, *ctl;
  float *Wt;
  unsigned int *done;
  CoopSlot *slots;
};
struct ClusterWs {     // workspace of one clustering problem
  double *key;
  int *cluster, *reps, *sizes, *part_idx;
  float *Wt;           // N x K transposed rows
  unsigned int *done;  // [0] arrivals / work-groups finished, [1] wait-bound flag
  CoopSlot *slots;     // 2 x work-groups
};
size_t cluster_ws_bytes(int K, int N);
ClusterWs carve_cluster_ws(void *ws, int K, int N);
size_t unique_workspace_bytes(int K, int N);
// grouping candidates: CONV rows, equal keys (cluster -1), others -2; writes cw.Wt
hipError_t launch_prep_groups(hipStream_t st, int K, int N, const uint8_t *status, const float *W,
                              const ClusterWs &cw);
size_t unique_batched_workspace_bytes(int D, const UJob *jobs);
hipError_t launch_unique_batched(hipStream_t st, int D, UJob *jobs, void *ws, int *counts_host);
hipError_t launch_groups(hipStream_t st, int N, int K, const float *W, const uint8_t *status,
                         double tau, void *ws, int *ctl_dev, int *ctl_host, int **cluster_out,
                         int **reps_out);
hipError_t launch_unique(hipStream_t st, int N, int64_t T, int K, const float *W,
                         const double *kurt, const uint8_t *status, double tau, int gtest,
                         int n_top, int cap, double *U, double *kurt_u, double *ups_u,
                         int32_t *rep_thread, int32_t *cluster_size, void *ws, int *counts_host,
                         int *counts_dev, int32_t *row_cluster = nullptr);

}  // namespace oica
