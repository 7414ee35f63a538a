// Batched kurtosis fixed point on gfx950 (Sec. 3.1-3.2 of the paper: the L
// random starts stacked as the rows of B, Z = B X, B <- (Z o Z o Z) X^T / M - 3B,
// converged rows removed from the product).
//
// One fused kernel does both contractions of a pass without storing Z:
//   GEMM1  Z^T = X^T B^T   (contraction over the N features, FP32 MFMA)
//   cube   P = Z o Z o Z   (in registers, on the accumulator layout of GEMM1)
//   GEMM2  G^T += X P^T    (contraction over the samples, FP32 MFMA)
// Work is split over (row block, sample split) pairs; each pair writes a
// partial G that the epilogue kernel sums in a fixed order, so results are
// deterministic.  The epilogue normalises, measures the step, updates the
// per-row state and appends still-moving rows to the next active list.
// The per-item device code is in fused_items.h.
#include "fused_items.h"

#include <algorithm>

#include <math.h>

namespace oica {

int fused_np(int N) { return ((N + 31) / 32) * 32; }

static inline int wk_for_np(int np) { return np <= 64 ? 2 : 1; }

// Rows per wave of the per-row passes: one while that leaves enough waves to
// fill the chip, up to EPI_ROWS for large K (fewer list-append atomics).
static int rows_per_wave(int kmax) {
  int r = kmax / 8192;
  return r < 1 ? 1 : (r > EPI_ROWS ? EPI_ROWS : r);
}

// The BF16 plan with one 32-row block per wave: for passes with at most
// bf16_waves(np) * 32 active rows (one row block either way, so the same sample splits
// and the same arithmetic per row, with half the padded rows).
FusedPlan narrow_plan(const FusedPlan &p, int np) {
  FusedPlan q = p;
  q.kwg = bf16_waves(np) * 32;
  return q;
}

// FP32 passes with at most THIN_PLAN_ROWS active rows: thin items (rows padded
// to 32, each wave on its own split, WAVES times the splits).
FusedPlan thin_plan(const FusedPlan &p) {
  FusedPlan q = p;
  q.kwg = 32;
  q.thin = 1;
  return q;
}

// Work-groups of a pass launch: as many as are resident at once for the FP32
// kernels and the BF16 variants at padded N <= 64 (four waves, two work-groups
// per CU), twice those for the BF16 variants at N >= 96 (eight waves, one per
// CU).  Against 1024: half the split partials written and no second dispatch
// round (EEG-shaped workload in BF16 7 % faster per step, in FP32 1 %;
// precision workload unchanged).
constexpr int GRID_PASS = 512;

FusedPlan make_plan(int N, int64_t T, int kmax, bool bf16) {
  (void)kmax;
  FusedPlan p;
  int np = fused_np(N);
  p.grid = GRID_PASS;
  p.kwg = (bf16 ? bf16_waves(np) : WAVES) * wk_for_np(np) * 32;
  int64_t n_sub = (T + 31) / 32;
  p.n_sub = (int)n_sub;
  int64_t ms = n_sub / MIN_SUB;
  if (ms < 1) ms = 1;
  if (ms > GRID_PASS) ms = GRID_PASS;
  p.max_splits = (int)ms;
  p.ld = T;
  return p;
}

constexpr int PAD_U = 8;  // elements per thread and trip, 256 apart

template <typename E>
__global__ __launch_bounds__(256) void k_pad_rows(const E *__restrict__ src, long long T,
                                                  E *__restrict__ dst, long long ld) {
  // row blockIdx.y; the work-groups of a row stride over its samples (no
  // division per element); each thread has all PAD_U loads of a trip in
  // flight before its stores (one load at a time left the copy latency-bound)
  const E *s = src + (size_t)blockIdx.y * (size_t)T;
  E *d = dst + (size_t)blockIdx.y * (size_t)ld;
  constexpr long long TILE = 256LL * PAD_U;
  for (long long b = (long long)blockIdx.x * TILE; b < T; b += (long long)gridDim.x * TILE) {
    const long long m0 = b + threadIdx.x;
    E v[PAD_U];
    if (b + TILE <= T) {  // work-group uniform: the whole tile inside the row
#pragma unroll
      for (int u = 0; u < PAD_U; ++u) v[u] = s[m0 + 256 * u];
#pragma unroll
      for (int u = 0; u < PAD_U; ++u) d[m0 + 256 * u] = v[u];
    } else {
#pragma unroll
      for (int u = 0; u < PAD_U; ++u) v[u] = s[m0 + 256 * u < T ? m0 + 256 * u : T - 1];
#pragma unroll
      for (int u = 0; u < PAD_U; ++u)
        if (m0 + 256 * u < T) d[m0 + 256 * u] = v[u];
    }
  }
}

hipError_t launch_pad_rows(hipStream_t st, const void *src, int esize, int N, long long T,
                           void *dst, long long ld) {
  if (N <= 0 || T <= 0) return hipSuccess;
  const int per_row = (int)std::min<long long>((T + 256 * PAD_U - 1) / (256 * PAD_U),
                                               std::max(1, 16384 / N));
  const dim3 grid(per_row, N);
  if (esize == 2)
    hipLaunchKernelGGL(k_pad_rows<uint16_t>, grid, dim3(256), 0, st, (const uint16_t *)src, T,
                       (uint16_t *)dst, ld);
  else
    hipLaunchKernelGGL(k_pad_rows<float>, grid, dim3(256), 0, st, (const float *)src, T,
                       (float *)dst, ld);
  return hipGetLastError();
}

// Partial-buffer rows per split: positions are padded to whole row blocks.
static inline __host__ __device__ int padded_rows(int kact, int kwg) {
  return ((kact + kwg - 1) / kwg) * kwg;
}

size_t fp_workspace_floats(const FusedPlan &p, int N, int kmax) {
  int np = fused_np(N);
  size_t worst = 0;
  // the partial buffer holds n_splits(n_kb) * n_kb * kwg rows; take the max
  // over every n_kb a run can reach, with the plan and with its thin form
  // (used while at most THIN_PLAN_ROWS rows are active)
  int kb_max = (kmax + p.kwg - 1) / p.kwg;
  for (int nkb = 1; nkb <= kb_max; ++nkb) {
    size_t rows = (size_t)plan_splits(p, nkb) * (size_t)nkb * (size_t)p.kwg;
    if (rows > worst) worst = rows;
  }
  const FusedPlan t = thin_plan(p);
  const int thin_rows = kmax < THIN_PLAN_ROWS ? kmax : THIN_PLAN_ROWS;
  for (int nkb = 1; nkb <= (thin_rows + 31) / 32; ++nkb) {
    size_t rows = (size_t)plan_splits(t, nkb) * (size_t)nkb * 32;
    if (rows > worst) worst = rows;
  }
  return worst * (size_t)np;
}

template <int NP, int WK, bool KURT>
__global__ __launch_bounds__(WAVES * 64, 2) void k_fused_f32(
    const float *__restrict__ X, int N, long long T, FusedPlan plan,
    const float *__restrict__ Bm, const int *__restrict__ act, const int *__restrict__ kact_dev,
    int kact_host, float *__restrict__ gpart, float *__restrict__ s4part,
    double *__restrict__ s4part64, FpControl *ctl, int pass) {
  constexpr int KWG = WAVES * WK * 32;
  __shared__ float xs[NP * TileF32<NP>::sx];

  const int kact = kact_dev ? kact_dev[pass & 1] : kact_host;
  if (ctl && blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->kact[(pass + 1) & 1] = 0;
    if (kact > 0) {
      ctl->passes = pass + 1;
      ctl->thread_iters += kact;
    }
  }
  if (kact <= 0) return;

  const int n_kb = (kact + KWG - 1) / KWG;
  const int n_sp = plan_splits(plan, n_kb);
  const int rows_pad = n_kb * KWG;
  const int work = n_kb * n_sp;
  const int per_xcd_items = (work + 7) / 8;
  const int per_xcd_wgs = plan.grid / 8;
  const int xcd = blockIdx.x % 8;
  const int local = blockIdx.x / 8;
  const ItemCtx c{X, N, T, plan.ld, plan.n_sub, n_sp, rows_pad, Bm, act, kact, gpart, s4part,
                  s4part64};
  for (int it = local; it < per_xcd_items; it += per_xcd_wgs) {
    const int w_item = xcd * per_xcd_items + it;
    if (w_item >= work) break;
    item_f32<NP, WK, KURT>(c, w_item % n_kb, w_item / n_kb, xs);
  }
}

// FP32 pass with the thin plan: work item (32-row block kb, split group g),
// wave w of the work-group on split WAVES * g + w with its own LDS tile.
template <int NP>
__global__ __launch_bounds__(WAVES * 64, 2) void k_fused_f32_thin(
    const float *__restrict__ X, int N, long long T, FusedPlan plan,
    const float *__restrict__ Bm, const int *__restrict__ act, const int *__restrict__ kact_dev,
    int kact_host, float *__restrict__ gpart, float *__restrict__ s4part, FpControl *ctl,
    int pass) {
  __shared__ float xs[WAVES * NP * ThinF32::sx];
  const int kact = kact_dev ? kact_dev[pass & 1] : kact_host;
  if (ctl && blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->kact[(pass + 1) & 1] = 0;
    if (kact > 0) {
      ctl->passes = pass + 1;
      ctl->thread_iters += kact;
    }
  }
  if (kact <= 0) return;
  const int n_kb = (kact + 31) / 32;
  const int n_sp = plan_splits(plan, n_kb);
  const int groups = (n_sp + WAVES - 1) / WAVES;
  const int work = n_kb * groups;
  const int per_xcd_items = (work + 7) / 8;
  const int per_xcd_wgs = plan.grid / 8;
  const int xcd = blockIdx.x % 8;
  const int local = blockIdx.x / 8;
  const int wave = threadIdx.x / 64;
  const ItemCtx c{X, N, T, plan.ld, plan.n_sub, n_sp, n_kb * 32, Bm, act, kact, gpart, s4part,
                  nullptr};
  for (int it = local; it < per_xcd_items; it += per_xcd_wgs) {
    const int w_item = xcd * per_xcd_items + it;
    if (w_item >= work) break;
    const int sp = (w_item / n_kb) * WAVES + wave;
    if (sp < n_sp) item_f32_wave<NP>(c, w_item % n_kb, sp, xs + wave * NP * ThinF32::sx);
  }
}

// FORM (BfRowForm): BF_HILO every row as hi + lo parts; BF_ONE every row
// rounded once to BF16; BF_SWITCH the first kc rows of the active list
// rounded once (every row at a run's first pass) and the rest as hi + lo, per
// work item (an item with any hi + lo row takes that form for all its rows).
template <int NP, int WK, int FORM>
__global__ __launch_bounds__(bf16_waves(NP) * 64, 2) void k_fused_bf16(
    const __bf16 *__restrict__ X, int N, long long T, FusedPlan plan, const float *__restrict__ Bm,
    const int *__restrict__ act, const int *__restrict__ kact_dev, int kact_host,
    float *__restrict__ gpart, float *__restrict__ s4part, FpControl *ctl, int pass) {
  constexpr int NW = bf16_waves(NP);
  constexpr int KWG = NW * WK * 32;
  constexpr int XTS = BfStride<NP>::v;
  __shared__ __attribute__((aligned(16))) __bf16 xs[2 * BfTile<NP>::xs_elems];
  __shared__ __attribute__((aligned(16))) __bf16 xt[2 * BfTile<NP>::xt_elems];

  const int kact = kact_dev ? kact_dev[pass & 1] : kact_host;
  // rows of the one-term form: the head of the list (read before block 0
  // resets the next pass's counters; kc of this pass is not written here)
  const int kc = (FORM == BF_SWITCH || FORM == BF_LATE) ? (pass == 0 ? kact : ctl->kc[pass & 1])
                                                        : (FORM == BF_ONE ? kact : 0);
  if (ctl && blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->kact[(pass + 1) & 1] = 0;
    if (FORM == BF_SWITCH || FORM == BF_LATE) ctl->kf = 0;
    if (kact > 0) {
      ctl->passes = pass + 1;
      ctl->thread_iters += kact;
    }
  }
  if (kact <= 0) return;

  const int n_kb = (kact + KWG - 1) / KWG;
  const int n_sp = plan_splits(plan, n_kb);
  const int rows_pad = n_kb * KWG;
  const int work = n_kb * n_sp;
  const int per_xcd_items = (work + 7) / 8;
  const int per_xcd_wgs = plan.grid / 8;
  const int xcd = blockIdx.x % 8;
  const int local = blockIdx.x / 8;
  const ItemCtx c{X, N, T, plan.ld, plan.n_sub, n_sp, rows_pad, Bm, act, kact, gpart, s4part,
                  nullptr};
  for (int it = local; it < per_xcd_items; it += per_xcd_wgs) {
    const int w_item = xcd * per_xcd_items + it;
    if (w_item >= work) break;
    const int kb = w_item % n_kb, sp = w_item / n_kb;
    // every row of the item takes the one-term form (BF_LATE: the list's tail)
    const bool one = FORM == BF_LATE ? kb * KWG >= kc
                                     : ((kb + 1) * KWG < kact ? (kb + 1) * KWG : kact) <= kc;
    if (FORM != BF_HILO && one) {
      if (s4part)
        item_bf16<NP, WK, true, NW, false>(c, kb, sp, xs, xt);
      else
        item_bf16<NP, WK, false, NW, false>(c, kb, sp, xs, xt);
    } else if (FORM != BF_ONE) {
      if (s4part)
        item_bf16<NP, WK, true, NW, true>(c, kb, sp, xs, xt);
      else
        item_bf16<NP, WK, false, NW, true>(c, kb, sp, xs, xt);
    }
  }
}

// ---------------------------------------------------------------------------
// First stage of the split reduction: sums of SPLIT_GROUP consecutive splits,
// in split order, for every (group, active position, feature) and for the
// z^4 partial (stored as feature NP).  Grid-stride over all items so the
// long-split tail passes (few rows, many splits) are as parallel as the
// full-width passes.
// ---------------------------------------------------------------------------

template <int NP>
__global__ __launch_bounds__(256) void k_split_reduce(FusedPlan plan, const FpControl *ctl, int pass,
                                                      const float *__restrict__ gpart,
                                                      const float *__restrict__ s4part,
                                                      double *__restrict__ red) {
  constexpr int RS = NP + 1;
  const int kact = ctl->kact[pass & 1];
  if (kact <= 0) return;
  const int n_kb = (kact + plan.kwg - 1) / plan.kwg;
  const int n_sp = plan_splits(plan, n_kb);
  const int rows_pad = n_kb * plan.kwg;
  const int groups = (n_sp + SPLIT_GROUP - 1) / SPLIT_GROUP;
  const long long per_group = (long long)kact * RS;
  const long long items = (long long)groups * per_group;
  for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < items;
       idx += (long long)gridDim.x * 256) {
    const int g = (int)(idx / per_group);
    const int rem = (int)(idx - (long long)g * per_group);
    const int posn = rem / RS;
    const int n = rem - posn * RS;
    const int sp0 = g * SPLIT_GROUP;
    float v[SPLIT_GROUP];
#pragma unroll
    for (int u = 0; u < SPLIT_GROUP; ++u) {
      const int sp = sp0 + u;
      v[u] = 0.f;
      if (sp < n_sp)
        v[u] = n < NP ? gpart[((size_t)sp * rows_pad + posn) * NP + n]
                      : (s4part ? s4part[(size_t)sp * rows_pad + posn] : 0.f);
    }
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < SPLIT_GROUP; ++u) acc += (double)v[u];
    red[(size_t)idx] = acc;
  }
}

size_t fp_reduce_doubles(const FusedPlan &p, int N, int kmax) {
  const size_t rows_max = fp_workspace_floats(p, N, kmax) / (size_t)fused_np(N);
  return (rows_max / SPLIT_GROUP + (size_t)kmax + 1) * (size_t)(fused_np(N) + 1);
}

// ---------------------------------------------------------------------------
// Epilogue: one wave per active position.
// ---------------------------------------------------------------------------
// Algorithm 1's projection w <- w - E w with E = P^T P for the n_proj unit
// rows of P (n_proj x N, FP64): the coefficients c_k = P_k . w of the whole
// vector first, then one subtraction.  A wave holds w in (lane, lane + 64).
__device__ inline void project_out(double &w0, double &w1, const double *__restrict__ P,
                                   int n_proj, int N, int lane) {
  if (n_proj <= 0) return;
  const int n0 = lane, n1 = lane + 64;
  double s0 = 0.0, s1 = 0.0;
  for (int k = 0; k < n_proj; ++k) {
    const double p0 = n0 < N ? P[(size_t)k * N + n0] : 0.0;
    const double p1 = n1 < N ? P[(size_t)k * N + n1] : 0.0;
    const double c = wave_sum(p0 * w0 + p1 * w1);
    s0 = fma(c, p0, s0);
    s1 = fma(c, p1, s1);
  }
  w0 -= s0;
  w1 -= s1;
}

template <int NP>
__global__ __launch_bounds__(256) void k_epilogue(
    FusedPlan plan, int N, long long T, float *__restrict__ Bm, const int *__restrict__ act_cur,
    int *__restrict__ act_next, FpControl *ctl, int pass, const double *__restrict__ red,
    double tol, int32_t *__restrict__ iters, uint8_t *__restrict__ status,
    float *__restrict__ traj, int traj_iters, int rows_per_wave, const double *__restrict__ proj,
    int n_proj, int bf_form, double switch_step, int *__restrict__ fine_list) {
  constexpr int RS = NP + 1;
  const int kact = ctl->kact[pass & 1];
  // rows of the one-term BF16 form (head of the list), as the fused kernel saw them
  const bool split = bf_form == BF_SWITCH || bf_form == BF_LATE;
  const int kc = split ? (pass == 0 ? kact : ctl->kc[pass & 1]) : (bf_form == BF_ONE ? kact : 0);
  const int lane = threadIdx.x % 64;
  // rows_per_wave (<= EPI_ROWS) rows per wave, one after the other; the rows
  // that stay active are appended with one atomic per wave
  const int posn0 = (blockIdx.x * 4 + threadIdx.x / 64) * rows_per_wave;
  if (posn0 >= kact) return;  // uniform over the wave
  const int n_kb = (kact + plan.kwg - 1) / plan.kwg;
  const int n_sp = plan_splits(plan, n_kb);
  const int groups = (n_sp + SPLIT_GROUP - 1) / SPLIT_GROUP;
  const int n0 = lane, n1 = lane + 64;
  const double invT = 1.0 / (double)T;
  bool stay = false, stay_one = false;
  int stay_row = -1;
  for (int r = 0; r < rows_per_wave && posn0 + r < kact; ++r) {
    const int posn = posn0 + r;
    const int row = act_cur[posn];
    const bool one = bf_form == BF_LATE ? posn >= kc : posn < kc;
    double g0 = 0.0, g1 = 0.0, s4 = 0.0;
    // second stage: group sums in group order, EPI_U loads in flight per lane
    constexpr int EPI_U = 8;
    for (int q0 = 0; q0 < groups; q0 += EPI_U) {
      double v0[EPI_U], v1[EPI_U], v4[EPI_U];
#pragma unroll
      for (int u = 0; u < EPI_U; ++u) {
        const int q = q0 + u;
        const bool ok = q < groups;
        const double *src = red + ((size_t)(ok ? q : 0) * kact + posn) * RS;
        v0[u] = (ok && n0 < NP) ? src[n0] : 0.0;
        v1[u] = (ok && n1 < NP) ? src[n1] : 0.0;
        v4[u] = (ok && lane == 0) ? src[NP] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < EPI_U; ++u) {
        g0 += v0[u];
        g1 += v1[u];
        s4 += v4[u];
      }
    }
    float *brow = Bm + (size_t)row * N;
    const double bp0 = n0 < N ? (double)brow[n0] : 0.0;
    const double bp1 = n1 < N ? (double)brow[n1] : 0.0;
    // the linear term: the row the pass's z came from (rounded to BF16 when
    // the pass ran on one BF16 part, so the pass is that row's exact update)
    const double bl0 = (one && n0 < N) ? (double)(float)(__bf16)brow[n0] : bp0;
    const double bl1 = (one && n1 < N) ? (double)(float)(__bf16)brow[n1] : bp1;
    g0 = n0 < N ? g0 * invT - 3.0 * bl0 : 0.0;
    g1 = n1 < N ? g1 * invT - 3.0 * bl1 : 0.0;
    project_out(g0, g1, proj, n_proj, N, lane);  // Algorithm 1 only (n_proj > 0)
    const double gn = sqrt(wave_sum(g0 * g0 + g1 * g1));
    s4 = __shfl(s4, 0);
    const double alpha = s4 * invT - 3.0;
    double d;
    if (!(gn > 0.0) || !isfinite(gn)) {
      d = NAN;
      if (lane == 0) status[row] = OICA_ROW_DEGENERATE;
    } else {
      const double b0 = g0 / gn, b1 = g1 / gn;
      const double dm = wave_sum((b0 - bp0) * (b0 - bp0) + (b1 - bp1) * (b1 - bp1));
      const double dp = wave_sum((b0 + bp0) * (b0 + bp0) + (b1 + bp1) * (b1 + bp1));
      d = sqrt(dm < dp ? dm : dp);
      if (n0 < N) brow[n0] = (float)b0;
      if (n1 < N) brow[n1] = (float)b1;
      // in the switched form a one-term row never converges: it takes the
      // hi + lo form once its step is below switch_step
      const bool coarse = bf_form == BF_SWITCH && one;
      if (lane == 0) {
        iters[row] += 1;
        if (!coarse && d < tol) status[row] = OICA_ROW_CONV;
      }
      if (lane == r && (coarse || !(d < tol))) {
        stay = true;
        stay_row = row;
        // BF_SWITCH: stays one-term while the step is large; BF_LATE: takes
        // the one-term form once the step is small (and keeps it)
        stay_one = bf_form == BF_LATE ? (one || d < switch_step) : (coarse && !(d < switch_step));
      }
    }
    if (lane == 0 && pass < traj_iters) {
      traj[((size_t)row * traj_iters + pass) * 2 + 0] = (float)alpha;
      traj[((size_t)row * traj_iters + pass) * 2 + 1] = (float)d;
    }
  }
  if (bf_form == BF_SWITCH) {
    wave_append(stay && stay_one, stay_row, act_next, &ctl->kact[(pass + 1) & 1]);
    wave_append(stay && !stay_one, stay_row, fine_list, &ctl->kf);
  } else if (bf_form == BF_LATE) {
    wave_append(stay && !stay_one, stay_row, act_next, &ctl->kact[(pass + 1) & 1]);
    wave_append(stay && stay_one, stay_row, fine_list, &ctl->kf);
  } else {
    wave_append(stay, stay_row, act_next, &ctl->kact[(pass + 1) & 1]);
  }
}

// Switched BF16 form: the rows staged for the hi + lo form join the next
// pass's list after its one-term rows; the one-term count is recorded.  One
// work-group.
__global__ __launch_bounds__(1024) void k_join_fine(int *__restrict__ act_next,
                                                    const int *__restrict__ fine_list,
                                                    FpControl *ctl, int pass) {
  const int nx = (pass + 1) & 1;
  const int kc = ctl->kact[nx];
  const int kf = ctl->kf;
  for (int j = threadIdx.x; j < kf; j += blockDim.x) act_next[kc + j] = fine_list[j];
  __syncthreads();  // every thread has read the counts
  if (threadIdx.x == 0) {
    ctl->kc[nx] = kc;
    ctl->kact[nx] = kc + kf;
  }
}

// Row initialisation: normalise W0 in FP64, mark zero/non-finite rows
// DEGENERATE, build the first active list.
__global__ void k_init_rows(int K, int N, const float *__restrict__ W0, float *__restrict__ Bm,
                            int32_t *__restrict__ iters, uint8_t *__restrict__ status,
                            int *__restrict__ act0, FpControl *ctl, float *__restrict__ traj,
                            int traj_iters, int rpw, const double *__restrict__ proj,
                            int n_proj) {
  const int lane = threadIdx.x % 64;
  const int row0 = (blockIdx.x * 4 + threadIdx.x / 64) * rpw;  // rpw rows per wave
  if (row0 >= K) return;  // uniform over the wave
  bool take = false;
  int take_row = -1;
  for (int r = 0; r < rpw && row0 + r < K; ++r) {
    const int row = row0 + r;
    const float *src = W0 + (size_t)row * N;
    const int n0 = lane, n1 = lane + 64;
    double w0 = n0 < N ? (double)src[n0] : 0.0;
    double w1 = n1 < N ? (double)src[n1] : 0.0;
    project_out(w0, w1, proj, n_proj, N, lane);  // Algorithm 1 only (n_proj > 0)
    const double nrm = sqrt(wave_sum(w0 * w0 + w1 * w1));
    const bool ok = nrm > 0.0 && isfinite(nrm);
    float *dst = Bm + (size_t)row * N;
    if (n0 < N) dst[n0] = (float)(w0 / nrm);
    if (n1 < N) dst[n1] = (float)(w1 / nrm);
    for (int t = lane; t < 2 * traj_iters; t += 64) traj[(size_t)row * traj_iters * 2 + t] = NAN;
    if (lane == 0) {
      iters[row] = 0;
      status[row] = ok ? OICA_ROW_NOTCONV : OICA_ROW_DEGENERATE;
    }
    if (lane == r) {
      take = ok;
      take_row = row;
    }
  }
  wave_append(take, take_row, act0, &ctl->kact[0]);
}

// Active set of the FP32 phase after a BF16 loop, built in `dst`: the rows that
// converged on BF16 data (status reset to NOTCONV until they pass the FP32
// test) and the `left` rows still active when the BF16 loop ended.
__global__ void k_refine_select(int K, uint8_t *__restrict__ status, int *__restrict__ dst,
                                FpControl *ctl, const int *__restrict__ left_list, int left) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool conv = i < K && status[i] == OICA_ROW_CONV;
  if (conv) status[i] = OICA_ROW_NOTCONV;
  wave_append(conv, i, dst, &ctl->kact[0]);
  wave_append(i < left, i < left ? left_list[i] : -1, dst, &ctl->kact[0]);
}

// Rows pruned earlier go back into the active set (status NOTCONV), their
// rows and iteration counts as they were left.
__global__ void k_unprune(int K, uint8_t *__restrict__ status, int *__restrict__ list,
                          FpControl *ctl) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  const bool back = row < K && status[row] == OICA_ROW_PRUNED;
  if (back) status[row] = OICA_ROW_NOTCONV;
  wave_append(back, row, list, &ctl->kact[0]);
}

hipError_t launch_unprune(hipStream_t st, int K, uint8_t *status, int *list, FpControl *ctl) {
  hipLaunchKernelGGL(k_unprune, dim3((K + 255) / 256), dim3(256), 0, st, K, status, list, ctl);
  return hipGetLastError();
}

// G = sum_sp gpart / T - 3 B and s4 = sum_sp s4part / T for rows 0..K-1
// (positions equal rows).
template <int NP>
__global__ void k_update_out(FusedPlan plan, int N, long long T, int K, const float *__restrict__ Bm,
                             const float *__restrict__ gpart, const float *__restrict__ s4part,
                             double *__restrict__ G, double *__restrict__ s4out) {
  const int lane = threadIdx.x % 64;
  const int row = blockIdx.x * 4 + threadIdx.x / 64;
  if (row >= K) return;
  const int n_kb = (K + plan.kwg - 1) / plan.kwg;
  const int n_sp = plan_splits(plan, n_kb);
  const int rows_pad = n_kb * plan.kwg;
  const double invT = 1.0 / (double)T;
  for (int n = lane; n < N; n += 64) {
    double g = 0.0;
    for (int sp = 0; sp < n_sp; ++sp) g += (double)gpart[((size_t)sp * rows_pad + row) * NP + n];
    G[(size_t)row * N + n] = g * invT - 3.0 * (double)Bm[(size_t)row * N + n];
  }
  if (lane == 0) {
    double s = 0.0;
    for (int sp = 0; sp < n_sp; ++sp) s += (double)s4part[(size_t)sp * rows_pad + row];
    s4out[row] = s * invT;
  }
}

// One wave per row: lanes take splits lane, lane + 64, ..., then a fixed
// shuffle tree (the splits' partial sums are independent loads in flight).
template <int NP>
__global__ void k_kurt_out(FusedPlan plan, long long T, int K, const double *__restrict__ s4part64,
                           double *__restrict__ kurt, const int *__restrict__ act,
                           const int *__restrict__ kact_dev) {
  const int posn = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  const int kact = kact_dev ? kact_dev[0] : K;
  if (posn >= kact) return;  // uniform over the wave
  const int row = act ? act[posn] : posn;
  const int kwg = plan.kwg;
  const int n_kb = (kact + kwg - 1) / kwg;
  const int n_sp = plan_splits(plan, n_kb);
  const int rows_pad = n_kb * kwg;
  double s = 0.0;
  for (int sp = lane; sp < n_sp; sp += 64) s += s4part64[(size_t)sp * rows_pad + posn];
  s = wave_sum(s);
  if (lane == 0) kurt[row] = s / (double)T - 3.0;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
#define OICA_NP_SWITCH(np, ...)                     \
  switch (np) {                                     \
    case 32: { constexpr int NP_ = 32; __VA_ARGS__; break; }   \
    case 64: { constexpr int NP_ = 64; __VA_ARGS__; break; }   \
    case 96: { constexpr int NP_ = 96; __VA_ARGS__; break; }   \
    case 128: { constexpr int NP_ = 128; __VA_ARGS__; break; } \
    default: return hipErrorInvalidValue;           \
  }

hipError_t launch_init_rows(hipStream_t st, int K, int N, const float *W0, float *B,
                            int32_t *iters, uint8_t *status, int *act0, FpControl *ctl,
                            float *traj, int traj_iters, const double *proj, int n_proj) {
  const int rpw = rows_per_wave(K);
  hipLaunchKernelGGL(k_init_rows, dim3((K + 4 * rpw - 1) / (4 * rpw)), dim3(256), 0, st, K, N, W0,
                     B, iters, status, act0, ctl, traj, traj_iters, rpw, proj, n_proj);
  return hipGetLastError();
}

hipError_t launch_fused_update(hipStream_t st, const FusedPlan &p, int N, int64_t T, const void *X,
                               bool bf16, const float *B, const int *act, const int *kact_dev,
                               int kact_host, float *gpart, float *s4part, FpControl *ctl,
                               int pass, int bf_form) {
  const int np = fused_np(N);
  if (bf16) {
    // the switched form needs the device counters (and a list to split)
    if ((bf_form == BF_SWITCH || bf_form == BF_LATE) && (!ctl || !kact_dev)) bf_form = BF_HILO;
    const bool wk1 = p.kwg == bf16_waves(np) * 32;  // one 32-row block per wave (narrow plan)
#define OICA_BF16_LAUNCH(WKV, FV)                                                          \
  hipLaunchKernelGGL((k_fused_bf16<NP_, WKV, FV>), dim3(p.grid), dim3(bf16_waves(NP_) * 64), 0,  \
                     st, (const __bf16 *)X, N, (long long)T, p, B, act, kact_dev, kact_host,    \
                     gpart, s4part, ctl, pass)
#define OICA_BF16_FORMS(WKV)                 \
  do {                                       \
    if (bf_form == BF_ONE)                   \
      OICA_BF16_LAUNCH(WKV, BF_ONE);         \
    else if (bf_form == BF_SWITCH)           \
      OICA_BF16_LAUNCH(WKV, BF_SWITCH);      \
    else if (bf_form == BF_LATE)             \
      OICA_BF16_LAUNCH(WKV, BF_LATE);        \
    else                                     \
      OICA_BF16_LAUNCH(WKV, BF_HILO);        \
  } while (0)
    OICA_NP_SWITCH(np, {
      constexpr int WK2 = NP_ <= 64 ? 2 : 1;  // the wide variant
      if (!wk1)
        OICA_BF16_FORMS(WK2);
      else
        OICA_BF16_FORMS(1);
    });
#undef OICA_BF16_FORMS
#undef OICA_BF16_LAUNCH
    return hipGetLastError();
  }
  const bool wk1 = p.kwg == WAVES * 32;  // one 32-row block per wave (narrow plan)
  if (p.thin) {
    OICA_NP_SWITCH(np, {
      hipLaunchKernelGGL((k_fused_f32_thin<NP_>), dim3(p.grid), dim3(WAVES * 64), 0, st,
                         (const float *)X, N, (long long)T, p, B, act, kact_dev, kact_host, gpart,
                         s4part, ctl, pass);
    });
    return hipGetLastError();
  }
  OICA_NP_SWITCH(np, {
    constexpr int WK2 = NP_ <= 64 ? 2 : 1;  // the wide variant
    if (!wk1)
      hipLaunchKernelGGL((k_fused_f32<NP_, WK2, false>), dim3(p.grid), dim3(WAVES * 64), 0, st,
                         (const float *)X, N, (long long)T, p, B, act, kact_dev, kact_host, gpart,
                         s4part, (double *)nullptr, ctl, pass);
    else
      hipLaunchKernelGGL((k_fused_f32<NP_, 1, false>), dim3(p.grid), dim3(WAVES * 64), 0, st,
                         (const float *)X, N, (long long)T, p, B, act, kact_dev, kact_host, gpart,
                         s4part, (double *)nullptr, ctl, pass);
  });
  return hipGetLastError();
}

hipError_t launch_epilogue(hipStream_t st, const FusedPlan &p, int N, int64_t T, int kmax, float *B,
                           const int *act_cur, int *act_next, FpControl *ctl, int pass,
                           const float *gpart, const float *s4part, double *red, double tol,
                           int32_t *iters, uint8_t *status, float *traj, int traj_iters,
                           const double *proj, int n_proj, int bf_form, double switch_step,
                           int *fine_list) {
  if ((bf_form == BF_SWITCH || bf_form == BF_LATE) && !fine_list) bf_form = BF_HILO;
  const int np = fused_np(N);
  OICA_NP_SWITCH(np, {
    hipLaunchKernelGGL((k_split_reduce<NP_>), dim3(RED_GRID), dim3(256), 0, st, p,
                       (const FpControl *)ctl, pass, gpart, s4part, red);
    const int rpw = rows_per_wave(kmax);
    hipLaunchKernelGGL((k_epilogue<NP_>), dim3((kmax + 4 * rpw - 1) / (4 * rpw)), dim3(256), 0,
                       st, p, N, (long long)T, B, act_cur, act_next, ctl, pass,
                       (const double *)red, tol, iters, status, traj, traj_iters, rpw, proj,
                       n_proj, bf_form, switch_step, fine_list);
  });
  if (bf_form == BF_SWITCH || bf_form == BF_LATE)
    hipLaunchKernelGGL(k_join_fine, dim3(1), dim3(1024), 0, st, act_next, (const int *)fine_list,
                       ctl, pass);
  return hipGetLastError();
}

hipError_t launch_refine_select(hipStream_t st, int K, uint8_t *status, int *dst, FpControl *ctl,
                                const int *left_list, int left) {
  hipLaunchKernelGGL(k_refine_select, dim3((K + 255) / 256), dim3(256), 0, st, K, status, dst, ctl,
                     left_list, left);
  return hipGetLastError();
}

hipError_t launch_update_out(hipStream_t st, const FusedPlan &p, int N, int64_t T, int K,
                             const float *B, const float *gpart, const float *s4part, double *G,
                             double *s4) {
  const int np = fused_np(N);
  OICA_NP_SWITCH(np, {
    hipLaunchKernelGGL((k_update_out<NP_>), dim3((K + 3) / 4), dim3(256), 0, st, p, N,
                       (long long)T, K, B, gpart, s4part, G, s4);
  });
  return hipGetLastError();
}

hipError_t launch_kurtosis(hipStream_t st, const FusedPlan &p, int N, int64_t T, const float *X,
                           int K, const float *W, double *s4part64, double *kurt, const int *act,
                           const int *kact_dev) {
  const int np = fused_np(N);
  OICA_NP_SWITCH(np, {
    constexpr int WK_ = NP_ <= 64 ? 2 : 1;
    hipLaunchKernelGGL((k_fused_f32<NP_, WK_, true>), dim3(p.grid), dim3(WAVES * 64), 0, st, X, N,
                       (long long)T, p, W, act, kact_dev, K, (float *)nullptr, (float *)nullptr,
                       s4part64, (FpControl *)nullptr, 0);
    hipLaunchKernelGGL((k_kurt_out<NP_>), dim3((K + 3) / 4), dim3(256), 0, st, p,
                       (long long)T, K, s4part64, kurt, act, kact_dev);
  });
  return hipGetLastError();
}

// Lists for the grouped FP32 finish: the representative of every group (status
// reset to NOTCONV until it passes the FP32 test) plus the `left` rows still
// active after the BF16 loop go to refine_list; every row that is not a
// non-representative group member goes to kurt_list.
__global__ void k_group_lists(int K, const int *__restrict__ cluster, const int *__restrict__ reps,
                              const int *__restrict__ n_groups_dev, uint8_t *__restrict__ status,
                              double *__restrict__ kurt_out,
                              int *__restrict__ refine_list, FpControl *ctl_refine,
                              const int *__restrict__ left_list, int left,
                              int *__restrict__ kurt_list, FpControl *ctl_kurt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool rep = i < *n_groups_dev;
  const int r = rep ? reps[i] : -1;
  if (rep) status[r] = OICA_ROW_NOTCONV;
  wave_append(rep, r, refine_list, &ctl_refine->kact[0]);
  wave_append(i < left, i < left ? left_list[i] : -1, refine_list, &ctl_refine->kact[0]);
  bool kurt = false;
  if (i < K) {
    const int c = cluster[i];
    const bool pruned = status[i] == OICA_ROW_PRUNED;  // left pruned: no kurtosis
    kurt = (c < 0 && !pruned) || (c >= 0 && reps[c] == i);
    if (pruned) kurt_out[i] = NAN;
  }
  wave_append(kurt, i, kurt_list, &ctl_kurt->kact[0]);
}

// Group members take their representative's refined row (with their own
// sign), status and kurtosis.  One wave per row.
__global__ void k_propagate(int K, int N, const int *__restrict__ cluster,
                            const int *__restrict__ reps, float *__restrict__ W,
                            uint8_t *__restrict__ status, double *__restrict__ kurt) {
  const int lane = threadIdx.x % 64;
  const int l = blockIdx.x * 4 + threadIdx.x / 64;
  if (l >= K) return;
  const int c = cluster[l];
  if (c < 0) return;
  const int r = reps[c];
  if (r == l) return;
  float *wl = W + (size_t)l * N;
  const float *wr = W + (size_t)r * N;
  double dot = 0.0;
  for (int n = lane; n < N; n += 64) dot += (double)wl[n] * (double)wr[n];
  dot = wave_sum(dot);
  const float sg = dot < 0.0 ? -1.f : 1.f;
  for (int n = lane; n < N; n += 64) wl[n] = sg * wr[n];
  if (lane == 0) {
    status[l] = status[r];
    kurt[l] = kurt[r];
  }
}

hipError_t launch_group_lists(hipStream_t st, int K, const int *cluster, const int *reps,
                              const int *n_groups_dev, uint8_t *status, double *kurt,
                              int *refine_list, FpControl *ctl_refine, const int *left_list,
                              int left, int *kurt_list, FpControl *ctl_kurt) {
  hipLaunchKernelGGL(k_group_lists, dim3((K + 255) / 256), dim3(256), 0, st, K, cluster, reps,
                     n_groups_dev, status, kurt, refine_list, ctl_refine, left_list, left,
                     kurt_list, ctl_kurt);
  return hipGetLastError();
}

hipError_t launch_propagate(hipStream_t st, int K, int N, const int *cluster, const int *reps,
                            float *W, uint8_t *status, double *kurt) {
  hipLaunchKernelGGL(k_propagate, dim3((K + 3) / 4), dim3(256), 0, st, K, N, cluster, reps, W,
                     status, kurt);
  return hipGetLastError();
}

}  // namespace oica
