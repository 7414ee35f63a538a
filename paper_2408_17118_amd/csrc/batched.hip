// Many independent datasets in one persistent launch per pass.
//
// Every dataset keeps its own rows, active lists, control block and partial
// buffers (BatchDesc).  A pass is four launches for the whole batch:
//   k_batch_plan      one work-group: reads every dataset's active count,
//                     does the per-dataset bookkeeping and builds prefix sums
//                     of the work items of the three batched kernels;
//   k_fused_batched   persistent work-groups pull (dataset, row block, sample
//                     split) items from an atomic queue and run the same
//                     per-item device code as the single-dataset kernels,
//                     dispatching on the dataset's padded N, rows per wave and
//                     data type;
//   k_split_reduce_batched, k_epilogue_batched   the split reduction and the
//                     per-row update of every dataset, grid-stride over the
//                     concatenated items.
// A dataset's sample partition depends on its own T only (splits of about
// BATCH_SPLIT samples), and rows per wave only regroup independent rows, so a
// dataset's arithmetic is the same alone or in any batch and under any tile
// choice the tuner makes.
#include "fused_items.h"

#include <math.h>

namespace oica {

constexpr int BATCH_SPLIT = 4096;   // samples per split in the batched form
constexpr int MAX_D = 1024;         // datasets per call
// FP32: one shared tile, or four one-wave tiles (NP = 128) for thin problems
constexpr int BUF_BYTES_F32 = WAVES * 128 * ThinF32::sx * 4;
constexpr int BUF_BYTES_BF16 = 2 * (128 * BSX + BT * (128 + 8)) * 2;  // two BF16 buffers at NP = 128

// Work items per row block: one per split, or one per THIN_SPLITS splits for
// thin problems (one split per wave).
__host__ __device__ inline int split_items(const BatchDesc &b) {
  return b.variant >= THIN_VARIANT ? (b.n_sp + THIN_SPLITS - 1) / THIN_SPLITS : b.n_sp;
}

int batch_splits(int64_t T) {
  int64_t s = (T + BATCH_SPLIT / 2) / BATCH_SPLIT;
  if (s < 1) s = 1;
  return (int)s;
}

__global__ __launch_bounds__(1024) void k_batch_plan(const BatchDesc *__restrict__ descs, int D,
                                                     BatchCtl *bctl, int *__restrict__ item_start,
                                                     long long *__restrict__ red_start,
                                                     int *__restrict__ epi_start, int pass,
                                                     int dry) {
  __shared__ int s_items[MAX_D], s_epi[MAX_D];
  __shared__ long long s_red[MAX_D];
  for (int d = threadIdx.x; d < D; d += blockDim.x) {
    const BatchDesc &b = descs[d];
    FpControl *c = b.ctl;
    const int kact = c->kact[pass & 1];
    if (!dry) {
      c->kact[(pass + 1) & 1] = 0;
      if (kact > 0) {
        c->passes = pass + 1;
        c->thread_iters += kact;
      }
    }
    int items = 0, epi = 0;
    long long red = 0;
    if (kact > 0) {
      const int n_kb = (kact + b.kwg - 1) / b.kwg;
      items = n_kb * split_items(b);
      const int groups = (b.n_sp + SPLIT_GROUP - 1) / SPLIT_GROUP;
      red = (long long)groups * kact * (b.np + 1);
      epi = kact;
    }
    s_items[d] = items;
    s_red[d] = red;
    s_epi[d] = epi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int it = 0, ep = 0;
    long long rd = 0;
    for (int d = 0; d < D; ++d) {
      item_start[d] = it;
      red_start[d] = rd;
      epi_start[d] = ep;
      it += s_items[d];
      rd += s_red[d];
      ep += s_epi[d];
    }
    item_start[D] = it;
    red_start[D] = rd;
    epi_start[D] = ep;
    bctl->total_items = it;
    bctl->total_red = rd;
    bctl->total_epi = ep;
    bctl->counter[pass & 1] = 0;
  }
}

// largest d with start[d] <= x (start non-decreasing, start[0] = 0 <= x)
template <typename I>
__device__ inline int find_dataset(const I *start, int D, I x) {
  int lo = 0, hi = D;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Persistent pass kernel of one data type (every dataset of a call uses the
// same one): work-groups pull (dataset, row block, sample split) items from the
// pass's atomic queue until it is empty.
// Each variant is its own (not inlined) function, so each gets the register
// budget of its single-dataset kernel instead of the union of all variants.
// FP32 items run without the next-tile register prefetch, which spills under
// the call convention's reserved registers at NP = 64, WK = 2.
template <int NP, int WK>
__device__ __noinline__ void call_f32(const ItemCtx &c, int kb, int sp, float *xs) {
  item_f32<NP, WK, false, false>(c, kb, sp, xs);
}
template <int NP, int WK, bool LO>
__device__ __noinline__ void call_bf16(const ItemCtx &c, int kb, int sp, __bf16 *xs, __bf16 *xt) {
  item_bf16<NP, WK, false, WAVES, LO>(c, kb, sp, xs, xt);   // no trajectories in the batched form
}

template <int NP>
__device__ __noinline__ void call_f32_thin(const ItemCtx &c, int kb, int sp, float *xs) {
  item_f32_wave<NP>(c, kb, sp, xs);
}

template <bool BF16>
__global__ __launch_bounds__(WAVES * 64, 2) void k_fused_batched(const BatchDesc *__restrict__ descs,
                                                                 int D, BatchCtl *bctl,
                                                                 const int *__restrict__ item_start,
                                                                 int pass) {
  __shared__ __attribute__((aligned(16))) char buf[BF16 ? BUF_BYTES_BF16 : BUF_BYTES_F32];
  __shared__ int s_start[MAX_D + 1];
  __shared__ int s_item;
  for (int d = threadIdx.x; d <= D; d += blockDim.x) s_start[d] = item_start[d];
  const int total = bctl->total_items;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(&bctl->counter[pass & 1], 1);
    __syncthreads();
    const int item = s_item;
    if (item >= total) break;
    const int d = find_dataset(s_start, D, item);
    const BatchDesc &b = descs[d];
    const int kact = b.ctl->kact[pass & 1];
    const int n_kb = (kact + b.kwg - 1) / b.kwg;
    const int local = item - s_start[d];
    const int kb = local % n_kb, sp = local / n_kb;
    const ItemCtx c{b.X, b.N, b.T, b.ld, b.n_sub, b.n_sp, n_kb * b.kwg, b.B,
                    (pass & 1) ? b.act1 : b.act0, kact, b.gpart, b.s4part, nullptr};
    if constexpr (!BF16) {
      float *xs32 = reinterpret_cast<float *>(buf);
      if (b.variant >= THIN_VARIANT) {
        // thin: each wave takes its own split of the item's THIN_SPLITS
        const int wave = threadIdx.x / 64;
        const int spw = sp * THIN_SPLITS + wave;
        float *xw = xs32 + wave * 128 * ThinF32::sx;
        if (spw < b.n_sp) switch (b.variant) {
            case THIN_VARIANT + 0: call_f32_thin<32>(c, kb, spw, xw); break;
            case THIN_VARIANT + 1: call_f32_thin<64>(c, kb, spw, xw); break;
            case THIN_VARIANT + 2: call_f32_thin<96>(c, kb, spw, xw); break;
            case THIN_VARIANT + 3: call_f32_thin<128>(c, kb, spw, xw); break;
            default: break;
          }
        continue;
      }
      switch (b.variant) {
        case 0: call_f32<32, 1>(c, kb, sp, xs32); break;
        case 1: call_f32<32, 2>(c, kb, sp, xs32); break;
        case 2: call_f32<64, 1>(c, kb, sp, xs32); break;
        case 3: call_f32<64, 2>(c, kb, sp, xs32); break;
        case 4: call_f32<96, 1>(c, kb, sp, xs32); break;
        case 6: call_f32<128, 1>(c, kb, sp, xs32); break;
        default: break;
      }
    } else {
      __bf16 *xs16 = reinterpret_cast<__bf16 *>(buf);
      __bf16 *xt16 = reinterpret_cast<__bf16 *>(buf + 2 * 128 * BSX * 2);
      if (b.bf_one) {
        switch (b.variant) {
          case 8: call_bf16<32, 1, false>(c, kb, sp, xs16, xt16); break;
          case 9: call_bf16<32, 2, false>(c, kb, sp, xs16, xt16); break;
          case 10: call_bf16<64, 1, false>(c, kb, sp, xs16, xt16); break;
          case 11: call_bf16<64, 2, false>(c, kb, sp, xs16, xt16); break;
          case 12: call_bf16<96, 1, false>(c, kb, sp, xs16, xt16); break;
          case 14: call_bf16<128, 1, false>(c, kb, sp, xs16, xt16); break;
          default: break;
        }
      } else {
        switch (b.variant) {
          case 8: call_bf16<32, 1, true>(c, kb, sp, xs16, xt16); break;
          case 9: call_bf16<32, 2, true>(c, kb, sp, xs16, xt16); break;
          case 10: call_bf16<64, 1, true>(c, kb, sp, xs16, xt16); break;
          case 11: call_bf16<64, 2, true>(c, kb, sp, xs16, xt16); break;
          case 12: call_bf16<96, 1, true>(c, kb, sp, xs16, xt16); break;
          case 14: call_bf16<128, 1, true>(c, kb, sp, xs16, xt16); break;
          default: break;
        }
      }
    }
  }
}

// A dataset's fields that the first-stage reduction reads, cached in LDS
// once per work-group (per element they were a dependent chain of global
// loads: the descriptor, then its control block's active count).
struct RedParams {
  const float *gpart, *s4part;
  double *red;
  int kact, rows_pad, np, n_sp;
};
static size_t red_lds_bytes(int D) {
  return (size_t)((D + 2) & ~1) * sizeof(long long) + (size_t)D * sizeof(RedParams);
}

__global__ __launch_bounds__(256) void k_split_reduce_batched(const BatchDesc *__restrict__ descs,
                                                              int D, const BatchCtl *bctl,
                                                              const long long *__restrict__ red_start,
                                                              int pass) {
  // dynamic LDS: (D + 1) starts, then D parameter sets (red_lds_bytes)
  extern __shared__ long long red_lds[];
  long long *s_start = red_lds;
  RedParams *s_p = (RedParams *)(red_lds + ((D + 2) & ~1));
  for (int d = threadIdx.x; d <= D; d += blockDim.x) s_start[d] = red_start[d];
  for (int d = threadIdx.x; d < D; d += blockDim.x) {
    const BatchDesc &b = descs[d];
    const int kact = b.ctl->kact[pass & 1];
    const int n_kb = (kact + b.kwg - 1) / b.kwg;
    s_p[d] = RedParams{b.gpart, b.s4part, b.red, kact, n_kb * b.kwg, b.np, b.n_sp};
  }
  __syncthreads();
  const long long total = bctl->total_red;
  for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * 256) {
    const int d = find_dataset(s_start, D, idx);
    const RedParams &q = s_p[d];
    const int kact = q.kact;
    const int rows_pad = q.rows_pad;
    const int RS = q.np + 1;
    const long long local = idx - s_start[d];
    const long long per_group = (long long)kact * RS;
    int g, rem;
    if (local <= 0x7fffffffLL && per_group <= 0x7fffffffLL) {
      // the usual case: 32-bit division (a 64-bit one is a long call)
      g = (int)local / (int)per_group;
      rem = (int)local - g * (int)per_group;
    } else {
      g = (int)(local / per_group);
      rem = (int)(local - (long long)g * per_group);
    }
    const int posn = rem / RS;
    const int n = rem - posn * RS;
    const int sp0 = g * SPLIT_GROUP;
    // every load of the group issued before the sums (a split past the last
    // reads the last and adds zero)
    // (one base and stride per element, read through a global pointer: a
    // generic load also counts against the LDS counter, so the LDS reads
    // between the loads would wait for each one)
    typedef __attribute__((address_space(1))) const float gcf;
    const bool is_g = n < q.np;
    gcf *src = is_g ? (gcf *)(q.gpart + (size_t)posn * q.np + n) : (gcf *)(q.s4part + posn);
    const size_t stride = is_g ? (size_t)rows_pad * q.np : (size_t)rows_pad;
    const int n_sp = q.n_sp;
    float v[SPLIT_GROUP];
#pragma unroll
    for (int u = 0; u < SPLIT_GROUP; ++u) {
      const int sp = sp0 + u < n_sp ? sp0 + u : n_sp - 1;
      const float x = src[(size_t)sp * stride];
      v[u] = sp0 + u < n_sp ? x : 0.f;
    }
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < SPLIT_GROUP; ++u) acc += (double)v[u];
    q.red[local] = acc;
  }
}

__global__ __launch_bounds__(256) void k_epilogue_batched(const BatchDesc *__restrict__ descs, int D,
                                                          const int *__restrict__ epi_start,
                                                          int pass, double tol) {
  __shared__ int s_start[MAX_D + 1];
  for (int d = threadIdx.x; d <= D; d += blockDim.x) s_start[d] = epi_start[d];
  __syncthreads();
  const int lane = threadIdx.x % 64;
  const int wid = blockIdx.x * 4 + threadIdx.x / 64;
  if (wid >= s_start[D]) return;
  const int d = find_dataset(s_start, D, wid);
  const BatchDesc &b = descs[d];
  FpControl *ctl = b.ctl;
  const int kact = ctl->kact[pass & 1];
  const int posn = wid - s_start[d];
  const int N = b.N, NP = b.np, RS = b.np + 1;
  const int groups = (b.n_sp + SPLIT_GROUP - 1) / SPLIT_GROUP;
  const int *act_cur = (pass & 1) ? b.act1 : b.act0;
  int *act_next = (pass & 1) ? b.act0 : b.act1;
  const int row = act_cur[posn];
  const int n0 = lane, n1 = lane + 64;
  double g0 = 0.0, g1 = 0.0, s4 = 0.0;
  // group sums in group order, EPI_U loads in flight per lane (a group past
  // the last adds zero)
  constexpr int EPI_U = 8;
  for (int q0 = 0; q0 < groups; q0 += EPI_U) {
    double v0[EPI_U], v1[EPI_U], v4[EPI_U];
#pragma unroll
    for (int u = 0; u < EPI_U; ++u) {
      const int q = q0 + u;
      const bool ok = q < groups;
      const double *src = b.red + ((size_t)(ok ? q : 0) * kact + posn) * RS;
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
  float *brow = b.B + (size_t)row * N;
  const double bp0 = n0 < N ? (double)brow[n0] : 0.0;
  const double bp1 = n1 < N ? (double)brow[n1] : 0.0;
  const double invT = 1.0 / (double)b.T;
  // one-term form: the linear term on the BF16-rounded row the pass's z came from
  const double bl0 = (b.bf_one && n0 < N) ? (double)(float)(__bf16)brow[n0] : bp0;
  const double bl1 = (b.bf_one && n1 < N) ? (double)(float)(__bf16)brow[n1] : bp1;
  g0 = n0 < N ? g0 * invT - 3.0 * bl0 : 0.0;
  g1 = n1 < N ? g1 * invT - 3.0 * bl1 : 0.0;
  const double gn = sqrt(wave_sum(g0 * g0 + g1 * g1));
  if (!(gn > 0.0) || !isfinite(gn)) {
    if (lane == 0) b.status[row] = OICA_ROW_DEGENERATE;
    return;
  }
  const double b0 = g0 / gn, b1 = g1 / gn;
  const double dm = wave_sum((b0 - bp0) * (b0 - bp0) + (b1 - bp1) * (b1 - bp1));
  const double dp = wave_sum((b0 + bp0) * (b0 + bp0) + (b1 + bp1) * (b1 + bp1));
  const double dd = sqrt(dm < dp ? dm : dp);
  if (n0 < N) brow[n0] = (float)b0;
  if (n1 < N) brow[n1] = (float)b1;
  if (lane == 0) {
    b.iters[row] += 1;
    if (dd < tol) {
      b.status[row] = OICA_ROW_CONV;
    } else {
      const int slot = atomicAdd(&ctl->kact[(pass + 1) & 1], 1);
      act_next[slot] = row;
    }
  }
}

hipError_t launch_batch_plan(hipStream_t st, const BatchDesc *descs, int D, BatchCtl *bctl,
                             int *item_start, long long *red_start, int *epi_start, int pass,
                             bool dry) {
  hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(1024), 0, st, descs, D, bctl, item_start,
                     red_start, epi_start, pass, dry ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_fused_batched(hipStream_t st, const BatchDesc *descs, int D, BatchCtl *bctl,
                                const int *item_start, int pass, int grid, bool bf16) {
  if (bf16)
    hipLaunchKernelGGL(k_fused_batched<true>, dim3(grid), dim3(WAVES * 64), 0, st, descs, D, bctl,
                       item_start, pass);
  else
    hipLaunchKernelGGL(k_fused_batched<false>, dim3(grid), dim3(WAVES * 64), 0, st, descs, D, bctl,
                       item_start, pass);
  return hipGetLastError();
}

hipError_t launch_epilogue_batched(hipStream_t st, const BatchDesc *descs, int D,
                                   const BatchCtl *bctl, const long long *red_start,
                                   const int *epi_start, int pass, double tol, int kmax_total) {
  hipLaunchKernelGGL(k_split_reduce_batched, dim3(RED_GRID), dim3(256), red_lds_bytes(D), st,
                     descs, D, bctl, red_start, pass);
  hipLaunchKernelGGL(k_epilogue_batched, dim3((kmax_total + 3) / 4), dim3(256), 0, st, descs, D,
                     epi_start, pass, tol);
  return hipGetLastError();
}

int batch_max_datasets() { return MAX_D; }

}  // namespace oica
