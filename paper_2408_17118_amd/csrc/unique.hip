// Unique components on gfx950: ordering criterion (eq. 1), greedy leader
// clustering up to sign in criterion order, Gaussianity walk (eq. 3).
//
// The greedy pass "each candidate, in order, joins the first representative
// within tau, else founds a cluster" is evaluated round by round: in round r
// the representative is the highest-ranked unassigned candidate (rank = the
// criterion descending, then row index), and every unassigned candidate within
// tau of it joins cluster r.  A candidate is only ever tested against
// representatives ranked above it and joins the first that matches, so this
// is the same partition as the sequential greedy pass.  Each round is one
// wide kernel (dot products and per-block arg-max) plus a one-block pick.
#include <atomic>

#include "oica_internal.h"

#include <math.h>

#include <algorithm>
#include <vector>

namespace oica {

constexpr int U_BLOCK = 256;

__device__ inline double upsilon_dev(double a) {
  if (!(a > -2.0)) return isnan(a) ? NAN : INFINITY;
  return a - 2.0 * log1p(0.5 * a);
}

// Rank comparison: true if candidate (ka, ia) ranks above (kb, ib).
__device__ inline bool ranks_above(double ka, int ia, double kb, int ib) {
  if (ib < 0) return ia >= 0;
  if (ia < 0) return false;
  return (ka > kb) || (ka == kb && ia < ib);
}

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t cluster_ws_bytes(int K, int N) {
  const int nb = (K + U_BLOCK - 1) / U_BLOCK;
  return al256((size_t)K * 8) + 3 * al256((size_t)(K + 1) * 4) + al256((size_t)nb * 4) +
         al256((size_t)K * N * 4) + al256(2 * sizeof(unsigned int)) +
         al256((size_t)2 * nb * sizeof(CoopSlot));
}

ClusterWs carve_cluster_ws(void *ws, int K, int N) {
  const int nb = (K + U_BLOCK - 1) / U_BLOCK;
  char *p = (char *)ws;
  auto take = [&](size_t bytes) {
    char *r = p;
    p += al256(bytes);
    return r;
  };
  ClusterWs w;
  w.key = (double *)take((size_t)K * 8);
  w.cluster = (int *)take((size_t)(K + 1) * 4);
  w.reps = (int *)take((size_t)(K + 1) * 4);
  w.sizes = (int *)take((size_t)(K + 1) * 4);
  w.part_idx = (int *)take((size_t)nb * 4);
  w.Wt = (float *)take((size_t)K * N * 4);
  w.done = (unsigned int *)take(2 * sizeof(unsigned int));
  w.slots = (CoopSlot *)take((size_t)2 * nb * sizeof(CoopSlot));
  return w;
}

size_t unique_workspace_bytes(int K, int N) { return cluster_ws_bytes(K, N); }

// Wt[n][l] = W[l][n]: the clustering reads candidate rows column by column, so
// the lanes of a wave (consecutive rows) read consecutive addresses.
__device__ inline void transpose_row(const float *__restrict__ W, float *__restrict__ Wt, int K,
                                     int N, int l) {
  for (int n = 0; n < N; ++n) Wt[(size_t)n * K + l] = W[(size_t)l * N + n];
}

__device__ inline const UJob &ujob(const UJob *jobs, const UJob &one) {
  return jobs ? jobs[blockIdx.y] : one;
}

__global__ void k_any_conv(const UJob *__restrict__ jobs, UJob one) {
  const UJob &j = ujob(jobs, one);
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < j.K && j.status[l] == OICA_ROW_CONV) j.ctl[0] = 1;
}

__global__ void k_prep(const UJob *__restrict__ jobs, UJob one) {
  const UJob &j = ujob(jobs, one);
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l == 0) {  // clustering counters
    j.done[0] = 0u;
    j.done[1] = 0u;
  }
  if (l >= j.K) return;
  const bool any_conv = j.ctl[0] != 0;
  const uint8_t s = j.status[l];
  bool cand = any_conv ? (s == OICA_ROW_CONV) : (s != OICA_ROW_DEGENERATE);
  const double a = j.kurt[l];
  cand = cand && isfinite(a);
  j.key[l] = cand ? upsilon_dev(a) : -INFINITY;
  j.cluster[l] = cand ? -1 : -2;
  j.sizes[l] = 0;
  transpose_row(j.W, j.Wt, j.K, j.N, l);
}

constexpr int DOT_CHUNK = 8;  // samples of a candidate row loaded before its FMAs

// One round: assign unassigned candidates within tau of representative
// reps[r] (skipped for r < 0), then per-block arg-max of the still unassigned.
__global__ __launch_bounds__(U_BLOCK) void k_assign(int K, int N, const float *__restrict__ W,
                                                    const float *__restrict__ Wt,
                                                    const double *__restrict__ key,
                                                    int *__restrict__ cluster,
                                                    int *__restrict__ reps, int r,
                                                    double tau, int *__restrict__ part_idx,
                                                    int *__restrict__ ctl,
                                                    unsigned int *__restrict__ done) {
  __shared__ double bk[U_BLOCK];
  __shared__ int bi[U_BLOCK];
  if (ctl[2]) return;  // finished in an earlier round
  const int l = blockIdx.x * U_BLOCK + threadIdx.x;
  const int rep = r >= 0 ? reps[r] : -1;
  int idx = -1;
  double kv = -INFINITY;
  if (l < K && cluster[l] == -1) {
    bool joined = false;
    if (rep >= 0) {
      const float *b = W + (size_t)rep * N;
      double dot = 0.0;
      for (int n0 = 0; n0 < N; n0 += DOT_CHUNK) {
        float v[DOT_CHUNK];  // loads of a chunk first, then the FMAs in order
#pragma unroll
        for (int j = 0; j < DOT_CHUNK; ++j)
          v[j] = n0 + j < N ? Wt[(size_t)(n0 + j) * K + l] : 0.f;
#pragma unroll
        for (int j = 0; j < DOT_CHUNK; ++j)
          if (n0 + j < N) dot = fma((double)v[j], (double)b[n0 + j], dot);
      }
      if (1.0 - fabs(dot) <= tau || l == rep) {
        cluster[l] = r;
        joined = true;
      }
    }
    if (!joined) {
      idx = l;
      kv = key[l];
    }
  }
  bk[threadIdx.x] = kv;
  bi[threadIdx.x] = idx;
  __syncthreads();
  for (int o = U_BLOCK / 2; o >= 1; o >>= 1) {
    if (threadIdx.x < o) {
      const int j = threadIdx.x + o;
      if (ranks_above(bk[j], bi[j], bk[threadIdx.x], bi[threadIdx.x])) {
        bk[threadIdx.x] = bk[j];
        bi[threadIdx.x] = bi[j];
      }
    }
    __syncthreads();
  }
  // the last work-group to finish picks the next representative from the
  // per-block arg-maxes (read past the L1, which may hold older values)
  __shared__ bool s_last;
  if (threadIdx.x == 0) {
    part_idx[blockIdx.x] = bi[0];
    __threadfence();
    s_last = atomicAdd(done, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  int best = -1;
  double bkv = -INFINITY;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += U_BLOCK) {
    const int i = __hip_atomic_load(&part_idx[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (i >= 0 && ranks_above(key[i], i, bkv, best)) {
      best = i;
      bkv = key[i];
    }
  }
  bk[threadIdx.x] = bkv;
  bi[threadIdx.x] = best;
  __syncthreads();
  for (int o = U_BLOCK / 2; o >= 1; o >>= 1) {
    if (threadIdx.x < o) {
      const int j = threadIdx.x + o;
      if (ranks_above(bk[j], bi[j], bk[threadIdx.x], bi[threadIdx.x])) {
        bk[threadIdx.x] = bk[j];
        bi[threadIdx.x] = bi[j];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    reps[r + 1] = bi[0];
    if (bi[0] < 0) {
      ctl[2] = 1;
      ctl[1] = r + 1;
    }
    *done = 0u;  // for the next round's launch
  }
}

// Cluster sizes: a work-group histogram in LDS for the first SIZE_BINS
// cluster ids (the usual case), global atomics beyond.
constexpr int SIZE_BINS = 1024;
__global__ __launch_bounds__(U_BLOCK) void k_sizes(const UJob *__restrict__ jobs, UJob one) {
  __shared__ int hist[SIZE_BINS];
  const UJob &j = ujob(jobs, one);
  for (int h = threadIdx.x; h < SIZE_BINS; h += U_BLOCK) hist[h] = 0;
  __syncthreads();
  const int l = blockIdx.x * U_BLOCK + threadIdx.x;
  if (l < j.K) {
    const int c = j.cluster[l];
    if (c >= 0 && c < SIZE_BINS)
      atomicAdd(&hist[c], 1);
    else if (c >= SIZE_BINS)
      atomicAdd(&j.sizes[c], 1);
    if (j.row_cluster) j.row_cluster[l] = c >= 0 ? c : -1;
  }
  __syncthreads();
  for (int h = threadIdx.x; h < SIZE_BINS; h += U_BLOCK)
    if (hist[h]) atomicAdd(&j.sizes[h], hist[h]);
}

// Output of the first min(U, cap) clusters, and the Gaussianity walk.
__global__ void k_finalize(const UJob *__restrict__ jobs, UJob one) {
  const UJob &j = ujob(jobs, one);
  const int N = j.N;
  const int nu = j.ctl[1];
  const int lim = nu < j.cap ? nu : j.cap;
  __shared__ int pm;
  for (int r = blockIdx.x; r < lim; r += gridDim.x) {
    const int rep = j.reps[r];
    const float *w = j.W + (size_t)rep * N;
    // sign rule: largest-magnitude entry positive, lowest index on ties
    if (threadIdx.x == 0) {
      int best = 0;
      double bv = -1.0;
      for (int n = 0; n < N; ++n) {
        const double v = fabs((double)w[n]);
        if (v > bv) {
          bv = v;
          best = n;
        }
      }
      pm = best;
    }
    __syncthreads();
    const double sg = w[pm] < 0.f ? -1.0 : 1.0;
    for (int n = threadIdx.x; n < N; n += blockDim.x) j.U[(size_t)r * N + n] = sg * (double)w[n];
    if (threadIdx.x == 0) {
      j.kurt_u[r] = j.kurt[rep];
      j.ups_u[r] = j.key[rep];
      j.rep_thread[r] = rep;
      j.csize[r] = j.sizes[r];
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int acc = nu;
    if (j.gtest) {
      acc = 0;
      for (int r = 1; r <= nu; ++r) {
        const double thr = 2.0 * (double)(N - r + 2) * (double)(N - r + 1) / (double)j.T;
        if (j.key[j.reps[r - 1]] < thr) break;
        acc = r;
      }
    }
    if (j.n_top > 0 && acc > j.n_top) acc = j.n_top;
    j.ctl[3] = acc;
  }
}

// All rounds in one work-group (problems with K <= CW_MAX_K; several problems
// in one launch, one work-group each).  Each thread keeps the cluster state
// and key of its rows in registers; a round is one pass (assign to the current
// representative, arg-max of the rest) and a block arg-max: three barriers per
// round instead of two kernel launches.  The dot products are the ones k_assign
// computes, in the same order, so the partition is identical.
constexpr int CW_THREADS = 1024;

__device__ inline void cw_better(double &bk, int &bi, double k2, int i2) {
  if (ranks_above(k2, i2, bk, bi)) {
    bk = k2;
    bi = i2;
  }
}

// R rows per thread (K <= R * CW_THREADS); each row's dot product loads C
// features before their FMAs (R = 1: up to 1024 rows, longer chunks keep more
// loads in flight).
template <int R, int C>
__global__ __launch_bounds__(CW_THREADS) void k_cluster_wg(const ClusterJob *__restrict__ jobs,
                                                           ClusterJob one, double tau) {
  __shared__ double lw[OICA_MAX_N];
  __shared__ double wk[CW_THREADS / 64];
  __shared__ int wi[CW_THREADS / 64];
  __shared__ int s_leader;
  // representatives in LDS while the rounds run (a global store in the
  // loop would leave the loads' wait counter ambiguous), written at the end
  __shared__ int s_reps[CW_MAX_K + 1];
  const ClusterJob jb = jobs ? jobs[blockIdx.x] : one;
  const int K = jb.K, N = jb.N;
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const float *__restrict__ Wt = jb.Wt;
  // this thread's rows l = tid + i * CW_THREADS: cluster state and key
  int cl[R];
  double key[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int l = tid + i * CW_THREADS;
    cl[i] = l < K ? jb.cluster[l] : -2;
    key[i] = cl[i] == -1 ? jb.key[l] : -INFINITY;
  }
  int leader = -1;
  int r = -1;
  for (;;) {
    // assign to the current leader (round r), arg-max of the unassigned rest
    if (leader >= 0) {
      double dot[R];
#pragma unroll
      for (int i = 0; i < R; ++i) dot[i] = 0.0;
      if constexpr (R == 1) {
        // one row per thread: the chunks unrolled up to OICA_MAX_N features,
        // the loads PF chunks ahead of the FMAs (no loop back-edge, so each
        // wait is for the chunk in use only; same FMAs in the same order)
        constexpr int NCH = (OICA_MAX_N + C - 1) / C;
        const bool live = cl[0] == -1;
        // feature n of this thread's row through a buffer resource: the
        // column offset n K is a scalar offset and the row the one vector
        // offset, so the loads need no address registers
        // (the job's fields are uniform; readfirstlane lets the compiler know)
        const unsigned long long wp = (unsigned long long)(size_t)Wt;
        const unsigned int wlo = __builtin_amdgcn_readfirstlane((unsigned int)wp);
        const unsigned int whi = __builtin_amdgcn_readfirstlane((unsigned int)(wp >> 32));
        const int Ku = __builtin_amdgcn_readfirstlane(K), Nu = __builtin_amdgcn_readfirstlane(N);
        const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(size_t)(((unsigned long long)whi << 32) | wlo), (short)0,
            Ku * Nu * (int)sizeof(float), 0x00020000);
        // A row that is not live takes a vector offset past the records, which
        // the range check turns into a zero without a memory access; features
        // past N (the prefetch of the last chunks) read feature N - 1, whose
        // products are never added.
        const int voff = live ? tid * (int)sizeof(float) : (int)0x80000000u;
        auto ld = [&](int n) -> float {
          const int soff = (n < Nu ? n : Nu - 1) * Ku * (int)sizeof(float);
          return __builtin_bit_cast(float,
                                    __builtin_amdgcn_raw_buffer_load_b32(rsrc, voff, soff, 0));
        };
        // PF chunks of loads in flight ahead of the FMAs (a chunk's FMAs are
        // far shorter than an L2 latency)
        constexpr int PF = 3;
        float v[PF + 1][C];
#pragma unroll
        for (int c0 = 0; c0 < PF && c0 < NCH; ++c0)
#pragma unroll
          for (int j = 0; j < C; ++j) v[c0][j] = ld(c0 * C + j);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          const int n0 = ch * C;
          if (n0 >= Nu) break;
          if (ch + PF < NCH) {
#pragma unroll
            for (int j = 0; j < C; ++j) v[(ch + PF) % (PF + 1)][j] = ld(n0 + PF * C + j);
          }
#pragma unroll
          for (int j = 0; j < C; ++j)
            if (n0 + j < Nu) dot[0] = fma((double)v[ch % (PF + 1)][j], lw[n0 + j], dot[0]);
          // keep each chunk's LDS reads in its own step (hoisted together
          // they would need 2 * OICA_MAX_N registers)
          __builtin_amdgcn_sched_barrier(0);
        }
      } else {
        for (int n0 = 0; n0 < N; n0 += C) {
          float v[R][C];  // every load of the chunk first, then the FMAs in order
#pragma unroll
          for (int i = 0; i < R; ++i)
#pragma unroll
            for (int j = 0; j < C; ++j)
              v[i][j] = (cl[i] == -1 && n0 + j < N)
                            ? Wt[(size_t)(n0 + j) * K + tid + i * CW_THREADS]
                            : 0.f;
#pragma unroll
          for (int i = 0; i < R; ++i)
#pragma unroll
            for (int j = 0; j < C; ++j)
              if (n0 + j < N) dot[i] = fma((double)v[i][j], lw[n0 + j], dot[i]);
        }
      }
#pragma unroll
      for (int i = 0; i < R; ++i)
        if (cl[i] == -1 && (1.0 - fabs(dot[i]) <= tau || tid + i * CW_THREADS == leader)) cl[i] = r;
    }
    double bk = -INFINITY;
    int bi = -1;
#pragma unroll
    for (int i = 0; i < R; ++i)
      if (cl[i] == -1) cw_better(bk, bi, key[i], tid + i * CW_THREADS);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double k2 = __shfl_xor(bk, o);
      const int i2 = __shfl_xor(bi, o);
      cw_better(bk, bi, k2, i2);
    }
    if (lane == 0) {
      wk[wave] = bk;
      wi[wave] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double k0 = wk[0];
      int i0 = wi[0];
      for (int w = 1; w < CW_THREADS / 64; ++w) cw_better(k0, i0, wk[w], wi[w]);
      s_leader = i0;
      s_reps[r + 1] = i0;  // -1 after the last cluster
    }
    __syncthreads();
    leader = s_leader;
    if (leader < 0) break;
    ++r;
    for (int n = tid; n < N; n += CW_THREADS) lw[n] = (double)jb.W[(size_t)leader * N + n];
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int l = tid + i * CW_THREADS;
    if (l < K) jb.cluster[l] = cl[i];
  }
  for (int i = tid; i <= r + 1; i += CW_THREADS) jb.reps[i] = s_reps[i];
  if (tid == 0) {
    jb.ctl[1] = r + 1;
    jb.ctl[2] = 1;
  }
}

hipError_t launch_cluster_wg(hipStream_t st, int D, const ClusterJob *jobs_dev,
                             const ClusterJob &one, double tau, int k_max) {
  if (k_max <= CW_THREADS)
    hipLaunchKernelGGL((k_cluster_wg<1, 16>), dim3(D), dim3(CW_THREADS), 0, st, jobs_dev, one, tau);
  else
    hipLaunchKernelGGL((k_cluster_wg<CW_MAX_K / CW_THREADS, DOT_CHUNK / 2>), dim3(D),
                       dim3(CW_THREADS), 0, st, jobs_dev, one, tau);
  return hipGetLastError();
}

// All rounds in one launch whose work-groups are all resident at once: each
// thread keeps its candidate row in registers; a round is the dot products
// with the current representative, a work-group arg-max, and a grid-wide
// exchange of the per-group arg-maxes through `slots` (two sets, by round
// parity): a work-group stores the round's stamp and its arg-max's row index
// in one 64-bit word of its slot, and the first wave of every work-group polls
// all slots (one lane per slot) until each carries the stamp, then reduces
// them by key[index].  No store is ordered after another, so no fence is
// needed (an acquire fence there would also drop the L2 lines that the next
// representative's row is read from).
// Every work-group reduces the same slots in the same way, so all agree on
// the next representative.  (An arrival counter that every work-group
// incremented, waited on by one thread before a separate read of the slots,
// took ~9.5 us per round at K = 16384.)  A wait that
// exceeds its bound (about half a second) sets done[1]; every work-group then
// ends at its next exchange and puts its rows back in their state on entry,
// and the host redoes the clustering round by round.  The dot products are
// k_assign's, in the same order, so the partition is identical.
constexpr int CO_BLOCK = 256;
constexpr int CO_SPIN_LIMIT = 1 << 24;

template <int NP>
__global__ __launch_bounds__(CO_BLOCK) void k_cluster_coop(int K, int N, const float *__restrict__ W,
                                                           const double *__restrict__ key,
                                                           int *__restrict__ cluster,
                                                           int *__restrict__ reps, double tau,
                                                           CoopSlot *slots, unsigned int *done,
                                                           int *__restrict__ ctl) {
  __shared__ double lw[NP];
  __shared__ double wk[CO_BLOCK / 64];
  __shared__ int wi[CO_BLOCK / 64];
  __shared__ int s_leader;
  const int nwg = gridDim.x;
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int l = blockIdx.x * CO_BLOCK + tid;
  const bool have = l < K;
  const int cl0 = have ? cluster[l] : -2;
  int cl = cl0;
  const double kv = cl == -1 ? key[l] : -INFINITY;
  float row[NP];
#pragma unroll
  for (int n = 0; n < NP; ++n) row[n] = (have && n < N) ? W[(size_t)l * N + n] : 0.f;
  int leader = -1, r = -1;
  for (unsigned int round = 0;; ++round) {
    if (leader >= 0 && cl == -1) {
      double dot = 0.0;
#pragma unroll
      for (int n = 0; n < NP; ++n)
        if (n < N) dot = fma((double)row[n], lw[n], dot);
      if (1.0 - fabs(dot) <= tau || l == leader) cl = r;
    }
    double bk = cl == -1 ? kv : -INFINITY;
    int bi = cl == -1 ? l : -1;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double k2 = __shfl_xor(bk, o);
      const int i2 = __shfl_xor(bi, o);
      if (ranks_above(k2, i2, bk, bi)) {
        bk = k2;
        bi = i2;
      }
    }
    if (lane == 0) {
      wk[wave] = bk;
      wi[wave] = bi;
    }
    __syncthreads();
    if (wave == 0) {
      // publish this work-group's arg-max for the round: the row index and
      // the round's stamp in one 64-bit word (its key is key[index], which
      // no work-group writes), so no other store needs ordering
      if (tid == 0) {
        double k0 = wk[0];
        int i0 = wi[0];
        for (int w = 1; w < CO_BLOCK / 64; ++w)
          if (ranks_above(wk[w], wi[w], k0, i0)) {
            k0 = wk[w];
            i0 = wi[w];
          }
        CoopSlot *sl = slots + (size_t)(round & 1) * nwg + blockIdx.x;
        const unsigned long long word =
            ((unsigned long long)(round + 1u) << 32) | (unsigned long long)(unsigned int)i0;
        __hip_atomic_store(&sl->word, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      // every work-group waits for and reduces the same slots (lane b polls
      // work-group b's), so all agree on the next representative
      double gk = -INFINITY;
      int gi = -1;
      bool quit = false;
      for (int b = lane; b < nwg && !quit; b += 64) {
        const CoopSlot *sl = slots + (size_t)(round & 1) * nwg + b;
        int spins = 0;
        unsigned long long word;
        while (((word = __hip_atomic_load(&sl->word, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT)) >> 32) != round + 1u) {
          if (++spins > CO_SPIN_LIMIT ||
              __hip_atomic_load(&done[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            quit = true;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        if (quit) break;
        const int i2 = (int)(unsigned int)word;
        const double k2 = i2 >= 0 ? key[i2] : -INFINITY;
        if (ranks_above(k2, i2, gk, gi)) {
          gk = k2;
          gi = i2;
        }
      }
      if (quit) atomicOr(&done[1], 1u);
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const double k2 = __shfl_xor(gk, o);
        const int i2 = __shfl_xor(gi, o);
        if (ranks_above(k2, i2, gk, gi)) {
          gk = k2;
          gi = i2;
        }
      }
      if (lane == 0) {
        if (__hip_atomic_load(&done[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) gi = -1;
        s_leader = gi;
        if (blockIdx.x == 0) reps[r + 1] = gi;  // -1 after the last cluster
      }
    }
    __syncthreads();
    leader = s_leader;
    if (leader < 0) break;
    ++r;
    for (int n = tid; n < N; n += CO_BLOCK) lw[n] = (double)W[(size_t)leader * N + n];
    __syncthreads();
  }
  // given up: the rows go back to their state on entry for the round-by-round
  // form (every work-group has seen done[1] by the time it leaves the loop)
  const bool gave_up = __hip_atomic_load(&done[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
  if (have) cluster[l] = gave_up ? cl0 : cl;
  if (blockIdx.x == 0 && tid == 0 && !gave_up) {
    ctl[1] = r + 1;
    ctl[2] = 1;
  }
}

// The stamps start at zero for every all-rounds launch, so a stamp left by an
// earlier launch on the same workspace never matches a round.
__global__ void k_coop_reset(CoopSlot *slots, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) slots[i].word = 0ull;
}

static std::atomic<int> g_coop_give_up{0};
static std::atomic<int> g_coop_fallbacks{0};
static std::atomic<int> g_coop_api{1};
void set_coop_give_up(bool on) { g_coop_give_up.store(on ? 1 : 0); }
void set_coop_launch_api(bool on) { g_coop_api.store(on ? 1 : 0); }
int coop_launch_api() { return g_coop_api.load(); }
int coop_fallbacks() { return g_coop_fallbacks.load(); }

// Launch of k_cluster_coop when every work-group fits on the device at once
// (the stream is in order, so the device is otherwise free for it);
// *launched = false (nothing enqueued) otherwise.
static hipError_t launch_cluster_coop(hipStream_t st, int N, int K, const float *W,
                                      const ClusterWs &cw, double tau, int *ctl_dev,
                                      bool *launched) {
  *launched = false;
  const int grid = (K + CO_BLOCK - 1) / CO_BLOCK;
  const int np = ((N + 31) / 32) * 32;
  const void *fn = np <= 32   ? (const void *)k_cluster_coop<32>
                   : np <= 64 ? (const void *)k_cluster_coop<64>
                   : np <= 96 ? (const void *)k_cluster_coop<96>
                              : (const void *)k_cluster_coop<128>;
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, CO_BLOCK, 0);
  if (e != hipSuccess) return e;
  if ((long long)per_cu * cus < grid) return hipSuccess;
  const double *key = cw.key;
  int *cluster = cw.cluster, *reps = cw.reps;
  CoopSlot *slots = cw.slots;
  unsigned int *done = cw.done;
  hipLaunchKernelGGL(k_coop_reset, dim3((2 * grid + 255) / 256), dim3(256), 0, st, slots, 2 * grid);
  if (g_coop_give_up.load()) {  // test switch: start with the give-up flag set
    e = hipMemsetAsync(done + 1, 0xFF, sizeof(unsigned int), st);
    if (e != hipSuccess) return e;
  }
  void *args[] = {(void *)&K, (void *)&N, (void *)&W, (void *)&key, (void *)&cluster, (void *)&reps,
                  (void *)&tau, (void *)&slots, (void *)&done, (void *)&ctl_dev};
  e = g_coop_api.load() ? hipLaunchCooperativeKernel(fn, dim3(grid), dim3(CO_BLOCK), args, 0, st)
                        : hipLaunchKernel(fn, dim3(grid), dim3(CO_BLOCK), args, 0, st);
  if (e != hipSuccess) {  // refused (not all co-resident): the round-by-round form
    (void)hipGetLastError();
    return hipSuccess;
  }
  *launched = true;
  return hipSuccess;
}

// Greedy leader clustering of the candidates (cluster[l] == -1 on entry) in
// (key descending, row index) order; writes cluster ids, the representative of
// every cluster (reps[0..n)), and n into ctl_dev[1] / ctl_host[1].
// ctl_dev (4 ints) must be zero on entry except ctl_dev[0].  Synchronises.
// W is read through its transposed copy in cw.Wt (written by the prep kernel).
hipError_t launch_cluster(hipStream_t st, int N, int K, const float *W, const ClusterWs &cw,
                          double tau, int *ctl_dev, int *ctl_host) {
  const int nb = (K + U_BLOCK - 1) / U_BLOCK;
  const double *key = cw.key;
  int *cluster = cw.cluster, *reps = cw.reps, *part_idx = cw.part_idx;
  const float *Wt = cw.Wt;
  if (cluster_in_one_wg(K, false)) {
    const ClusterJob job{K, N, W, Wt, key, cluster, reps, ctl_dev};
    hipError_t e = launch_cluster_wg(st, 1, nullptr, job, tau, K);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(ctl_host, ctl_dev, 4 * sizeof(int), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
  }
  {
    bool launched = false;
    hipError_t e = launch_cluster_coop(st, N, K, W, cw, tau, ctl_dev, &launched);
    if (e != hipSuccess) return e;
    if (launched) {
      unsigned int flags[2] = {0u, 0u};
      e = hipMemcpyAsync(ctl_host, ctl_dev, 4 * sizeof(int), hipMemcpyDeviceToHost, st);
      if (e != hipSuccess) return e;
      e = hipMemcpyAsync(flags, cw.done, sizeof flags, hipMemcpyDeviceToHost, st);
      if (e != hipSuccess) return e;
      e = hipStreamSynchronize(st);
      if (e != hipSuccess) return e;
      if (!flags[1]) return hipSuccess;
      // the bounded wait gave up: redo the clustering round by round from the
      // rows' state on entry (restored by the kernel)
      g_coop_fallbacks.fetch_add(1);
      e = hipMemsetAsync(ctl_dev + 1, 0, 3 * sizeof(int), st);
      if (e != hipSuccess) return e;
      e = hipMemsetAsync(cw.done, 0, 2 * sizeof(unsigned int), st);
      if (e != hipSuccess) return e;
    }
  }
  // round -1: arg-max only; then rounds 0, 1, ... until no candidate is left.
  // Each round is one launch; its last work-group picks the next representative.
  hipLaunchKernelGGL(k_assign, dim3(nb), dim3(U_BLOCK), 0, st, K, N, W, Wt, key, cluster, reps,
                     -1, tau, part_idx, ctl_dev, cw.done);
  const int BATCH = 16;
  for (int r0 = 0; r0 <= K; r0 += BATCH) {
    for (int r = r0; r < r0 + BATCH && r <= K; ++r)
      hipLaunchKernelGGL(k_assign, dim3(nb), dim3(U_BLOCK), 0, st, K, N, W, Wt, key, cluster,
                         reps, r, tau, part_idx, ctl_dev, cw.done);
    hipError_t e = hipMemcpyAsync(ctl_host, ctl_dev, 4 * sizeof(int), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    if (ctl_host[2]) break;
  }
  return hipGetLastError();
}

// Candidates for grouping the rows that converged on BF16 data: every CONV row,
// all with the same key, so the lowest row index of a group represents it.
__global__ void k_prep_groups(int K, int N, const uint8_t *__restrict__ status,
                              const float *__restrict__ W, ClusterWs cw) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l == 0) {  // clustering counters
    cw.done[0] = 0u;
    cw.done[1] = 0u;
  }
  if (l >= K) return;
  const bool cand = status[l] == OICA_ROW_CONV;
  cw.key[l] = cand ? 0.0 : -INFINITY;
  cw.cluster[l] = cand ? -1 : -2;
  transpose_row(W, cw.Wt, K, N, l);
}

hipError_t launch_prep_groups(hipStream_t st, int K, int N, const uint8_t *status, const float *W,
                              const ClusterWs &cw) {
  hipLaunchKernelGGL(k_prep_groups, dim3((K + U_BLOCK - 1) / U_BLOCK), dim3(U_BLOCK), 0, st, K, N,
                     status, W, cw);
  return hipGetLastError();
}

hipError_t launch_groups(hipStream_t st, int N, int K, const float *W, const uint8_t *status,
                         double tau, void *ws, int *ctl_dev, int *ctl_host, int **cluster_out,
                         int **reps_out) {
  const ClusterWs cw = carve_cluster_ws(ws, K, N);
  hipError_t e = launch_prep_groups(st, K, N, status, W, cw);
  if (e != hipSuccess) return e;
  e = launch_cluster(st, N, K, W, cw, tau, ctl_dev, ctl_host);
  *cluster_out = cw.cluster;
  *reps_out = cw.reps;
  return e;
}

// Carve one problem's workspace (unique_workspace_bytes(K, N) bytes at ws).
static ClusterWs carve_ujob(UJob &j, void *ws) {
  const ClusterWs cw = carve_cluster_ws(ws, j.K, j.N);
  j.key = cw.key;
  j.cluster = cw.cluster;
  j.part_idx = cw.part_idx;
  j.reps = cw.reps;
  j.sizes = cw.sizes;
  j.Wt = cw.Wt;
  j.done = cw.done;
  j.slots = cw.slots;
  return cw;
}

hipError_t launch_unique(hipStream_t st, int N, int64_t T, int K, const float *W,
                         const double *kurt, const uint8_t *status, double tau, int gtest,
                         int n_top, int cap, double *U, double *kurt_u, double *ups_u,
                         int32_t *rep_thread, int32_t *cluster_size, void *ws, int *counts_host,
                         int *counts_dev, int32_t *row_cluster) {
  const int nb = (K + U_BLOCK - 1) / U_BLOCK;
  UJob j{K, N, (long long)T, W, kurt, status, tau, gtest, n_top, cap, U, kurt_u, ups_u,
         rep_thread, cluster_size, row_cluster};
  const ClusterWs cw = carve_ujob(j, ws);
  j.ctl = counts_dev;  // 4 ints, zeroed by the caller
  hipLaunchKernelGGL(k_any_conv, dim3(nb), dim3(U_BLOCK), 0, st, nullptr, j);
  hipLaunchKernelGGL(k_prep, dim3(nb), dim3(U_BLOCK), 0, st, nullptr, j);
  hipError_t e = launch_cluster(st, N, K, W, cw, tau, j.ctl, counts_host);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sizes, dim3(nb), dim3(U_BLOCK), 0, st, nullptr, j);
  hipLaunchKernelGGL(k_finalize, dim3(64), dim3(128), 0, st, nullptr, j);
  e = hipMemcpyAsync(counts_host, j.ctl, 4 * sizeof(int), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

size_t unique_batched_workspace_bytes(int D, const UJob *jobs) {
  size_t b = 2 * (((size_t)D * sizeof(UJob) + 255) & ~(size_t)255) + (size_t)D * 4 * sizeof(int) + 512;
  for (int d = 0; d < D; ++d) b += unique_workspace_bytes(jobs[d].K, jobs[d].N) + 256;
  return b;
}

// Many problems: the per-row kernels cover every problem in one launch
// (blockIdx.y = problem), the problems small enough for one work-group are
// clustered in one launch, the others round by round one after another.
// jobs: host table with the problem fields set; counts_host: D x 4 ints
// ([1] clusters, [3] accepted per problem).  Synchronises.
hipError_t launch_unique_batched(hipStream_t st, int D, UJob *jobs, void *ws, int *counts_host) {
  char *p = (char *)ws;
  auto take = [&](size_t bytes) {
    char *r = p;
    p += (bytes + 255) & ~(size_t)255;
    return r;
  };
  UJob *jobs_dev = (UJob *)take((size_t)D * sizeof(UJob));
  ClusterJob *cjobs_dev = (ClusterJob *)take((size_t)D * sizeof(UJob));
  int *ctl = (int *)take((size_t)D * 4 * sizeof(int));
  int k_max = 1;
  std::vector<ClusterJob> small;
  std::vector<ClusterWs> cws(D);
  for (int d = 0; d < D; ++d) {
    cws[d] = carve_ujob(jobs[d], take(unique_workspace_bytes(jobs[d].K, jobs[d].N)));
    jobs[d].ctl = ctl + 4 * d;
    k_max = std::max(k_max, jobs[d].K);
    if (cluster_in_one_wg(jobs[d].K, true))
      small.push_back(ClusterJob{jobs[d].K, jobs[d].N, jobs[d].W, jobs[d].Wt, jobs[d].key,
                                 jobs[d].cluster, jobs[d].reps, jobs[d].ctl});
  }
  hipError_t e = hipMemsetAsync(ctl, 0, (size_t)D * 4 * sizeof(int), st);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(jobs_dev, jobs, (size_t)D * sizeof(UJob), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  if (!small.empty()) {
    e = hipMemcpyAsync(cjobs_dev, small.data(), small.size() * sizeof(ClusterJob),
                       hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
  }
  e = hipStreamSynchronize(st);  // the host tables may go out of scope
  if (e != hipSuccess) return e;
  const int nb = (k_max + U_BLOCK - 1) / U_BLOCK;
  const UJob none{};
  hipLaunchKernelGGL(k_any_conv, dim3(nb, D), dim3(U_BLOCK), 0, st, jobs_dev, none);
  hipLaunchKernelGGL(k_prep, dim3(nb, D), dim3(U_BLOCK), 0, st, jobs_dev, none);
  if (!small.empty()) {
    int k_small = 0;
    for (const ClusterJob &j : small) k_small = std::max(k_small, j.K);
    e = launch_cluster_wg(st, (int)small.size(), cjobs_dev, small[0], jobs[0].tau, k_small);
    if (e != hipSuccess) return e;
  }
  for (int d = 0; d < D; ++d)
    if (!cluster_in_one_wg(jobs[d].K, true)) {
      e = launch_cluster(st, jobs[d].N, jobs[d].K, jobs[d].W, cws[d], jobs[d].tau, jobs[d].ctl,
                         counts_host);
      if (e != hipSuccess) return e;
    }
  hipLaunchKernelGGL(k_sizes, dim3(nb, D), dim3(U_BLOCK), 0, st, jobs_dev, none);
  hipLaunchKernelGGL(k_finalize, dim3(64, D), dim3(128), 0, st, jobs_dev, none);
  e = hipMemcpyAsync(counts_host, ctl, (size_t)D * 4 * sizeof(int), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace oica
