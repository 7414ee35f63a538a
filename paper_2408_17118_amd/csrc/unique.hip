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
#include "oica_internal.h"

#include <math.h>

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

struct UniqueWs {
  double *key;      // K: criterion of each candidate
  int *cluster;     // K: -2 not a candidate, -1 unassigned, >= 0 cluster id
  int *part_idx;    // blocks: best unassigned index per block
  int *reps;        // K + 1: representative of each round
  int *ctl;         // [0] any CONV, [1] number of clusters, [2] done, [3] accepted
  int *sizes;       // K
};

size_t unique_workspace_bytes(int K) {
  const int nb = (K + U_BLOCK - 1) / U_BLOCK;
  return (size_t)K * 8 + (size_t)K * 4 + (size_t)nb * 4 + (size_t)(K + 1) * 4 + 64 +
         (size_t)K * 4 + 6 * 256;
}

__global__ void k_any_conv(int K, const uint8_t *__restrict__ status, int *ctl) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < K && status[l] == OICA_ROW_CONV) ctl[0] = 1;
}

__global__ void k_prep(int K, const double *__restrict__ kurt, const uint8_t *__restrict__ status,
                       const int *__restrict__ ctl, double *__restrict__ key,
                       int *__restrict__ cluster, int *__restrict__ sizes) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= K) return;
  const bool any_conv = ctl[0] != 0;
  const uint8_t s = status[l];
  bool cand = any_conv ? (s == OICA_ROW_CONV) : (s != OICA_ROW_DEGENERATE);
  const double a = kurt[l];
  cand = cand && isfinite(a);
  key[l] = cand ? upsilon_dev(a) : -INFINITY;
  cluster[l] = cand ? -1 : -2;
  sizes[l] = 0;
}

// One round: assign unassigned candidates within tau of representative
// reps[r] (skipped for r < 0), then per-block arg-max of the still unassigned.
__global__ __launch_bounds__(U_BLOCK) void k_assign(int K, int N, const float *__restrict__ W,
                                                    const double *__restrict__ key,
                                                    int *__restrict__ cluster,
                                                    const int *__restrict__ reps, int r,
                                                    double tau, int *__restrict__ part_idx,
                                                    const int *__restrict__ ctl) {
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
      const float *a = W + (size_t)l * N;
      const float *b = W + (size_t)rep * N;
      double dot = 0.0;
      for (int n = 0; n < N; ++n) dot = fma((double)a[n], (double)b[n], dot);
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
  if (threadIdx.x == 0) part_idx[blockIdx.x] = bi[0];
}

__global__ __launch_bounds__(U_BLOCK) void k_pick(int nblocks, const double *__restrict__ key,
                                                  const int *__restrict__ part_idx,
                                                  int *__restrict__ reps, int r,
                                                  int *__restrict__ ctl) {
  __shared__ double bk[U_BLOCK];
  __shared__ int bi[U_BLOCK];
  if (ctl[2]) return;
  int best = -1;
  double bkv = -INFINITY;
  for (int b = threadIdx.x; b < nblocks; b += U_BLOCK) {
    const int i = part_idx[b];
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
  }
}

__global__ void k_sizes(int K, const int *__restrict__ cluster, int *__restrict__ sizes,
                        int32_t *__restrict__ row_cluster) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= K) return;
  const int c = cluster[l];
  if (c >= 0) atomicAdd(&sizes[c], 1);
  if (row_cluster) row_cluster[l] = c >= 0 ? c : -1;
}

// Output of the first min(U, cap) clusters, and the Gaussianity walk.
__global__ void k_finalize(int N, long long T, const float *__restrict__ W,
                           const double *__restrict__ kurt, const double *__restrict__ key,
                           const int *__restrict__ reps, const int *__restrict__ sizes, int gtest,
                           int n_top, int cap, double *__restrict__ U, double *__restrict__ kurt_u,
                           double *__restrict__ ups_u, int32_t *__restrict__ rep_thread,
                           int32_t *__restrict__ csize, int *__restrict__ ctl) {
  const int nu = ctl[1];
  const int lim = nu < cap ? nu : cap;
  __shared__ int pm;
  for (int r = blockIdx.x; r < lim; r += gridDim.x) {
    const int rep = reps[r];
    const float *w = W + (size_t)rep * N;
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
    for (int n = threadIdx.x; n < N; n += blockDim.x) U[(size_t)r * N + n] = sg * (double)w[n];
    if (threadIdx.x == 0) {
      kurt_u[r] = kurt[rep];
      ups_u[r] = key[rep];
      rep_thread[r] = rep;
      csize[r] = sizes[r];
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int acc = nu;
    if (gtest) {
      acc = 0;
      for (int r = 1; r <= nu; ++r) {
        const double thr = 2.0 * (double)(N - r + 2) * (double)(N - r + 1) / (double)T;
        if (key[reps[r - 1]] < thr) break;
        acc = r;
      }
    }
    if (n_top > 0 && acc > n_top) acc = n_top;
    ctl[3] = acc;
  }
}

// Greedy leader clustering of the candidates (cluster[l] == -1 on entry) in
// (key descending, row index) order; writes cluster ids, the representative of
// every cluster (reps[0..n)), and n into ctl_dev[1] / ctl_host[1].
// ctl_dev (4 ints) must be zero on entry except ctl_dev[0].  Synchronises.
hipError_t launch_cluster(hipStream_t st, int N, int K, const float *W, const double *key,
                          int *cluster, int *reps, int *part_idx, double tau, int *ctl_dev,
                          int *ctl_host) {
  const int nb = (K + U_BLOCK - 1) / U_BLOCK;
  // round -1: arg-max only; then rounds 0, 1, ... until no candidate is left
  hipLaunchKernelGGL(k_assign, dim3(nb), dim3(U_BLOCK), 0, st, K, N, W, key, cluster, reps, -1,
                     tau, part_idx, ctl_dev);
  hipLaunchKernelGGL(k_pick, dim3(1), dim3(U_BLOCK), 0, st, nb, key, part_idx, reps, -1,
                     ctl_dev);  // writes reps[0]
  const int BATCH = 16;
  for (int r0 = 0; r0 <= K; r0 += BATCH) {
    for (int r = r0; r < r0 + BATCH && r <= K; ++r) {
      hipLaunchKernelGGL(k_assign, dim3(nb), dim3(U_BLOCK), 0, st, K, N, W, key, cluster, reps, r,
                         tau, part_idx, ctl_dev);
      hipLaunchKernelGGL(k_pick, dim3(1), dim3(U_BLOCK), 0, st, nb, key, part_idx, reps, r,
                         ctl_dev);
    }
    hipError_t e = hipMemcpyAsync(ctl_host, ctl_dev, 4 * sizeof(int), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    if (ctl_host[2]) break;
  }
  return hipGetLastError();
}

size_t cluster_workspace_bytes(int K) { return unique_workspace_bytes(K); }

// Candidates for grouping the rows that converged on BF16 data: every CONV row,
// all with the same key, so the lowest row index of a group represents it.
__global__ void k_prep_groups(int K, const uint8_t *__restrict__ status, double *__restrict__ key,
                              int *__restrict__ cluster) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= K) return;
  const bool cand = status[l] == OICA_ROW_CONV;
  key[l] = cand ? 0.0 : -INFINITY;
  cluster[l] = cand ? -1 : -2;
}

hipError_t launch_groups(hipStream_t st, int N, int K, const float *W, const uint8_t *status,
                         double tau, void *ws, int *ctl_dev, int *ctl_host, int **cluster_out,
                         int **reps_out) {
  const int nb = (K + U_BLOCK - 1) / U_BLOCK;
  char *p = (char *)ws;
  auto take = [&](size_t bytes) {
    char *r = p;
    p += (bytes + 255) & ~(size_t)255;
    return r;
  };
  double *key = (double *)take((size_t)K * 8);
  int *cluster = (int *)take((size_t)K * 4);
  int *part_idx = (int *)take((size_t)nb * 4);
  int *reps = (int *)take((size_t)(K + 1) * 4);
  hipLaunchKernelGGL(k_prep_groups, dim3(nb), dim3(U_BLOCK), 0, st, K, status, key, cluster);
  hipError_t e = launch_cluster(st, N, K, W, key, cluster, reps, part_idx, tau, ctl_dev, ctl_host);
  *cluster_out = cluster;
  *reps_out = reps;
  return e;
}

hipError_t launch_unique(hipStream_t st, int N, int64_t T, int K, const float *W,
                         const double *kurt, const uint8_t *status, double tau, int gtest,
                         int n_top, int cap, double *U, double *kurt_u, double *ups_u,
                         int32_t *rep_thread, int32_t *cluster_size, void *ws, int *counts_host,
                         int *counts_dev, int32_t *row_cluster) {
  const int nb = (K + U_BLOCK - 1) / U_BLOCK;
  char *p = (char *)ws;
  auto take = [&](size_t bytes) {
    char *r = p;
    p += (bytes + 255) & ~(size_t)255;
    return r;
  };
  UniqueWs w;
  w.key = (double *)take((size_t)K * 8);
  w.cluster = (int *)take((size_t)K * 4);
  w.part_idx = (int *)take((size_t)nb * 4);
  w.reps = (int *)take((size_t)(K + 1) * 4);
  w.sizes = (int *)take((size_t)K * 4);
  w.ctl = counts_dev;  // 4 ints, zeroed by the caller

  hipLaunchKernelGGL(k_any_conv, dim3(nb), dim3(U_BLOCK), 0, st, K, status, w.ctl);
  hipLaunchKernelGGL(k_prep, dim3(nb), dim3(U_BLOCK), 0, st, K, kurt, status, w.ctl, w.key,
                     w.cluster, w.sizes);
  hipError_t e = launch_cluster(st, N, K, W, w.key, w.cluster, w.reps, w.part_idx, tau, w.ctl,
                                counts_host);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sizes, dim3(nb), dim3(U_BLOCK), 0, st, K, w.cluster, w.sizes, row_cluster);
  hipLaunchKernelGGL(k_finalize, dim3(64), dim3(128), 0, st, N, (long long)T, W, kurt, w.key,
                     w.reps, w.sizes, gtest, n_top, cap, U, kurt_u, ups_u, rep_thread,
                     cluster_size, w.ctl);
  e = hipMemcpyAsync(counts_host, w.ctl, 4 * sizeof(int), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace oica
