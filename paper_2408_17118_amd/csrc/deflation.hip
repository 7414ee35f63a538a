// Small FP64 kernels of the deflation driver (Sec. 3.3, eqs. 6-8): the basis
// of the complement of the components found so far, and the mapping of a
// reduced-space row back to the whitened space.  All sizes are at most
// OICA_MAX_N, so each kernel is one or a few work-groups; the dominant work of
// a step (the reduction X~ = G Xw and the fixed point) runs in the apply and
// fused kernels.
#include "oica_internal.h"

namespace oica {

namespace {

constexpr int DT = 256;  // threads per work-group

// Ft[a][j] = delta_aj - sum_k W[k][a] W[k][j] for a < n = N - n_prev (the
// first n rows of F = I - W^T W, eq. 6, i.e. F with its bottom n_prev rows
// deleted); then C = Ft Ft^T (n x n).
__global__ __launch_bounds__(DT) void k_defl_ft(int N, int n_prev, const double *__restrict__ W,
                                                double *__restrict__ Ft) {
  const int n = N - n_prev;
  for (int e = blockIdx.x * DT + threadIdx.x; e < n * N; e += gridDim.x * DT) {
    const int a = e / N, j = e % N;
    double s = 0.0;
    for (int k = 0; k < n_prev; ++k) s = fma(W[k * N + a], W[k * N + j], s);
    Ft[e] = (a == j ? 1.0 : 0.0) - s;
  }
}

__global__ __launch_bounds__(DT) void k_defl_gram(int N, int n_prev, const double *__restrict__ Ft,
                                                  double *__restrict__ C) {
  const int n = N - n_prev;
  for (int e = blockIdx.x * DT + threadIdx.x; e < n * n; e += gridDim.x * DT) {
    const int a = e / n, b = e % n;
    double s = 0.0;
    for (int j = 0; j < N; ++j) s = fma(Ft[a * N + j], Ft[b * N + j], s);
    C[e] = s;
  }
}

// One work-group: rank check, S = E D^(-1/2) E^T in LDS rows computed on the
// fly, G = S Ft, Wh = G with rows n .. N-1 zero.
__global__ __launch_bounds__(DT) void k_defl_basis(int N, int n_prev, const double *__restrict__ Ft,
                                                   const double *__restrict__ E, double rank_tol,
                                                   double *__restrict__ G, double *__restrict__ Wh,
                                                   int *flag) {
  const int n = N - n_prev;
  const double *lam = E + n * n;
  __shared__ double isq[OICA_MAX_N];
  __shared__ double srow[OICA_MAX_N];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) {
    double mn = lam[0], mx = lam[0];
    bool fin = true;
    for (int c = 0; c < n; ++c) {
      fin &= isfinite(lam[c]);
      mn = fmin(mn, lam[c]);
      mx = fmax(mx, lam[c]);
    }
    bad = (!fin || !(mx > 0.0) || !(mn > rank_tol * mx)) ? 1 : 0;
    if (bad) atomicOr(flag, 1);
  }
  __syncthreads();
  if (bad) return;
  for (int c = tid; c < n; c += DT) isq[c] = 1.0 / sqrt(lam[c]);
  __syncthreads();
  for (int a = 0; a < N; ++a) {
    if (a < n) {
      // row a of S: S[a][b] = sum_c E[a][c] isq[c] E[b][c] (column c = vector c)
      for (int b = tid; b < n; b += DT) {
        double s = 0.0;
        for (int c = 0; c < n; ++c) s = fma(E[a * n + c] * isq[c], E[b * n + c], s);
        srow[b] = s;
      }
      __syncthreads();
      for (int j = tid; j < N; j += DT) {
        double g = 0.0;
        for (int b = 0; b < n; ++b) g = fma(srow[b], Ft[b * N + j], g);
        G[a * N + j] = g;
        Wh[a * N + j] = g;
      }
      __syncthreads();
    } else {
      for (int j = tid; j < N; j += DT) Wh[a * N + j] = 0.0;
    }
  }
}

// w = B[p] G in FP64 (b_p held in FP32), orthogonalised against the earlier
// rows twice (classical Gram-Schmidt) and normalised: b_p G is orthogonal to
// them in exact arithmetic, but the rounding of F~ and of the inverse square
// root would otherwise compound from step to step.  One wave.
__global__ __launch_bounds__(64) void k_defl_append(int N, int n_prev, const double *__restrict__ G,
                                                    const float *__restrict__ B,
                                                    const int32_t *__restrict__ rep,
                                                    double *__restrict__ W) {
  const int n = N - n_prev;
  const int p = rep[0];
  const int lane = threadIdx.x;
  double w0 = 0.0, w1 = 0.0;
  const int j0 = lane, j1 = lane + 64;
  for (int a = 0; a < n; ++a) {
    const double b = (double)B[(size_t)p * n + a];
    if (j0 < N) w0 = fma(b, G[a * N + j0], w0);
    if (j1 < N) w1 = fma(b, G[a * N + j1], w1);
  }
  for (int pass = 0; pass < 2; ++pass) {
    // coefficients against every earlier row, then one subtraction
    double c0 = 0.0, c1 = 0.0;  // lanes hold rows k = lane and lane + 64
    for (int k = 0; k < n_prev; ++k) {
      double d = 0.0;
      if (j0 < N) d = fma(W[(size_t)k * N + j0], w0, d);
      if (j1 < N) d = fma(W[(size_t)k * N + j1], w1, d);
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) d += __shfl_xor(d, o);
      if (k == lane) c0 = d;
      if (k == lane + 64) c1 = d;
    }
    double s0 = 0.0, s1 = 0.0;
    for (int k = 0; k < n_prev; ++k) {
      const double ck = k < 64 ? __shfl(c0, k) : __shfl(c1, k - 64);
      if (j0 < N) s0 = fma(ck, W[(size_t)k * N + j0], s0);
      if (j1 < N) s1 = fma(ck, W[(size_t)k * N + j1], s1);
    }
    w0 -= s0;
    w1 -= s1;
  }
  double ss = w0 * w0 + w1 * w1;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) ss += __shfl_xor(ss, o);
  const double inv = 1.0 / sqrt(ss);
  if (j0 < N) W[(size_t)n_prev * N + j0] = w0 * inv;
  if (j1 < N) W[(size_t)n_prev * N + j1] = w1 * inv;
}

// Algorithm 1 takes the argmax over every run, converged or not: the
// candidates of the selection are all rows that did not degenerate.
__global__ __launch_bounds__(DT) void k_mark_runs(int K, uint8_t *__restrict__ status) {
  const int l = blockIdx.x * DT + threadIdx.x;
  if (l < K && status[l] == OICA_ROW_NOTCONV) status[l] = OICA_ROW_CONV;
}

// W[n_prev] = B[rep[0]] (an N-entry FP32 row, already projected and
// normalised by the fixed point), normalised again in FP64.  One wave.
__global__ __launch_bounds__(64) void k_append_row(int N, int n_prev, const float *__restrict__ B,
                                                   const int32_t *__restrict__ rep,
                                                   double *__restrict__ W) {
  const int p = rep[0];
  const int lane = threadIdx.x, j0 = lane, j1 = lane + 64;
  const double w0 = j0 < N ? (double)B[(size_t)p * N + j0] : 0.0;
  const double w1 = j1 < N ? (double)B[(size_t)p * N + j1] : 0.0;
  double ss = w0 * w0 + w1 * w1;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) ss += __shfl_xor(ss, o);
  const double inv = 1.0 / sqrt(ss);
  if (j0 < N) W[(size_t)n_prev * N + j0] = w0 * inv;
  if (j1 < N) W[(size_t)n_prev * N + j1] = w1 * inv;
}

}  // namespace

hipError_t launch_mark_runs(hipStream_t st, int K, uint8_t *status) {
  hipLaunchKernelGGL(k_mark_runs, dim3((K + DT - 1) / DT), dim3(DT), 0, st, K, status);
  return hipGetLastError();
}

hipError_t launch_append_row(hipStream_t st, int N, int n_prev, const float *B, const int32_t *rep,
                             double *W) {
  hipLaunchKernelGGL(k_append_row, dim3(1), dim3(64), 0, st, N, n_prev, B, rep, W);
  return hipGetLastError();
}

hipError_t launch_defl_gram(hipStream_t st, int N, int n_prev, const double *W, double *Ft,
                            double *C) {
  const int n = N - n_prev;
  hipLaunchKernelGGL(k_defl_ft, dim3((n * N + DT - 1) / DT), dim3(DT), 0, st, N, n_prev, W, Ft);
  hipLaunchKernelGGL(k_defl_gram, dim3((n * n + DT - 1) / DT), dim3(DT), 0, st, N, n_prev, Ft, C);
  return hipGetLastError();
}

hipError_t launch_defl_basis(hipStream_t st, int N, int n_prev, const double *Ft, const double *E,
                             double rank_tol, double *G, double *Wh, int *flag) {
  hipLaunchKernelGGL(k_defl_basis, dim3(1), dim3(DT), 0, st, N, n_prev, Ft, E, rank_tol, G, Wh,
                     flag);
  return hipGetLastError();
}

hipError_t launch_defl_append(hipStream_t st, int N, int n_prev, const double *G, const float *B,
                              const int32_t *rep, double *W) {
  hipLaunchKernelGGL(k_defl_append, dim3(1), dim3(64), 0, st, N, n_prev, G, B, rep, W);
  return hipGetLastError();
}

}  // namespace oica
