// The learned pruner: a 16 -> 64 -> 64 -> 1 network (ReLU, sigmoid) on the
// first eight passes of a start vector (kurtosis before the pass and log10 of
// the step), standardised with fixed statistics.  Forward passes use the FP16
// copy of the weights with FP32 arithmetic; training keeps FP32 master weights
// and Adam moments.  Gradients are summed per block of rows into partial
// vectors and the partials are added in block order, so a training step is
// deterministic.
//
// Parameter packing: W1 (64 x 16, row-major), b1 (64), W2 (64 x 64), b2 (64),
// w3 (64), b3 (1).
#include <hip/hip_fp16.h>
#include <math.h>

#include "oica_internal.h"

namespace oica {

constexpr int PH = 64;
constexpr int PF = 16;
constexpr int O_W1 = 0, O_B1 = O_W1 + PH * PF, O_W2 = O_B1 + PH, O_B2 = O_W2 + PH * PH,
              O_W3 = O_B2 + PH, O_B3 = O_W3 + PH, N_PAR = O_B3 + 1;
static_assert(N_PAR == OICA_PRUNER_PARAMS, "parameter count");
constexpr int GB = 128;  // rows per gradient block

struct FeatNorm {
  float mean[PF];
  float inv_std[PF];
};

__device__ inline void load_features(const float *__restrict__ traj, int stride, long long row,
                                     const FeatNorm &nm, float f[PF]) {
  const float *t = traj + (size_t)row * stride;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const float a = t[2 * s];
    const float d = t[2 * s + 1];
    f[2 * s] = (a - nm.mean[2 * s]) * nm.inv_std[2 * s];
    f[2 * s + 1] = (log10f(fmaxf(d, 1e-12f)) - nm.mean[2 * s + 1]) * nm.inv_std[2 * s + 1];
  }
}

__device__ inline void load_weights_lds(const __half *__restrict__ w16, float *sw) {
  for (int i = threadIdx.x; i < N_PAR; i += blockDim.x) sw[i] = __half2float(w16[i]);
  __syncthreads();
}

// logit of one row; h1 kept for the caller
__device__ inline float mlp_logit(const float *sw, const float f[PF], float h1[PH]) {
#pragma unroll
  for (int j = 0; j < PH; ++j) {
    float a = sw[O_B1 + j];
#pragma unroll
    for (int i = 0; i < PF; ++i) a = fmaf(sw[O_W1 + j * PF + i], f[i], a);
    h1[j] = fmaxf(a, 0.f);
  }
  float z = sw[O_B3];
  for (int j = 0; j < PH; ++j) {
    float a = sw[O_B2 + j];
#pragma unroll
    for (int k = 0; k < PH; ++k) a = fmaf(sw[O_W2 + j * PH + k], h1[k], a);
    z = fmaf(sw[O_W3 + j], fmaxf(a, 0.f), z);
  }
  return z;
}

__device__ inline float sigmoidf_stable(float z) {
  const float e = expf(-fabsf(z));
  return z >= 0.f ? 1.f / (1.f + e) : e / (1.f + e);
}

// Probability for rows 0..R-1 (rows given directly) or for the entries of a
// row list (list != nullptr, count from *count_dev).
__global__ __launch_bounds__(256) void k_mlp_predict(const __half *__restrict__ w16, FeatNorm nm,
                                                     const float *__restrict__ traj, long long R,
                                                     const int *__restrict__ list,
                                                     const int *__restrict__ count_dev,
                                                     float *__restrict__ prob) {
  __shared__ float sw[N_PAR];
  load_weights_lds(w16, sw);
  const long long n = count_dev ? *count_dev : R;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long row = list ? list[i] : i;
  float f[PF], h1[PH];
  load_features(traj, 16, row, nm, f);
  prob[list ? row : i] = sigmoidf_stable(mlp_logit(sw, f, h1));
}

// Pruning at a fixed pass: active rows whose probability is below theta are
// marked PRUNED (their row, iteration count and trajectory stay as they are)
// and dropped from the active list; the survivors go to `keep`.
__global__ __launch_bounds__(256) void k_prune(const __half *__restrict__ w16, FeatNorm nm,
                                               float theta, const float *__restrict__ traj,
                                               int traj_stride,
                                               const int *__restrict__ list, const int *count_dev,
                                               uint8_t *__restrict__ status, int *__restrict__ keep,
                                               int *keep_count, int *pruned_count) {
  __shared__ float sw[N_PAR];
  load_weights_lds(w16, sw);
  const int n = *count_dev;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool prune = false;
  int row = -1;
  if (i < n) {
    row = list[i];
    float f[PF], h1[PH];
    load_features(traj, traj_stride, row, nm, f);
    const float p = sigmoidf_stable(mlp_logit(sw, f, h1));
    prune = p < theta;
    if (prune) status[row] = OICA_ROW_PRUNED;
  }
  const unsigned long long pm = __ballot(prune);
  if (__lane_id() == 0 && pm) atomicAdd(pruned_count, __popcll(pm));
  wave_append(i < n && !prune, row, keep, keep_count);
}

__global__ void k_prune_commit(int *__restrict__ list, int *count_dev, const int *__restrict__ keep,
                               const int *keep_count) {
  const int n = *keep_count;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    list[i] = keep[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) *count_dev = n;
}

// Loss and gradient partials of one block of GB rows (one thread per row).
// Rows i = 0..R-1 of the step are source rows base + i, or, with perm.on,
// row_perm(perm, base + i).
__global__ __launch_bounds__(GB) void k_mlp_grad_block(const __half *__restrict__ w16, FeatNorm nm,
                                                       const float *__restrict__ traj,
                                                       const uint8_t *__restrict__ labels,
                                                       long long R, RowPerm perm,
                                                       long long base, float w_pos,
                                                       float *__restrict__ gpart,
                                                       double *__restrict__ lpart) {
  __shared__ float sw[N_PAR];
  __shared__ float sa[GB][PH + 1];   // per-row vectors, reused by phase
  __shared__ float sb[GB][PH + 1];
  __shared__ float sdz[GB];
  __shared__ double sloss[GB];
  load_weights_lds(w16, sw);
  const int t = threadIdx.x;
  const long long row = (long long)blockIdx.x * GB + t;
  const bool valid = row < R;
  float f[PF], h1[PH];
  float dz = 0.f;
  double lrow = 0.0;
  if (valid) {
    const long long src = perm.on ? row_perm(perm, base + row) : base + row;
    load_features(traj, 16, src, nm, f);
    const float z = mlp_logit(sw, f, h1);
    const float y = labels[src] ? 1.f : 0.f;
    const float s = sigmoidf_stable(z);
    dz = ((1.f - y) * s - w_pos * y * (1.f - s)) / (float)R;
    // softplus(-z) and softplus(z), stable
    const double zd = (double)z;
    const double spn = fmax(-zd, 0.0) + log1p(exp(-fabs(zd)));
    const double spp = fmax(zd, 0.0) + log1p(exp(-fabs(zd)));
    lrow = (double)w_pos * y * spn + (1.0 - y) * spp;
  } else {
#pragma unroll
    for (int i = 0; i < PF; ++i) f[i] = 0.f;
#pragma unroll
    for (int j = 0; j < PH; ++j) h1[j] = 0.f;
  }
  // recompute a2 row by row: h2 and dh2 = dz w3 [a2 > 0]
  float dh1[PH];
#pragma unroll
  for (int k = 0; k < PH; ++k) dh1[k] = 0.f;
  for (int j = 0; j < PH; ++j) {
    float a = sw[O_B2 + j];
#pragma unroll
    for (int k = 0; k < PH; ++k) a = fmaf(sw[O_W2 + j * PH + k], h1[k], a);
    const float h2 = fmaxf(a, 0.f);
    const float g2 = a > 0.f ? dz * sw[O_W3 + j] : 0.f;
    sa[t][j] = g2;       // dh2
    sb[t][j] = h2;       // h2
#pragma unroll
    for (int k = 0; k < PH; ++k) dh1[k] = fmaf(g2, sw[O_W2 + j * PH + k], dh1[k]);
  }
  sdz[t] = dz;
  sloss[t] = lrow;
  __syncthreads();
  float *gp = gpart + (size_t)blockIdx.x * N_PAR;
  // w3, b3, b2
  if (t < PH) {
    float g3 = 0.f, gb2 = 0.f;
    for (int r = 0; r < GB; ++r) {
      g3 = fmaf(sdz[r], sb[r][t], g3);
      gb2 += sa[r][t];
    }
    gp[O_W3 + t] = g3;
    gp[O_B2 + t] = gb2;
  }
  if (t == PH) {
    float g = 0.f;
    double l = 0.0;
    for (int r = 0; r < GB; ++r) {
      g += sdz[r];
      l += sloss[r];
    }
    gp[O_B3] = g;
    lpart[blockIdx.x] = l;
  }
  __syncthreads();
  // h1 into sb; W2 gradient = sum_r dh2[r] (x) h1[r]
#pragma unroll
  for (int k = 0; k < PH; ++k) sb[t][k] = h1[k];
  __syncthreads();
  for (int o = t; o < PH * PH; o += GB) {
    const int j = o / PH, k = o % PH;
    float g = 0.f;
    for (int r = 0; r < GB; ++r) g = fmaf(sa[r][j], sb[r][k], g);
    gp[O_W2 + o] = g;
  }
  __syncthreads();
  // dh1 (masked by a1 > 0, i.e. h1 > 0) into sa; features into sb
#pragma unroll
  for (int k = 0; k < PH; ++k) sa[t][k] = h1[k] > 0.f ? dh1[k] : 0.f;
#pragma unroll
  for (int i = 0; i < PF; ++i) sb[t][i] = f[i];
  __syncthreads();
  for (int o = t; o < PH * PF + PH; o += GB) {
    if (o < PH * PF) {
      const int k = o / PF, i = o % PF;
      float g = 0.f;
      for (int r = 0; r < GB; ++r) g = fmaf(sa[r][k], sb[r][i], g);
      gp[O_W1 + o] = g;
    } else {
      const int k = o - PH * PF;
      float g = 0.f;
      for (int r = 0; r < GB; ++r) g += sa[r][k];
      gp[O_B1 + k] = g;
    }
  }
}

// grad[i] = sum over blocks of the partials, in block order
__global__ void k_mlp_grad_reduce(int nblocks, const float *__restrict__ gpart,
                                  const double *__restrict__ lpart, float *__restrict__ grad,
                                  double *__restrict__ loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N_PAR) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += (double)gpart[(size_t)b * N_PAR + i];
    grad[i] = (float)s;
  }
  if (i == 0) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += lpart[b];
    *loss = s;
  }
}

__global__ void k_adam(float *__restrict__ w32, __half *__restrict__ w16, float *__restrict__ m,
                       float *__restrict__ v, const float *__restrict__ g, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N_PAR) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float w = w32[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w32[i] = w;
  w16[i] = __float2half(w);
}

__global__ void k_refresh_half(const float *__restrict__ w32, __half *__restrict__ w16) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N_PAR) w16[i] = __float2half(w32[i]);
}

// ---------------------------------------------------------------------------
static FeatNorm make_norm(const float *mean, const float *stdv) {
  FeatNorm nm;
  for (int i = 0; i < PF; ++i) {
    nm.mean[i] = mean[i];
    nm.inv_std[i] = 1.f / stdv[i];
  }
  return nm;
}

hipError_t pruner_alloc(PrunerState *p, const float *init_w, const float *mean, const float *stdv) {
  hipError_t e = hipMalloc(&p->w32, N_PAR * sizeof(float));
  if (e != hipSuccess) return e;
  e = hipMalloc(&p->w16, N_PAR * sizeof(__half));
  if (e != hipSuccess) return e;
  e = hipMalloc(&p->m, N_PAR * sizeof(float));
  if (e != hipSuccess) return e;
  e = hipMalloc(&p->v, N_PAR * sizeof(float));
  if (e != hipSuccess) return e;
  e = hipMemcpy(p->w32, init_w, N_PAR * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  e = hipMemset(p->m, 0, N_PAR * sizeof(float));
  if (e != hipSuccess) return e;
  e = hipMemset(p->v, 0, N_PAR * sizeof(float));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_refresh_half, dim3((N_PAR + 255) / 256), dim3(256), 0, 0, p->w32,
                     (__half *)p->w16);
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return e;
  for (int i = 0; i < PF; ++i) {
    p->mean[i] = mean[i];
    p->stdv[i] = stdv[i];
  }
  p->theta = 0.f;
  p->step = 0;
  return hipSuccess;
}

void pruner_free(PrunerState *p) {
  if (p->w32) (void)hipFree(p->w32);
  if (p->w16) (void)hipFree(p->w16);
  if (p->m) (void)hipFree(p->m);
  if (p->v) (void)hipFree(p->v);
}

hipError_t launch_pruner_predict(hipStream_t st, const PrunerState *p, const float *traj, long long R,
                                 const int *list, const int *count_dev, float *prob) {
  const long long n = R;
  hipLaunchKernelGGL(k_mlp_predict, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     (const __half *)p->w16, make_norm(p->mean, p->stdv), traj, R, list, count_dev,
                     prob);
  return hipGetLastError();
}

size_t pruner_grad_workspace_bytes(long long R) {
  const long long nb = (R + GB - 1) / GB;
  return (size_t)nb * N_PAR * sizeof(float) + (size_t)nb * sizeof(double) + 1024;
}

hipError_t launch_pruner_grad(hipStream_t st, const PrunerState *p, const float *traj,
                              const uint8_t *labels, long long R, const RowPerm &perm,
                              long long base, float w_pos, void *ws, float *grad,
                              double *loss_dev) {
  const int nb = (int)((R + GB - 1) / GB);
  float *gpart = (float *)ws;
  double *lpart = (double *)((char *)ws + (((size_t)nb * N_PAR * sizeof(float) + 255) & ~(size_t)255));
  hipLaunchKernelGGL(k_mlp_grad_block, dim3(nb), dim3(GB), 0, st, (const __half *)p->w16,
                     make_norm(p->mean, p->stdv), traj, labels, R, perm, base, w_pos, gpart,
                     lpart);
  hipLaunchKernelGGL(k_mlp_grad_reduce, dim3((N_PAR + 255) / 256), dim3(256), 0, st, nb, gpart,
                     lpart, grad, loss_dev);
  return hipGetLastError();
}

hipError_t launch_pruner_adam(hipStream_t st, PrunerState *p, const float *grad, float lr) {
  p->step += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)p->step), c2 = 1.f - powf(b2, (float)p->step);
  hipLaunchKernelGGL(k_adam, dim3((N_PAR + 255) / 256), dim3(256), 0, st, p->w32, (__half *)p->w16,
                     p->m, p->v, grad, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_prune(hipStream_t st, const PrunerState *p, const float *traj, int traj_stride,
                        int *list, int *count_dev, int kmax, uint8_t *status, int *keep,
                        int *keep_count, int *pruned_count) {
  hipLaunchKernelGGL(k_prune, dim3((kmax + 255) / 256), dim3(256), 0, st, (const __half *)p->w16,
                     make_norm(p->mean, p->stdv), p->theta, traj, traj_stride, list, count_dev,
                     status, keep, keep_count, pruned_count);
  hipLaunchKernelGGL(k_prune_commit, dim3((kmax + 255) / 256 < 1024 ? (kmax + 255) / 256 : 1024),
                     dim3(256), 0, st, list, count_dev, keep, keep_count);
  return hipGetLastError();
}


// Number of non-zero labels (one 64-bit counter, zeroed by the caller).
__global__ __launch_bounds__(256) void k_count_pos(const uint8_t *__restrict__ labels, long long R,
                                                   unsigned long long *__restrict__ count) {
  __shared__ unsigned int part[4];
  unsigned int c = 0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < R;
       i += (long long)gridDim.x * 256)
    c += labels[i] != 0;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o);
  if (threadIdx.x % 64 == 0) part[threadIdx.x / 64] = c;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicAdd(count, (unsigned long long)(part[0] + part[1] + part[2] + part[3]));
}

hipError_t launch_count_pos(hipStream_t st, const uint8_t *labels, long long R,
                            unsigned long long *count_dev) {
  const long long want = (R + 255) / 256;
  const int grid = (int)(want < 1024 ? want : 1024);
  hipLaunchKernelGGL(k_count_pos, dim3(grid), dim3(256), 0, st, labels, R, count_dev);
  return hipGetLastError();
}

}  // namespace oica
