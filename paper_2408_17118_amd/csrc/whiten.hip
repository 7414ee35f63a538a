// PCA whitening on gfx950, all in FP64 (the paper whitens the observations
// before the method runs; Theorem 1's constraints are zero sample mean and
// identity sample covariance, the covariance normalised by the sample count).
//
//   k_mean_part / k_mean_final   mu = X 1 / T          (two-level, fixed order)
//   k_cov_part  / k_cov_final    C = Xc Xc^T / T       (FP64 MFMA, split over T, fixed order)
//   k_jacobi_values / _vectors   C = E D E^T            (cyclic Jacobi: eigenvalues in one
//                                                        work-group with A in LDS, then E
//                                                        from the logged rotations)
//   k_canon                      descending order, sign rule, rank check,
//                                Wh = D^(-1/2) E^T
//   k_apply<BIG>                 Xw = Wh (X - mu)       (FP64 MFMA; FP32 / BF16 out)
// The mean is HBM-bound; the covariance and apply passes are FP64 contractions over
// the samples (N^2 T multiply-adds each); the Jacobi solve is O(N^3) on N <= 128.
// Every kernel takes a table of problems, so many datasets share each launch
// (a single problem is passed by value); a problem's arithmetic does not
// depend on the others.
#include "oica_internal.h"

#include <math.h>

#include <algorithm>
#include <vector>

namespace oica {

constexpr int NMAX = OICA_MAX_N;
constexpr int MIN_CHUNK = 256;    // fewest samples per work-group in the reduction passes
constexpr int MAX_CHUNKS = 1024;  // mean pass
constexpr int MAX_COV_CHUNKS = 512;

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <typename TIN>
__device__ inline double ld(const TIN *p, size_t i) {
  return (double)p[i];
}

static inline int n_chunks(int64_t T, int cap = MAX_CHUNKS) {
  int64_t c = T / MIN_CHUNK;
  if (c > cap) c = cap;
  if (c < 1) c = 1;
  return (int)c;
}
static inline int n_cov_chunks(int N, int64_t T) {
  return n_chunks(T, N <= 64 ? MAX_COV_CHUNKS : MAX_COV_CHUNKS / 2);
}

// One problem of the statistics, canon and apply kernels.  Many problems run
// in one launch from a device table; a single problem is passed by value.
struct WJob {
  const void *X;
  int f64;              // raw data FP64 (else FP32)
  int N;
  long long T;
  long long ld;         // row stride of X in elements
  int ch, cch;          // sample chunks of the mean and covariance passes
  double *mpart, *cpart;
  double *mean, *C, *E, *Wh, *eig;
  int *flags;
  float *o32, *o32b;    // FP32 outputs (either may be null)
  uint16_t *obf;        // BF16 output (may be null)
  int n_out;            // apply: output rows (the first n_out rows of Wh); 0 = N
};

// Launch-wide ranges: problem d owns work-groups (or waves) [start[d],
// start[d + 1]) of a launch.  start == nullptr: one problem, passed by value.
enum { W_MEAN = 0, W_MEANF, W_COV4, W_COV8, W_COVF, W_APPLY4, W_APPLY8, W_KINDS };

__device__ inline int job_of(const int *start, int D, int b) {
  int lo = 0, hi = D - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Partial row sums over a sample chunk; one wave per row (strided), lanes over samples.
template <typename TIN>
__device__ void mean_part_body(const WJob &j, int c) {
  const TIN *X = (const TIN *)j.X;
  const int N = j.N;
  const long long T = j.T;
  const long long t0 = (long long)c * T / j.ch, t1 = (long long)(c + 1) * T / j.ch;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  // a lane's samples m, m + 64, ... are loaded U at a time ahead of their
  // (in-order) adds, through a buffer resource over the row's chunk: a load
  // past the chunk's end reads zero without a memory access and adds +0.0,
  // which leaves the sum as it is (it starts at +0.0, so it is never -0.0);
  // each load takes a 32-bit offset register instead of a 64-bit address
  constexpr int U = 8;
  constexpr int ES = (int)sizeof(TIN);
  // a chunk holds about 256 samples of a row, or T / 1024 once T > 2.6e5
  // (n_chunks): far below 2^31 bytes for any T whose N x T input fits the device
  const long long len = t1 - t0;
  for (int n = wave; n < N; n += 4) {
    double s = 0.0;
    bool bad = false;
    // the chunk's base and size are uniform; readfirstlane keeps the
    // resource in scalar registers
    const unsigned long long cb = (unsigned long long)(size_t)(X + (size_t)n * (size_t)j.ld + t0);
    const unsigned int blo = __builtin_amdgcn_readfirstlane((unsigned int)cb);
    const unsigned int bhi = __builtin_amdgcn_readfirstlane((unsigned int)(cb >> 32));
    const int nrec = __builtin_amdgcn_readfirstlane((int)(len * ES));
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(size_t)(((unsigned long long)bhi << 32) | blo), (short)0, nrec, 0x00020000);
    for (long long m = lane; m < len; m += 64 * U) {
      const int vo = (int)m * ES;
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if constexpr (ES == 8)
          v[u] = __builtin_bit_cast(
              double, __builtin_amdgcn_raw_buffer_load_b64(rsrc, vo + 64 * u * ES, 0, 0));
        else
          v[u] = (double)__builtin_bit_cast(
              float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, vo + 64 * u * ES, 0, 0));
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        bad |= !isfinite(v[u]);
        s += v[u];
      }
    }
    s = wsum(s);
    if (bad) atomicOr(j.flags, 1);
    if (lane == 0) j.mpart[(size_t)c * N + n] = s;
  }
}

__global__ __launch_bounds__(256) void k_mean_part(const WJob *__restrict__ jobs, WJob one,
                                                   const int *__restrict__ start, int D) {
  int c = blockIdx.x;
  const int d = start ? job_of(start, D, c) : 0;
  if (start) c -= start[d];
  const WJob j = start ? jobs[d] : one;
  if (j.f64) mean_part_body<double>(j, c);
  else mean_part_body<float>(j, c);
}

// One wave per (problem, row): lanes take chunks lane, lane + 64, ...; fixed
// shuffle tree.
__global__ void k_mean_final(const WJob *__restrict__ jobs, WJob one, const int *__restrict__ start,
                             int D, int total) {
  int w = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (w >= total) return;
  const int d = start ? job_of(start, D, w) : 0;
  if (start) w -= start[d];
  const WJob j = start ? jobs[d] : one;
  const int n = w;
  double s = 0.0;
  for (int c = lane; c < j.ch; c += 64) s += j.mpart[(size_t)c * j.N + n];
  s = wsum(s);
  if (lane == 0) j.mean[n] = s / (double)j.T;
}

// Partial centred second moments over a chunk, on FP64 MFMA
// (v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// result register r holds D[l / 16 + 4 r][l % 16]).  At one step the operand
// of row block b is the same register on the A and the B side (lane l: row
// 16 b + l % 16 of X - mean at sample s + l / 16), so block (bi, bj) of the
// chunk's X_c X_c^T accumulates mfma(v[bi], v[bj]); only blocks bi <= bj are
// formed (the final pass reads the upper triangle).  Wave w takes the 16-sample
// groups w, w + 4, ... of the chunk (step k of a group: samples g + 4 k + l / 16),
// its loads issued one group ahead, and the four waves' sums are added in
// LDS in wave order, so a chunk still yields one partial, in a fixed order.
// Rows past N are read as row N - 1: they only reach entries that are not
// stored.  Samples past the chunk are zero.
typedef double cov_f64x4 __attribute__((ext_vector_type(4)));
constexpr int WAVES_WH = 4;  // waves of a 256-thread work-group
static size_t cov_lds_bytes(int N) {  // the sample-split form's exchange (N <= 64)
  const int nrb = (N + 15) / 16;
  return nrb > 4 ? 0 : (size_t)(nrb * (nrb + 1) / 2) * 4 * 64 * sizeof(double);
}
template <int NRB, typename TIN>
__device__ __forceinline__ void cov_part_body(const WJob &j, int c, double *lds) {
  typedef __attribute__((address_space(1))) const TIN gin;
  constexpr int NPAIR = NRB * (NRB + 1) / 2;
  const int N = j.N;
  const long long T = j.T;
  const long long t0 = (long long)c * T / j.cch, t1 = (long long)(c + 1) * T / j.cch;
  gin *X = (gin *)j.X;
  const long long ldx = j.ld;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int rr = lane % 16, q = lane / 16;
  double mu[NRB];
  int row[NRB];
#pragma unroll
  for (int b = 0; b < NRB; ++b) {
    row[b] = b * 16 + rr < N ? b * 16 + rr : N - 1;
    mu[b] = j.mean[row[b]];
  }
  auto load = [&](long long m, int b) -> double {
    return (double)X[(size_t)row[b] * (size_t)ldx + (size_t)(m < t1 ? m : t1 - 1)];
  };
  cov_f64x4 acc[NPAIR];
#pragma unroll
  for (int p = 0; p < NPAIR; ++p) acc[p] = cov_f64x4{0.0, 0.0, 0.0, 0.0};
  // nxt[b][k]: step k of the wave's current group, replaced by the same step
  // of its next group as soon as it is used
  double nxt[NRB][4];
  long long g = t0 + 16 * wave;
  if (g < t1) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int b = 0; b < NRB; ++b) nxt[b][k] = load(g + 4 * k + q, b);
  }
  for (; g < t1; g += 64) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const long long m = g + 4 * k + q;
      double v[NRB];
#pragma unroll
      for (int b = 0; b < NRB; ++b) {
        v[b] = m < t1 ? nxt[b][k] - mu[b] : 0.0;
        nxt[b][k] = load(m + 64, b);
      }
      int p = 0;
#pragma unroll
      for (int bi = 0; bi < NRB; ++bi)
#pragma unroll
        for (int bj = bi; bj < NRB; ++bj, ++p)
          acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[bi], v[bj], acc[p], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // waves 1..3 hand their sums to wave 0 in turn
#pragma unroll 1
  for (int w = 1; w < WAVES_WH; ++w) {
    __syncthreads();
    if (wave == w) {
#pragma unroll
      for (int p = 0; p < NPAIR; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) lds[(p * 4 + r) * 64 + lane] = acc[p][r];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int p = 0; p < NPAIR; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[p][r] += lds[(p * 4 + r) * 64 + lane];
    }
  }
  if (wave == 0) {
    int p = 0;
#pragma unroll
    for (int bi = 0; bi < NRB; ++bi)
#pragma unroll
      for (int bj = bi; bj < NRB; ++bj, ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = bi * 16 + q + 4 * r, jj = bj * 16 + rr;
          if (i < N && jj < N) j.cpart[((size_t)c * N + i) * N + jj] = acc[p][r];
        }
  }
}

// N > 64 (5 to 8 row blocks, up to 36 block pairs): the four waves split the
// block pairs instead of the samples (wave w forms the pairs p = w mod 4 of
// the bi <= bj enumeration over every sample of the chunk, at most 9
// accumulators) and each writes its own entries.  The chunk passes through
// LDS in tiles of COV_TS samples, stored as X - mean in FP64 (rows past N and
// samples past the chunk as zero), in two buffers: the work-group's loads of
// tile i + 1 (4 consecutive samples of a row per thread, so 8 threads read one
// row's 32 samples) are issued before the MFMAs of tile i and written to the
// other buffer after them, with one barrier per tile, so no load is still in
// flight at the loop's back-edge (a prefetch carried in registers across it
// was waited for at every iteration).  Step s of a tile takes samples
// tb + 4 s + (0..3), the order of a walk over the chunk in steps of four.
constexpr int COV_TS = 32;   // samples per tile
// LDS row stride in doubles, 2 mod 32: the 16 rows x 4 samples of an operand
// read fall in distinct banks
constexpr int COV_LDR = COV_TS + 2;
static size_t cov_tile_lds_bytes(int N) {
  const int nrb = (N + 15) / 16;
  return (size_t)2 * 16 * nrb * COV_LDR * sizeof(double);
}
template <typename TIN> struct Vec4;
template <> struct Vec4<float> {
  // dword alignment is all a multi-dword global load needs
  typedef float type __attribute__((ext_vector_type(4), aligned(4)));
};
template <> struct Vec4<double> {
  typedef double type __attribute__((ext_vector_type(4), aligned(8)));
};
template <int NRB, int PH, typename TIN>
__device__ __forceinline__ void cov_pairs_body(const WJob &j, int c, double *lds) {
  typedef __attribute__((address_space(1))) const TIN gin;
  typedef __attribute__((address_space(1))) const typename Vec4<TIN>::type gin4;
  constexpr int NP = 16 * NRB;
  constexpr int NPAIR = NRB * (NRB + 1) / 2;
  constexpr int NMINE = (NPAIR - PH + 3) / 4;
  constexpr int SPT = COV_TS / 4;       // threads per row of a tile
  constexpr int RSTEP = 256 / SPT;      // rows staged per pass of the work-group
  constexpr int RPT = (NP + RSTEP - 1) / RSTEP;
  const int N = j.N;
  const long long T = j.T;
  const long long t0 = (long long)c * T / j.cch, t1 = (long long)(c + 1) * T / j.cch;
  gin *X = (gin *)j.X;
  const long long ldx = j.ld;
  const int tid = threadIdx.x, lane = tid % 64;
  const int rr = lane % 16, q = lane / 16;
  const int sr = tid / SPT, sj = tid % SPT;  // staging: rows sr + RSTEP i, samples 4 sj .. 4 sj + 3
  double smu[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int row = sr + RSTEP * i;
    smu[i] = row < N ? j.mean[row] : 0.0;
  }
  // rows past N load row N - 1 (stored as zero)
  gin *srow[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int row = sr + RSTEP * i;
    srow[i] = X + (size_t)(row < N ? row : N - 1) * (size_t)ldx;
  }
  TIN reg[RPT][4];
  // a whole tile inside the chunk: one vector load per row, no branch
  auto load_full = [&](long long tb) {
    const size_t m = (size_t)(tb + 4 * sj);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const typename Vec4<TIN>::type v = *(gin4 *)(srow[i] + m);
#pragma unroll
      for (int e = 0; e < 4; ++e) reg[i][e] = v[e];
    }
  };
  // the chunk's last, partial tile: element loads at indices clamped into it
  auto load_tail = [&](long long tb) {
    const long long m = tb + 4 * sj;
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) reg[i][e] = srow[i][m + e < t1 ? m + e : t1 - 1];
  };
  auto store_tile = [&](double *buf, long long tb) {
    const long long m = tb + 4 * sj;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int row = sr + RSTEP * i;
      if (RSTEP * i + RSTEP <= NP || row < NP) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          buf[row * COV_LDR + 4 * sj + e] =
              row < N && m + e < t1 ? (double)reg[i][e] - smu[i] : 0.0;
      }
    }
  };
  cov_f64x4 acc[NMINE];
#pragma unroll
  for (int p = 0; p < NMINE; ++p) acc[p] = cov_f64x4{0.0, 0.0, 0.0, 0.0};
  double *buf0 = lds, *buf1 = lds + NP * COV_LDR;
  // nfull whole tiles, then at most one partial tile (work-group uniform)
  const long long nfull = (t1 - t0) / COV_TS;
  const long long ntiles = nfull + ((t1 - t0) % COV_TS != 0);
  if (ntiles > 0) {
    if (nfull > 0) load_full(t0);
    else load_tail(t0);
    store_tile(buf0, t0);
  }
  __syncthreads();
  for (long long it = 0; it < ntiles; ++it) {
    const long long tb = t0 + it * COV_TS;
    const double *cur = (it & 1) ? buf1 : buf0;
    double *nxt = (it & 1) ? buf0 : buf1;
    if (it + 1 < nfull) load_full(tb + COV_TS);
    else if (it + 1 < ntiles) load_tail(tb + COV_TS);
#pragma unroll
    for (int s = 0; s < COV_TS / 4; ++s) {
      double v[NRB];
#pragma unroll
      for (int b = 0; b < NRB; ++b) v[b] = cur[(16 * b + rr) * COV_LDR + 4 * s + q];
      int p = 0, mine = 0;
#pragma unroll
      for (int bi = 0; bi < NRB; ++bi)
#pragma unroll
        for (int bj = bi; bj < NRB; ++bj, ++p)
          if (p % 4 == PH) {
            acc[mine] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[bi], v[bj], acc[mine], 0, 0, 0);
            ++mine;
          }
    }
    if (it + 1 < ntiles) store_tile(nxt, tb + COV_TS);
    __syncthreads();
  }
  int p = 0, mine = 0;
#pragma unroll
  for (int bi = 0; bi < NRB; ++bi)
#pragma unroll
    for (int bj = bi; bj < NRB; ++bj, ++p)
      if (p % 4 == PH) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = bi * 16 + q + 4 * r, jj = bj * 16 + rr;
          if (i < N && jj < N) j.cpart[((size_t)c * N + i) * N + jj] = acc[mine][r];
        }
        ++mine;
      }
}

template <int NRB, typename TIN>
__device__ __forceinline__ void cov_pairs(const WJob &j, int c, double *lds) {
  switch (threadIdx.x / 64) {
    case 0: cov_pairs_body<NRB, 0, TIN>(j, c, lds); break;
    case 1: cov_pairs_body<NRB, 1, TIN>(j, c, lds); break;
    case 2: cov_pairs_body<NRB, 2, TIN>(j, c, lds); break;
    default: cov_pairs_body<NRB, 3, TIN>(j, c, lds); break;
  }
}

// RB = 4: problems with N <= 64 (1 to 4 row blocks, the waves split the
// samples); RB = 8: N > 64 (5 to 8, the waves split the block pairs); one
// launch per class, each kernel with the registers of its own sizes.
template <int RB, typename TIN>
__device__ __forceinline__ void cov_dispatch(const WJob &j, int c, double *lds) {
  const int nrb = (j.N + 15) / 16;
  if constexpr (RB == 8) {
    switch (nrb) {
      case 5: cov_pairs<5, TIN>(j, c, lds); break;
      case 6: cov_pairs<6, TIN>(j, c, lds); break;
      case 7: cov_pairs<7, TIN>(j, c, lds); break;
      default: cov_pairs<8, TIN>(j, c, lds); break;
    }
  } else {
    switch (nrb) {
      case 1: cov_part_body<1, TIN>(j, c, lds); break;
      case 2: cov_part_body<2, TIN>(j, c, lds); break;
      case 3: cov_part_body<3, TIN>(j, c, lds); break;
      default: cov_part_body<4, TIN>(j, c, lds); break;
    }
  }
}

// RB = 8: two work-groups per CU (the tile buffers take 68 KiB of LDS each)
template <int RB>
__global__ __launch_bounds__(256, RB == 8 ? 2 : 1) void k_cov_part(const WJob *__restrict__ jobs,
                                                                   WJob one,
                                                                   const int *__restrict__ start,
                                                                   int D) {
  extern __shared__ double cov_lds[];
  int c = blockIdx.x;
  const int d = start ? job_of(start, D, c) : 0;
  if (start) c -= start[d];
  const WJob j = start ? jobs[d] : one;
  if (j.f64) cov_dispatch<RB, double>(j, c, cov_lds);
  else cov_dispatch<RB, float>(j, c, cov_lds);
}

// Dynamic LDS of k_cov_part<RB> for problems up to n_max features.
template <int RB>
static size_t cov_prepare(int n_max) {
  const size_t lds = RB == 8 ? cov_tile_lds_bytes(n_max) : cov_lds_bytes(n_max);
  (void)hipFuncSetAttribute((const void *)k_cov_part<RB>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)hipGetLastError();
  return lds;
}

// One wave per (problem, matrix element) (lanes over chunks, fixed shuffle
// tree); the upper-triangle partial is used for both (i, j) and (j, i), so C
// is exactly symmetric.
__global__ void k_cov_final(const WJob *__restrict__ jobs, WJob one, const int *__restrict__ start,
                            int D, int total) {
  int w = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (w >= total) return;
  const int d = start ? job_of(start, D, w) : 0;
  if (start) w -= start[d];
  const WJob j = start ? jobs[d] : one;
  const int N = j.N;
  const int i = w / N, jj = w % N;
  const int a = i < jj ? i : jj, b = i < jj ? jj : i;
  double s = 0.0;
  for (int c = lane; c < j.cch; c += 64) s += j.cpart[((size_t)c * N + a) * N + b];
  s = wsum(s);
  if (lane == 0) j.C[w] = s / (double)j.T;
}

// Cyclic Jacobi with round-robin pairing: each round applies N/2 disjoint
// rotations at once, a sweep is N-1 rounds (N rounded up to even; the padding
// index is never rotated).  A rotation is applied only while |a_pq| exceeds
// both N eps sqrt(|a_pp a_qq|) and eps max_i |a_ii| (the rounding floor that
// rotations themselves leave in every element, the absolute accuracy a dense
// symmetric eigensolver reaches); a sweep without rotations ends the solve.
//
// Two kernels:
//   k_jacobi_values   one work-group per matrix; the upper triangle of A in
//                     LDS.  Rotations of one round act on disjoint index pairs,
//                     so A <- J^T A J splits into independent 2 x 2 blocks
//                     (pair k rows, pair l columns): each block is updated in
//                     one step from the round's (c, s), and only blocks with
//                     k <= l are touched (A stays symmetric).  Two barriers per
//                     round.  Every round's rotations are appended to a log.
//   k_jacobi_vectors  E = product of the logged rotations.  Rows of E evolve
//                     independently (E <- E J acts on columns p, q of each row),
//                     so work-groups own row blocks of E in LDS and replay the
//                     log round by round.
// Several matrices (the batched whitening) run in one launch, one job each.
constexpr int JAC_THREADS = 1024;
// 2 x 2 blocks per thread and round, at most: npair (npair / 2 + 1) blocks
constexpr int JAC_UNITS = ((NMAX / 2) * (NMAX / 4 + 1) + JAC_THREADS - 1) / JAC_THREADS;
constexpr int JAC_MAX_SWEEPS = 30;
constexpr int JAC_FIRST = JAC_UNITS < 2 ? JAC_UNITS : 2;  // units of a round's first batch
template <int V> struct JacC { static constexpr int value = V; };
static int g_jacobi_sweeps = JAC_MAX_SWEEPS;
int jacobi_max_sweeps() { return g_jacobi_sweeps; }
void set_jacobi_max_sweeps(int s) { g_jacobi_sweeps = s; }
constexpr double JAC_EPS = 2.220446049250313e-16;
constexpr int JV_ROWS = 8;       // rows of E per work-group, at most (two per wave)
constexpr int JV_THREADS = 256;
constexpr int JV_CHUNK = 32;     // logged rounds staged in LDS at a time
constexpr int JAC_STAGE = 8;     // loads in flight per thread while staging C
// log entries per thread and staged chunk
constexpr int JV_STAGE = JV_CHUNK * (NMAX / 2) / JV_THREADS;
static_assert(JV_STAGE * JV_THREADS == JV_CHUNK * (NMAX / 2), "a chunk splits evenly");
typedef double jac_dv2 __attribute__((ext_vector_type(2)));  // the log's (c, s)
typedef __attribute__((address_space(1))) double jac_gd;
typedef __attribute__((address_space(1))) jac_dv2 jac_gd2;
typedef __attribute__((address_space(1))) int jac_gi;

size_t jacobi_log_entries(int N) {
  const int ne = N + (N & 1);
  return (size_t)JAC_MAX_SWEEPS * (size_t)(ne > 1 ? ne - 1 : 1) * (size_t)(ne / 2 > 0 ? ne / 2 : 1);
}

// Element (i, j) of the upper triangle.  Indices and LD are below 2^24, so
// the full-rate 24-bit multiply gives the row offset (a 32-bit multiply
// issues at a quarter of the rate, and the solve is bound by its issue rate).
__device__ inline int jac_sym(int i, int j, int LD) {
  return i <= j ? (int)__umul24(i, LD) + j : (int)__umul24(j, LD) + i;
}

// Row stride of A in LDS: the smallest LD >= N + 1 with LD = 2 (mod 4).  In a
// round, neighbouring lanes' elements often differ by one row and one column
// in opposite directions (LD - 1 doubles) or the same one (LD + 1); both are
// odd, so those lanes fall in distinct banks, and a pure row step (LD) costs
// at most a 2-way conflict.  (With LD = N + 1 = 129, LD - 1 = 128 doubles put
// whole half-waves on one bank.)  Non-decreasing in N.
__host__ __device__ constexpr int jac_ld(int N) { return N + 1 + ((2 - (N + 1) % 4) + 4) % 4; }

__global__ __launch_bounds__(JAC_THREADS) void k_jacobi_values(const JacJob *__restrict__ jobs,
                                                               JacJob one) {
  extern __shared__ double jac_smem[];
  __shared__ double rc[NMAX / 2], rs[NMAX / 2];
  __shared__ int rp[NMAX / 2], rq[NMAX / 2];
  __shared__ int rotated;
  __shared__ double dscale;
  const JacJob jb = jobs ? jobs[blockIdx.x] : one;
  // global (not generic) pointers: a generic store counts against the LDS
  // counter too, so the LDS wait before each round's barrier would also wait
  // for the round's log stores to reach memory
  const jac_gd *Cg = (const jac_gd *)jb.C;
  jac_gd2 *rot_log = (jac_gd2 *)jb.rot;
  jac_gi *pq_log = (jac_gi *)jb.pq;
  const int N = jb.N;
  const int LD = jac_ld(N);
  double *a = jac_smem;
  const int tid = threadIdx.x;
  const double thr = JAC_EPS * (double)N;
  // the upper triangle into LDS, JAC_STAGE loads in flight per thread
  const int NN = N * N;
  for (int e0 = 0; e0 < NN; e0 += JAC_STAGE * JAC_THREADS) {
    double v[JAC_STAGE];
#pragma unroll
    for (int k = 0; k < JAC_STAGE; ++k) {
      const int e = e0 + k * JAC_THREADS + tid;
      v[k] = Cg[e < NN ? e : NN - 1];
    }
#pragma unroll
    for (int k = 0; k < JAC_STAGE; ++k) {
      const int e = e0 + k * JAC_THREADS + tid;
      const int i = e / N, j = e - i * N;
      if (e < NN && i <= j) a[i * LD + j] = v[k];
    }
  }
  __syncthreads();
  // the largest |C_ii|, over the diagonal now in LDS (one wave; the maximum
  // does not depend on the order it is taken in)
  if (tid < 64) {
    double m = 0.0;
    for (int i = tid; i < N; i += 64) m = fmax(m, fabs(a[i * LD + i]));
    for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if (tid == 0) dscale = JAC_EPS * m;
  }
  __syncthreads();
  const int ne = N + (N & 1);
  const int npair = ne / 2;
  const int H = npair / 2;
  const int units = npair * (H + 1);
  int sweep = 0;
  bool still = false;  // the last sweep run rotated
  const int limit = jb.max_sweeps;
  for (; sweep < limit && ne > 1; ++sweep) {
    // A sweep rotates iff some pair passes the rotation test on entry (until
    // a rotation, every round tests pairs of the entry matrix), so a sweep
    // that would rotate nothing is not run: every pair is tested first.
    if (tid == 0) rotated = 0;
    __syncthreads();
    {
      bool any = false;  // wave per row p, lanes over q > p
      for (int p = tid / 64; p < N; p += JAC_THREADS / 64) {
        const double app = a[p * LD + p];
        for (int q = p + 1 + tid % 64; q < N; q += 64) {
          const double apq = a[p * LD + q], aqq = a[q * LD + q];
          any = any || (fabs(apq) > dscale && apq * apq > thr * thr * fabs(app * aqq));
        }
      }
      if (any) rotated = 1;
    }
    __syncthreads();
    if (rotated == 0) break;
    __syncthreads();
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < ne - 1; ++r) {
      if (tid < npair) {
        int p, q;
        if (tid == 0) {
          p = ne - 1;
          q = r;
        } else {
          p = r + tid;
          if (p >= ne - 1) p -= ne - 1;
          q = r - tid;
          if (q < 0) q += ne - 1;
        }
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double c = 1.0, sn = 0.0;
        if (q < N) {
          const double apq = a[__umul24(p, LD) + q];
          const double app = a[__umul24(p, LD) + p], aqq = a[__umul24(q, LD) + q];
          // both comparisons taken (no short circuit), so that the three
          // reads above go out together
          if ((fabs(apq) > dscale) & (apq * apq > thr * thr * fabs(app * aqq))) {
            // With x = a_qq - a_pp, y = 2 a_pq (cot 2phi = x / y) and r = |(x, y)|,
            // the smaller rotation angle has t = tan phi = sgn(xy) |y| / (|x| + r),
            // so cos phi = (|x| + r) / w and sin phi = sgn(xy) |y| / w with
            // w = sqrt(2 r (r + |x|)): two square roots and one division.
            const double x = aqq - app, y = 2.0 * apq;
            const double r = sqrt(x * x + y * y);
            const double u = r + fabs(x);
            const double inv = 1.0 / sqrt(2.0 * r * u);
            c = u * inv;
            sn = ((x >= 0.0) == (y >= 0.0) ? 1.0 : -1.0) * fabs(y) * inv;
            rotated = 1;
          }
        }
        rc[tid] = c;
        rs[tid] = sn;
        rp[tid] = p;
        rq[tid] = q < N ? q : -1;
        const size_t li = ((size_t)sweep * (ne - 1) + r) * npair + tid;
        rot_log[li] = jac_dv2{c, sn};
        pq_log[li] = p | ((q < N ? q : 0xFFFF) << 16);
      }
      __syncthreads();
      // block (k, l), l = k + m (mod npair): every unordered pair of index
      // pairs once (m = H twice when npair is even: keep k < H).  The blocks
      // of a round hold disjoint elements, so they may be loaded and stored
      // in any order: a thread loads units [J0, J1) of its blocks before it
      // stores them (one LDS latency per batch, not one per block), first
      // units 0 and 1, then the rest (the first wave's only), and keeps each
      // unit's rotations and element offsets from its loads for its stores,
      // within the register budget of 1024 threads.
      auto blocks = [&](auto j0c, auto j1c) {
        constexpr int J0 = decltype(j0c)::value, J1 = decltype(j1c)::value;
        constexpr int NU = J1 - J0;
        double b[NU][4], ck[NU], sk[NU], cl[NU], sl[NU];
        int o00[NU], o01[NU], o10[NU], o11[NU];  // element offsets, -1: none
        bool live[NU], diag[NU];
#pragma unroll
        for (int i = 0; i < NU; ++i) {
          const int u = tid + (J0 + i) * JAC_THREADS;
          live[i] = false;
          if (u >= units) continue;
          const int m = u / npair, k = u - m * npair;
          if (m == H && !((npair & 1) || k < H)) continue;
          int l = k + m;
          if (l >= npair) l -= npair;
          sk[i] = rs[k];
          sl[i] = rs[l];
          if (sk[i] == 0.0 && sl[i] == 0.0) continue;
          live[i] = true;
          diag[i] = k == l;  // then pk < qk, and (qk, pk) is (pk, qk)
          ck[i] = rc[k];
          cl[i] = rc[l];
          const int pk = rp[k], qk = rq[k], pl = rp[l], ql = rq[l];
          o00[i] = jac_sym(pk, pl, LD);
          o01[i] = ql >= 0 ? jac_sym(pk, ql, LD) : -1;
          o10[i] = qk >= 0 ? jac_sym(qk, pl, LD) : -1;
          o11[i] = (qk >= 0 && ql >= 0) ? jac_sym(qk, ql, LD) : -1;
          b[i][0] = a[o00[i]];
          b[i][1] = o01[i] >= 0 ? a[o01[i]] : 0.0;
          b[i][2] = o10[i] >= 0 ? a[o10[i]] : 0.0;
          b[i][3] = o11[i] >= 0 ? a[o11[i]] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < NU; ++i) {
          if (!live[i]) continue;
          const double b00 = b[i][0], b01 = b[i][1], b10 = b[i][2], b11 = b[i][3];
          // rows of pair k, then columns of pair l; each x y +- z w as
          // fma(x, y, +-(z w)), the second product rounded (written out, so
          // that the contraction does not depend on how the code is arranged)
          const double r00 = fma(ck[i], b00, -(sk[i] * b10)), r01 = fma(ck[i], b01, -(sk[i] * b11));
          const double r10 = fma(sk[i], b00, ck[i] * b10), r11 = fma(sk[i], b01, ck[i] * b11);
          const double n00 = fma(cl[i], r00, -(sl[i] * r01)), n01 = fma(sl[i], r00, cl[i] * r01);
          const double n10 = fma(cl[i], r10, -(sl[i] * r11)), n11 = fma(sl[i], r10, cl[i] * r11);
          a[o00[i]] = n00;
          if (o01[i] >= 0) a[o01[i]] = n01;
          if (!diag[i] && o10[i] >= 0) a[o10[i]] = n10;
          if (o11[i] >= 0) a[o11[i]] = n11;
        }
      };
      blocks(JacC<0>(), JacC<JAC_FIRST>());
      if constexpr (JAC_FIRST < JAC_UNITS) blocks(JacC<JAC_FIRST>(), JacC<JAC_UNITS>());
      __syncthreads();
    }
    if (rotated == 0) break;
    still = sweep + 1 == limit;
    __syncthreads();
  }
  // eigenvalues: the diagonal, stored after E
  for (int i = tid; i < N; i += JAC_THREADS) jb.E[N * N + i] = a[i * LD + i];
  if (tid == 0) {
    jb.sweeps[0] = sweep;  // sweeps that rotated (all logged)
    if (still && jb.flags) atomicOr(jb.flags, 4);
  }
}

// rows_wg (<= JV_ROWS) rows of E per work-group: one per wave for a single
// matrix (twice the work-groups, each wave half the work), two per wave in a
// batched call (where twice the work-groups, each staging the whole rotation
// log, measured slower)
__global__ __launch_bounds__(JV_THREADS) void k_jacobi_vectors(const JacJob *__restrict__ jobs,
                                                               JacJob one, int rows_wg) {
  __shared__ double e[JV_ROWS][NMAX + 1];
  __shared__ jac_dv2 cs[JV_CHUNK * (NMAX / 2)];
  __shared__ int pqs[JV_CHUNK * (NMAX / 2)];
  const JacJob jb = jobs ? jobs[blockIdx.x] : one;
  const jac_gd2 *rot_log = (const jac_gd2 *)jb.rot;
  const jac_gi *pq_log = (const jac_gi *)jb.pq;
  const int N = jb.N;
  const int row0 = blockIdx.y * rows_wg;
  if (row0 >= N) return;  // uniform over the work-group
  const int rows = N - row0 < rows_wg ? N - row0 : rows_wg;
  const int tid = threadIdx.x;
  for (int x = tid; x < rows * N; x += JV_THREADS) {
    const int i = x / N, j = x % N;
    e[i][j] = (row0 + i == j) ? 1.0 : 0.0;
  }
  const int ne = N + (N & 1);
  const int npair = ne / 2;
  const long long rounds = (long long)jb.sweeps[0] * (ne - 1);
  // a chunk of the log is loaded into registers while the previous one is
  // replayed, and stored to LDS between two barriers
  jac_dv2 vcs[JV_STAGE];
  int vpq[JV_STAGE];
  auto fetch = [&](long long r0) {
    const int cnt = (rounds - r0 < JV_CHUNK ? (int)(rounds - r0) : JV_CHUNK) * npair;
    const size_t base = (size_t)r0 * npair;
#pragma unroll
    for (int k = 0; k < JV_STAGE; ++k) {
      const int x = tid + k * JV_THREADS;
      const size_t o = base + (size_t)(x < cnt ? x : cnt - 1);
      vcs[k] = rot_log[o];
      vpq[k] = pq_log[o];
    }
  };
  if (rounds > 0) fetch(0);
  for (long long r0 = 0; r0 < rounds; r0 += JV_CHUNK) {
    const int nr = rounds - r0 < JV_CHUNK ? (int)(rounds - r0) : JV_CHUNK;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < JV_STAGE; ++k) {
      const int x = tid + k * JV_THREADS;
      if (x < nr * npair) {
        cs[x] = vcs[k];
        pqs[x] = vpq[k];
      }
    }
    __syncthreads();
    if (r0 + JV_CHUNK < rounds) fetch(r0 + JV_CHUNK);
    // a row of E is one wave's alone: lane k applies pair k of every round in
    // turn, and the wave's LDS accesses complete in order, so the rounds of a
    // chunk need no work-group barrier
    const int lane = tid % 64, wave = tid / 64;
    for (int rr = 0; rr < nr; ++rr) {
      if (lane < npair) {
        const jac_dv2 v = cs[rr * npair + lane];
        if (v.y != 0.0) {
          const int pq = pqs[rr * npair + lane];
          const int p = pq & 0xFFFF, q = pq >> 16;
          for (int i = wave; i < rows; i += JV_THREADS / 64) {
            const double x0 = e[i][p], x1 = e[i][q];
            e[i][p] = v.x * x0 - v.y * x1;
            e[i][q] = v.y * x0 + v.x * x1;
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  __syncthreads();
  for (int x = tid; x < rows * N; x += JV_THREADS) {
    const int i = x / N, j = x % N;
    jb.E[(size_t)(row0 + i) * N + j] = e[i][j];
  }
}

static size_t jacobi_lds_bytes(int N) { return (size_t)N * jac_ld(N) * sizeof(double); }

hipError_t launch_jacobi(hipStream_t st, int D, const JacJob *jobs_dev, const JacJob &one,
                         int n_max) {
  const size_t lds = jacobi_lds_bytes(n_max);
  // raise the dynamic-LDS cap where the runtime asks for it; a refusal
  // surfaces as a launch error below
  (void)hipFuncSetAttribute((const void *)k_jacobi_values,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_jacobi_values, dim3(D), dim3(JAC_THREADS), lds, st, jobs_dev, one);
  const int rows_wg = D == 1 ? JV_THREADS / 64 : JV_ROWS;
  hipLaunchKernelGGL(k_jacobi_vectors, dim3(D, (n_max + rows_wg - 1) / rows_wg), dim3(JV_THREADS),
                     0, st, jobs_dev, one, rows_wg);
  return hipGetLastError();
}

// Sort descending (rank by count, ties by index), sign rule, rank check,
// whitening matrix Wh = D^(-1/2) E^T.  One work-group per problem.
__global__ void k_canon(const WJob *__restrict__ jobs, WJob one) {
  const WJob j = jobs ? jobs[blockIdx.x] : one;
  const int N = j.N;
  const double *E = j.E;
  const int i = threadIdx.x;  // one thread per eigenpair, N <= 128
  __shared__ double d[NMAX];
  __shared__ int rank_of[NMAX];
  const double *dv = E + N * N;
  if (i < N) d[i] = dv[i];
  __syncthreads();
  if (i < N) {
    int r = 0;
    for (int k = 0; k < N; ++k)
      if (d[k] > d[i] || (d[k] == d[i] && k < i)) ++r;
    rank_of[i] = r;
  }
  __syncthreads();
  if (i < N) {
    const int r = rank_of[i];
    // sign: largest-magnitude entry of column i positive (lowest row on ties)
    int pm = 0;
    double best = -1.0;
    for (int row = 0; row < N; ++row) {
      const double v = fabs(E[row * N + i]);
      if (v > best) {
        best = v;
        pm = row;
      }
    }
    const double sg = E[pm * N + i] < 0 ? -1.0 : 1.0;
    const double lam = d[i];
    const double sc = sg / sqrt(lam);
    for (int col = 0; col < N; ++col) j.Wh[r * N + col] = sc * E[col * N + i];
    j.eig[r] = lam;
  }
  __syncthreads();
  if (i == 0) {
    double mx = -INFINITY, mn = INFINITY;
    bool fin = true;
    for (int k = 0; k < N; ++k) {
      mx = fmax(mx, d[k]);
      mn = fmin(mn, d[k]);
      fin &= isfinite(d[k]);
    }
    if (!fin || !(mx > 0.0) || !(mn > 1e-12 * mx)) atomicOr(j.flags, 2);
  }
}

// Round a double to bfloat16, nearest-even, directly from the double bits
// (no intermediate FP32 rounding).
__device__ inline uint16_t bf16_rne(double x) {
  const unsigned long long u = __double_as_longlong(x);
  const unsigned sgn = (unsigned)(u >> 63) << 15;
  const int exp = (int)((u >> 52) & 0x7FF);
  const unsigned long long mag = u & 0x7FFFFFFFFFFFFFFFull;
  const unsigned long long lsb = (mag >> 45) & 1ull;
  const unsigned long long r = (mag + 0x0FFFFFFFFFFFull + lsb) >> 45;  // 11-bit exp : 7-bit mant
  const int e = (int)(r >> 7) - 1023 + 127;
  // the normal result is r with its exponent rebiased; the special cases
  // replace it through masks (a select chain here was compiled to branches):
  // zero / subnormal input or underflow -> signed 0, overflow -> Inf,
  // Inf/NaN input -> NaN (the data are finite)
  const unsigned norm = sgn | (unsigned)(r - ((1023ull - 127ull) << 7));
  const unsigned m_zero = 0u - (unsigned)((exp == 0) | (e <= 0));
  const unsigned m_inf = 0u - (unsigned)(e >= 255);
  const unsigned m_nan = 0u - (unsigned)(exp == 0x7FF);
  unsigned v = norm;
  v = (v & ~m_inf) | ((sgn | 0x7F80u) & m_inf);
  v = (v & ~m_zero) | (sgn & m_zero);
  v = (v & ~m_nan) | ((sgn | 0x7FC0u) & m_nan);
  return (uint16_t)v;
}

// Xw = Wh (X - mu) on FP64 MFMA (v_mfma_f64_16x16x4f64: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; result register r holds
// D[l / 16 + 4 r][l % 16]).  A work-group takes apply_cols(N) consecutive
// samples of one problem (1024 for N > 64; 256 below, so that short problems
// still spread over the CUs); a problem's work items are numbered in sample
// order.  Every output accumulates the feature steps 0, 1, ... in order from
// zero, as a single dot product would, in both forms:
//   N <= 64 (apply_stream_body): Wh, zero-padded to 16 * NRB rows and
//     columns, sits in LDS with a row stride of 2 mod 32 doubles (the 16 rows
//     x 2 columns of one A-operand read per half-wave fall in distinct banks).
//     Each wave takes 16-sample column blocks in turn; its B operands (4
//     features x 16 samples of X per step, less the means) come straight from
//     global memory into registers, the next block's loads issued before the
//     current block's MFMAs, so the reduction over features needs no barrier.
//   N > 64 (apply_tiled_body): wave w keeps the A operands of row blocks w and
//     w + 4 of Wh in registers for the whole item (64 doubles per lane) and
//     takes both 16-sample blocks of each 32-sample tile.  The samples pass
//     through LDS as X - mu in FP64, sample-major with a row stride of 2 mod
//     32 doubles (the 16 samples x 2 features of one B-operand read per
//     half-wave fall in distinct banks; features past N and samples past the
//     item are zero), in two buffers: the work-group's loads of the next tile
//     (4 consecutive samples of a feature per thread) are issued before the
//     current tile's MFMAs and written to the other buffer after them and
//     after the current tile's outputs, one barrier per tile.  One B read
//     serves two MFMAs, and two waves fit on a SIMD.  (For N <= 64 the tiles
//     hold too little MFMA work per barrier: measured slower there.)
constexpr int AP_MAX_RB = NMAX / 16;
__host__ __device__ constexpr int apply_cols(int N) { return N > 64 ? 1024 : 256; }
static inline int apply_tiles(int N, long long T) {
  return (int)((T + apply_cols(N) - 1) / apply_cols(N));
}
__host__ __device__ constexpr int wh_ld(int nrb) {
  return nrb * 16 + ((2 - (nrb * 16) % 32) + 32) % 32;
}
constexpr int AP_TS = 32;  // samples per tile of the tiled form
static size_t apply_lds_bytes(int N) {
  const int nrb = (N + 15) / 16;
  if (nrb > 4) return (size_t)2 * AP_TS * wh_ld(nrb) * sizeof(double);  // two tiles
  return ((size_t)wh_ld(nrb) * nrb * 16 + (size_t)nrb * 16) * sizeof(double);  // Wh, means
}
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int NRB, typename TIN>
__device__ __forceinline__ void apply_stream_body(const WJob &j, int item, double *lds) {
  typedef __attribute__((address_space(1))) const TIN gin;
  typedef __attribute__((address_space(1))) float gf32;
  typedef __attribute__((address_space(1))) uint16_t gu16;
  constexpr int NP = NRB * 16;
  constexpr int NK = NRB * 4;          // steps of 4 features
  constexpr int LD = wh_ld(NRB);
  double *whs = lds;                   // NP x LD
  double *mus = lds + NP * LD;         // NP means (0 past N)
  gin *X = (gin *)j.X;
  gf32 *o32 = (gf32 *)j.o32, *o32b = (gf32 *)j.o32b;
  gu16 *obf = (gu16 *)j.obf;
  const int N = j.N;
  const int n_out = j.n_out > 0 ? j.n_out : N;
  const long long T = j.T;
  const long long ldx = j.ld;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int li = lane % 16, lk = lane / 16;
  for (int e = tid; e < NP * NP; e += 256) {
    const int r = e / NP, c = e % NP;
    whs[r * LD + c] = (r < N && c < N) ? j.Wh[r * N + c] : 0.0;
  }
  for (int e = tid; e < NP; e += 256) mus[e] = e < N ? j.mean[e] : 0.0;
  __syncthreads();
  constexpr int COLS = apply_cols(NP);
  const long long m_item = (long long)item * COLS;
  long long m_end = m_item + COLS;
  if (m_end > T) m_end = T;
  // raw X of feature step s at sample m (already clamped into the problem's
  // range).  Indices are clamped into the data instead of masked: a feature
  // past N meets a zero column of Wh (the data are finite, or the call has
  // already failed on them), a sample past the end is never stored, and the
  // loads for the block after the last one are simply not used.  kl is an
  // opaque copy of this lane's feature offset, taken per block, so that the
  // per-step row offsets are recomputed rather than all kept live.
  auto load = [&](long long m, int s, int kl) -> double {
    int f = 4 * s + kl;
    if (f > N - 1) f = N - 1;
    return (double)X[(size_t)f * (size_t)ldx + (size_t)m];
  };
  auto clampm = [&](long long m) { return m < m_end ? m : m_end - 1; };
  // nxt[s] holds step s of the wave's current column block; it is replaced by
  // the same step of the next block as soon as it is used, so every load has
  // a whole block of MFMA work to arrive
  double nxt[NK];
  long long m0 = m_item + 16 * wave;
  if (m0 < m_end) {
#pragma unroll
    for (int s = 0; s < NK; ++s) nxt[s] = load(clampm(m0 + li), s, lk);
  }
  for (; m0 < m_end; m0 += 64) {
    int kl = lk;
    asm volatile("" : "+v"(kl));
    const long long mn = clampm(m0 + 64 + li);
    f64x4 acc[NRB];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) acc[rb] = f64x4{0.0, 0.0, 0.0, 0.0};
    // A operands (Wh) one feature step ahead; fences keep the scheduler from
    // hoisting every step's LDS reads at once, and an opaque zero offset keeps
    // the compiler from lifting all of them (NRB x NK registers) out of the
    // sample loop as loop-invariant
    int wofs = 0;
    asm volatile("" : "+v"(wofs));
    const double *wl = whs + wofs;
    double a[2][NRB];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) a[0][rb] = wl[(rb * 16 + li) * LD + lk];
#pragma unroll
    for (int s = 0; s < NK; ++s) {
      if (s + 1 < NK) {
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb)
          a[(s + 1) % 2][rb] = wl[(rb * 16 + li) * LD + 4 * (s + 1) + lk];
      }
      const double b = nxt[s] - mus[4 * s + lk];
      nxt[s] = load(mn, s, kl);
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb)
        acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s % 2][rb], b, acc[rb], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
    const long long m = m0 + li;
    if (m < m_end) {
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = rb * 16 + lk + 4 * r;
          if (i >= n_out) continue;
          const size_t o = (size_t)i * (size_t)T + (size_t)m;
          const double v = acc[rb][r];
          if (o32) o32[o] = (float)v;
          if (obf) obf[o] = bf16_rne(v);
          if (o32b) o32b[o] = (float)v;
        }
      }
    }
  }
}

template <int R> struct RowCount { static constexpr int value = R; };

template <int NRB, typename TIN>
__device__ __forceinline__ void apply_tiled_body(const WJob &j, int item, double *lds) {
  typedef __attribute__((address_space(1))) const TIN gin;
  typedef __attribute__((address_space(1))) const typename Vec4<TIN>::type gin4;
  typedef __attribute__((address_space(1))) float gf32;
  typedef __attribute__((address_space(1))) uint16_t gu16;
  static_assert(NRB > 4, "the tiled form takes N > 64");
  constexpr int NP = NRB * 16;
  constexpr int NK = NRB * 4;          // steps of 4 features
  constexpr int LDF = wh_ld(NRB);      // tile row stride (one row per sample)
  constexpr int TS = AP_TS;            // samples per tile
  constexpr int RBW = 2;               // row blocks per wave
  constexpr int SBW = TS / 16;         // 16-sample blocks per wave and tile
  constexpr int SPT = TS / 4;          // staging threads per feature
  constexpr int FSTEP = 256 / SPT;     // features staged per pass of the work-group
  constexpr int FPT = (NP + FSTEP - 1) / FSTEP;
  gin *X = (gin *)j.X;
  gf32 *o32 = (gf32 *)j.o32, *o32b = (gf32 *)j.o32b;
  gu16 *obf = (gu16 *)j.obf;
  const int N = j.N;
  const int n_out = j.n_out > 0 ? j.n_out : N;
  const long long T = j.T;
  const long long ldx = j.ld;
  const int tid = threadIdx.x, lane = tid % 64;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);  // uniform: row blocks in SGPRs
  const int li = lane % 16, lk = lane / 16;
  const long long m_item = (long long)item * apply_cols(NP);
  long long m_end = m_item + apply_cols(NP);
  if (m_end > T) m_end = T;
  // this wave's row blocks.  NRB 7 and 8: blocks w and w + 4 on both sample
  // blocks of a tile (for NRB 7, wave 3's block 7 multiplies zeros and stores
  // nothing, in the time the wave would otherwise wait at the tile barrier).
  // NRB 5 and 6 (SPLIT): block w on both sample blocks and block 4 + w / 2
  // (NRB 6; NRB 5: block 4, waves 0 and 1 only) on sample block w % 2 only,
  // so that no wave multiplies a block of zeros and the longest wave does 3
  // block products per tile instead of 4.  Every output comes from the same
  // chain of MFMAs either way.
  constexpr bool SPLIT = NRB <= 6;
  static_assert(!SPLIT || SBW == 2, "the split takes two sample blocks per tile");
  int rbw[RBW];
  rbw[0] = wave;
  rbw[1] = SPLIT ? 4 + (NRB == 6 ? wave / 2 : 0) : wave + 4;
  const bool extra = !SPLIT || NRB == 6 || wave < 2;  // wave uniform
  const int xsb = SPLIT ? wave % 2 : 0;               // sample block with both rows
  // A operands: wa[i][s] = Wh[16 rb + li][4 s + lk], read at clamped indices
  // and zeroed past N
  const double *Wh = j.Wh;
  double wa[RBW][NK];
#pragma unroll
  for (int i = 0; i < RBW; ++i) {
    const int row = rbw[i] * 16 + li;
    const int rowc = row < N ? row : N - 1;
#pragma unroll
    for (int s = 0; s < NK; ++s) {
      const int col = 4 * s + lk;
      const double w = Wh[rowc * N + (col < N ? col : N - 1)];
      wa[i][s] = row < N && col < N ? w : 0.0;
    }
  }
  // staging: features sf + FSTEP i, samples 4 sj .. 4 sj + 3 of a tile;
  // features past N load feature N - 1 (stored as zero)
  const int sf = tid / SPT, sj = tid % SPT;
  double smu[FPT];
  gin *srow[FPT];
#pragma unroll
  for (int i = 0; i < FPT; ++i) {
    const int f = sf + FSTEP * i;
    smu[i] = f < N ? j.mean[f] : 0.0;
    srow[i] = X + (size_t)(f < N ? f : N - 1) * (size_t)ldx;
  }
  TIN reg[FPT][4];
  auto load_full = [&](long long tb) {
    const size_t m = (size_t)(tb + 4 * sj);
#pragma unroll
    for (int i = 0; i < FPT; ++i) {
      const typename Vec4<TIN>::type v = *(gin4 *)(srow[i] + m);
#pragma unroll
      for (int e = 0; e < 4; ++e) reg[i][e] = v[e];
    }
  };
  auto load_tail = [&](long long tb) {
    const long long m = tb + 4 * sj;
#pragma unroll
    for (int i = 0; i < FPT; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) reg[i][e] = srow[i][m + e < m_end ? m + e : m_end - 1];
  };
  auto store_tile = [&](double *buf, long long tb) {
    const long long m = tb + 4 * sj;
#pragma unroll
    for (int i = 0; i < FPT; ++i) {
      const int f = sf + FSTEP * i;
      if (FSTEP * i + FSTEP <= NP || f < NP) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          buf[(4 * sj + e) * LDF + f] = f < N && m + e < m_end ? (double)reg[i][e] - smu[i] : 0.0;
      }
    }
  };
  double *buf0 = lds, *buf1 = lds + TS * LDF;
  const long long nfull = (m_end - m_item) / TS;
  const long long ntiles = nfull + ((m_end - m_item) % TS != 0);
  if (ntiles > 0) {
    if (nfull > 0) load_full(m_item);
    else load_tail(m_item);
    store_tile(buf0, m_item);
  }
  __syncthreads();
  for (long long it = 0; it < ntiles; ++it) {
    const long long tb = m_item + it * TS;
    const double *cur = (it & 1) ? buf1 : buf0;
    double *nxt = (it & 1) ? buf0 : buf1;
    if (it + 1 < nfull) load_full(tb + TS);
    else if (it + 1 < ntiles) load_tail(tb + TS);
    // the products of R of this wave's row blocks with sample block sb of
    // the tile, and their stores
    auto block = [&](auto rows, int sb) {
      constexpr int R = decltype(rows)::value;
      f64x4 acc[R];
#pragma unroll
      for (int i = 0; i < R; ++i) acc[i] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < NK; ++s) {
        const double bv = cur[(sb * 16 + li) * LDF + 4 * s + lk];
#pragma unroll
        for (int i = 0; i < R; ++i)
          acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa[i][s], bv, acc[i], 0, 0, 0);
      }
      const long long m = tb + sb * 16 + li;
      // an opaque copy of the lane's row offset, so that the output rows'
      // 64-bit offsets are formed here rather than all kept live
      int lko = lk;
      asm volatile("" : "+v"(lko));
      const bool all_m = tb + sb * 16 + 16 <= m_end;  // work-group uniform
#pragma unroll
      for (int i = 0; i < R; ++i) {
        // every row of the block stored (wave uniform); a block past NRB
        // stores nothing, its rows being past n_out
        const bool all_r = rbw[i] * 16 + 16 <= n_out;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rbw[i] * 16 + lko + 4 * r;
          if (!(all_m && all_r) && (m >= m_end || row >= n_out)) continue;
          const size_t o = (size_t)row * (size_t)T + (size_t)m;
          const double v = acc[i][r];
          if (o32) o32[o] = (float)v;
          if (obf) obf[o] = bf16_rne(v);
          if (o32b) o32b[o] = (float)v;
        }
      }
    };
    if (SPLIT) {
      if (extra) block(RowCount<2>(), xsb);
      else block(RowCount<1>(), xsb);
      block(RowCount<1>(), 1 - xsb);
    } else {
#pragma unroll
      for (int sb = 0; sb < SBW; ++sb) block(RowCount<RBW>(), sb);
    }
    if (it + 1 < ntiles) store_tile(nxt, tb + TS);
    __syncthreads();
  }
}

// BIG: the kernel for N > 64 (5 to 8 row blocks); the other takes N <= 64,
// so each has the register budget of its own row-block counts.
template <bool BIG, typename TIN>
__device__ __forceinline__ void apply_dispatch(const WJob &j, int item, double *lds) {
  const int nrb = (j.N + 15) / 16;
  if constexpr (BIG) {
    switch (nrb) {
      case 5: apply_tiled_body<5, TIN>(j, item, lds); break;
      case 6: apply_tiled_body<6, TIN>(j, item, lds); break;
      case 7: apply_tiled_body<7, TIN>(j, item, lds); break;
      default: apply_tiled_body<8, TIN>(j, item, lds); break;
    }
  } else {
    switch (nrb) {
      case 1: apply_stream_body<1, TIN>(j, item, lds); break;
      case 2: apply_stream_body<2, TIN>(j, item, lds); break;
      case 3: apply_stream_body<3, TIN>(j, item, lds); break;
      default: apply_stream_body<4, TIN>(j, item, lds); break;
    }
  }
}

// two work-groups per CU (LDS: at most 66 KiB of tiles or 34 KiB of Wh each)
template <bool BIG>
__global__ __launch_bounds__(256, 2) void k_apply(const WJob *__restrict__ jobs, WJob one,
                                                  const int *__restrict__ start, int D) {
  extern __shared__ double ap_lds[];
  int t = blockIdx.x;
  const int d = start ? job_of(start, D, t) : 0;
  if (start) t -= start[d];
  const WJob j = start ? jobs[d] : one;
  if (j.f64) apply_dispatch<BIG, double>(j, t, ap_lds);
  else apply_dispatch<BIG, float>(j, t, ap_lds);
}
static_assert(AP_MAX_RB == 8, "the apply and covariance dispatches cover N up to 128");

// Dynamic LDS of k_apply<BIG> for problems up to n_max features.
template <bool BIG>
static size_t apply_prepare(int n_max) {
  const size_t lds = apply_lds_bytes(n_max);
  (void)hipFuncSetAttribute((const void *)k_apply<BIG>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  (void)hipGetLastError();
  return lds;
}

// Per-problem buffers that live from the statistics to the apply phase.
struct WhitenBufs {
  double *C, *E, *Wh, *mean, *eig;
  int *sweeps;
  double2 *rot;
  int *pq;
};

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// partial sums of the statistics kernels of one problem
static size_t mean_part_bytes(int N, int64_t T) { return al256((size_t)n_chunks(T) * N * sizeof(double)); }
static size_t cov_part_bytes(int N, int64_t T) {
  return al256((size_t)n_cov_chunks(N, T) * N * N * sizeof(double));
}
static size_t stats_scratch_bytes(int N, int64_t T) { return mean_part_bytes(N, T) + cov_part_bytes(N, T); }

// The batched statistics run on groups of problems whose partial sums fit
// this many bytes together (a single larger problem forms a group alone).
constexpr size_t PART_CAP = size_t(256) << 20;

static size_t bufs_bytes(int N) {
  return al256((size_t)N * N * sizeof(double)) +            // C
         al256((size_t)(N * N + N) * sizeof(double)) +      // E + eigenvalues
         3 * al256((size_t)N * N * sizeof(double)) +        // Wh (+ slack for mean, eig)
         al256(64) +                                        // sweeps
         al256(jacobi_log_entries(N) * sizeof(double2)) + al256(jacobi_log_entries(N) * sizeof(int));
}

static WhitenBufs carve_bufs(char *&p, int N, double *V_out, double *mean_out, double *eig_out) {
  auto take = [&](size_t bytes) {
    char *r = p;
    p += al256(bytes);
    return r;
  };
  WhitenBufs b;
  b.C = (double *)take((size_t)N * N * sizeof(double));
  b.E = (double *)take((size_t)(N * N + N) * sizeof(double));
  b.Wh = (double *)take((size_t)N * N * sizeof(double));
  b.mean = (double *)take((size_t)N * sizeof(double));
  b.eig = (double *)take((size_t)N * sizeof(double));
  if (V_out) b.Wh = V_out;
  if (mean_out) b.mean = mean_out;
  if (eig_out) b.eig = eig_out;
  b.sweeps = (int *)take(64);
  b.rot = (double2 *)take(jacobi_log_entries(N) * sizeof(double2));
  b.pq = (int *)take(jacobi_log_entries(N) * sizeof(int));
  return b;
}

static WJob make_wjob(const WhitenJob &w, const WhitenBufs &b, double *mpart, double *cpart,
                      int *flags) {
  WJob j{};
  j.X = w.X;
  j.f64 = w.raw_t == OICA_F64;
  j.N = w.N;
  j.T = w.T;
  j.ld = w.ld;
  j.ch = n_chunks(w.T);
  j.cch = n_cov_chunks(w.N, w.T);
  j.mpart = mpart;
  j.cpart = cpart;
  j.mean = b.mean;
  j.C = b.C;
  j.E = b.E;
  j.Wh = b.Wh;
  j.eig = b.eig;
  j.flags = flags;
  if (w.out_t == OICA_F32) {
    j.o32 = (float *)w.Xw;
  } else {
    j.obf = (uint16_t *)w.Xw;
    j.o32b = w.Xw_f32;
  }
  return j;
}

// Launch ranges (W_KINDS x (D + 1) ints) of the problems of one table.
static void job_starts(const WJob *jj, int D, int *st) {
  for (int k = 0; k < W_KINDS; ++k) st[k * (D + 1)] = 0;
  for (int d = 0; d < D; ++d) {
    const WJob &j = jj[d];
    const int cnt[W_KINDS] = {j.ch, j.N, j.N <= 64 ? j.cch : 0, j.N <= 64 ? 0 : j.cch, j.N * j.N,
                              j.N <= 64 ? apply_tiles(j.N, j.T) : 0,
                              j.N <= 64 ? 0 : apply_tiles(j.N, j.T)};
    for (int k = 0; k < W_KINDS; ++k) st[k * (D + 1) + d + 1] = st[k * (D + 1) + d] + cnt[k];
  }
}

size_t whiten_workspace_bytes(int N, int64_t T) {
  return stats_scratch_bytes(N, T) + bufs_bytes(N) + 1024;
}

// Groups of consecutive problems for the batched statistics.
static std::vector<int> stats_groups(int D, const WhitenJob *jobs, size_t *part_bytes) {
  std::vector<int> first = {0};
  size_t cur = 0, mx = 0;
  for (int d = 0; d < D; ++d) {
    const size_t b = stats_scratch_bytes(jobs[d].N, jobs[d].T);
    if (cur > 0 && cur + b > PART_CAP) {
      first.push_back(d);
      cur = 0;
    }
    cur += b;
    mx = std::max(mx, cur);
  }
  first.push_back(D);
  *part_bytes = mx;
  return first;
}

// Tables of one size class of a batch (Jacobi jobs, problems, launch ranges).
static size_t class_tables_bytes(int D) {
  return al256((size_t)D * sizeof(JacJob)) + al256((size_t)D * sizeof(WJob)) +
         al256((size_t)W_KINDS * (D + 1) * sizeof(int));
}

size_t whiten_batched_workspace_bytes(int D, const WhitenJob *jobs) {
  size_t part = 0, b = 0;
  stats_groups(D, jobs, &part);
  for (int d = 0; d < D; ++d) b += bufs_bytes(jobs[d].N);
  // tables: Jacobi jobs, problems, launch ranges (all problems, then per group)
  return part + b + al256((size_t)D * sizeof(JacJob)) + al256((size_t)D * sizeof(WJob)) +
         al256((size_t)W_KINDS * (D + 1) * sizeof(int)) +
         al256((size_t)W_KINDS * 2 * (D + 1) * sizeof(int)) + 2 * class_tables_bytes(D) + 1024;
}

hipError_t launch_whiten(hipStream_t st, int N, int64_t T, const void *X, oica_dtype raw_t,
                         int64_t ld, void *Xw, oica_dtype out_t, float *Xw_f32, double *V_out,
                         double *mean_out, double *eig_out, void *ws, size_t ws_bytes,
                         int *flags_dev) {
  (void)ws_bytes;
  const WhitenJob w{N, T, X, raw_t, ld, Xw, out_t, Xw_f32, V_out, mean_out, eig_out};
  char *scratch = (char *)ws;
  char *p = scratch + stats_scratch_bytes(N, T);
  const WhitenBufs b = carve_bufs(p, N, V_out, mean_out, eig_out);
  const WJob j = make_wjob(w, b, (double *)scratch, (double *)(scratch + mean_part_bytes(N, T)),
                           flags_dev);
  hipLaunchKernelGGL(k_mean_part, dim3(j.ch), dim3(256), 0, st, nullptr, j, nullptr, 1);
  hipLaunchKernelGGL(k_mean_final, dim3((N + 3) / 4), dim3(256), 0, st, nullptr, j, nullptr, 1, N);
  if (N <= 64)
    hipLaunchKernelGGL(k_cov_part<4>, dim3(j.cch), dim3(256), cov_prepare<4>(N), st, nullptr, j,
                       nullptr, 1);
  else
    hipLaunchKernelGGL(k_cov_part<8>, dim3(j.cch), dim3(256), cov_prepare<8>(N), st, nullptr, j,
                       nullptr, 1);
  hipLaunchKernelGGL(k_cov_final, dim3((N * N + 3) / 4), dim3(256), 0, st, nullptr, j, nullptr, 1,
                     N * N);
  const JacJob job{N, b.C, b.E, b.rot, b.pq, b.sweeps, j.flags, jacobi_max_sweeps()};
  hipError_t e = launch_jacobi(st, 1, nullptr, job, N);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_canon, dim3(1), dim3(NMAX), 0, st, nullptr, j);
  if (N <= 64)
    hipLaunchKernelGGL(k_apply<false>, dim3(apply_tiles(N, T)), dim3(256), apply_prepare<false>(N),
                       st, nullptr, j, nullptr, 1);
  else
    hipLaunchKernelGGL(k_apply<true>, dim3(apply_tiles(N, T)), dim3(256), apply_prepare<true>(N), st,
                       nullptr, j, nullptr, 1);
  return hipGetLastError();
}

// Rows 0 .. n_out-1 of Wh (X - mean) for an N x N FP64 matrix Wh, FP32 data X
// (row stride ld) and FP64 means (zeros for data already centred): the apply
// kernel of the whitening with fewer output rows.  Outputs of T samples per
// row (row stride T): o32 FP32 and/or obf BF16 (either may be null).
hipError_t launch_apply_rows(hipStream_t st, int N, int n_out, int64_t T, const float *X,
                             int64_t ld, const double *Wh, const double *mean, float *o32,
                             uint16_t *obf) {
  WJob j{};
  j.X = X;
  j.f64 = 0;
  j.N = N;
  j.T = T;
  j.ld = ld;
  j.mean = (double *)mean;
  j.Wh = (double *)Wh;
  j.o32 = o32;
  j.obf = obf;
  j.n_out = n_out;
  if (N <= 64)
    hipLaunchKernelGGL(k_apply<false>, dim3(apply_tiles(N, T)), dim3(256), apply_prepare<false>(N),
                       st, nullptr, j, nullptr, 1);
  else
    hipLaunchKernelGGL(k_apply<true>, dim3(apply_tiles(N, T)), dim3(256), apply_prepare<true>(N), st,
                       nullptr, j, nullptr, 1);
  return hipGetLastError();
}

// Many problems: the statistics kernels run on groups of problems (all the
// problems of a group in one launch each, their partial sums side by side),
// every eigenproblem in one launch of the Jacobi kernels (one work-group
// each), then canon and apply for every problem in one launch each.  Each
// problem's arithmetic is that of a single call.  flags_dev: D ints, zero on
// entry; the job tables are copied to the device first and the stream
// synchronised, so `jobs` may be freed on return.
hipError_t launch_whiten_batched(hipStream_t st, int D, const WhitenJob *jobs, void *ws,
                                 int *flags_dev, hipStream_t aux, hipEvent_t fork,
                                 hipEvent_t join) {
  size_t part_bytes = 0;
  const std::vector<int> groups = stats_groups(D, jobs, &part_bytes);
  int n_max = 1;
  for (int d = 0; d < D; ++d) n_max = std::max(n_max, jobs[d].N);
  char *scratch = (char *)ws;
  char *p = scratch + part_bytes;
  JacJob *jac_dev = (JacJob *)p;
  p += al256((size_t)D * sizeof(JacJob));
  WJob *wj_dev = (WJob *)p;
  p += al256((size_t)D * sizeof(WJob));
  int *starts_dev = (int *)p;
  p += al256((size_t)W_KINDS * (D + 1) * sizeof(int));
  std::vector<WhitenBufs> bufs(D);
  std::vector<JacJob> jj(D);
  std::vector<WJob> wj(D);
  // partial buffers: offsets restart at each group
  size_t off = 0;
  for (size_t g = 0; g + 1 < groups.size(); ++g) {
    off = 0;
    for (int d = groups[g]; d < groups[g + 1]; ++d) {
      bufs[d] = carve_bufs(p, jobs[d].N, jobs[d].V, jobs[d].mean, jobs[d].eig);
      jj[d] = JacJob{jobs[d].N, bufs[d].C, bufs[d].E, bufs[d].rot, bufs[d].pq, bufs[d].sweeps,
                     flags_dev + d, jacobi_max_sweeps()};
      double *mp = (double *)(scratch + off);
      double *cp = (double *)(scratch + off + mean_part_bytes(jobs[d].N, jobs[d].T));
      off += stats_scratch_bytes(jobs[d].N, jobs[d].T);
      wj[d] = make_wjob(jobs[d], bufs[d], mp, cp, flags_dev + d);
    }
  }
  // launch ranges: per group for the statistics kernels (ranges start at the
  // group's first problem), over all problems for canon and apply
  std::vector<int> starts((size_t)W_KINDS * (D + 1));
  std::vector<int> gstarts;  // per group: W_KINDS x (size + 1)
  std::vector<size_t> gofs;
  for (size_t g = 0; g + 1 < groups.size(); ++g) {
    const int n = groups[g + 1] - groups[g];
    gofs.push_back(gstarts.size());
    gstarts.resize(gstarts.size() + (size_t)W_KINDS * (n + 1));
    job_starts(wj.data() + groups[g], n, gstarts.data() + gofs.back());
  }
  job_starts(wj.data(), D, starts.data());
  int *gstarts_dev = nullptr;
  hipError_t e = hipMemcpyAsync(jac_dev, jj.data(), (size_t)D * sizeof(JacJob),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(wj_dev, wj.data(), (size_t)D * sizeof(WJob), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(starts_dev, starts.data(), starts.size() * sizeof(int),
                       hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  // group ranges go after the problems' buffers
  gstarts_dev = (int *)p;
  e = hipMemcpyAsync(gstarts_dev, gstarts.data(), gstarts.size() * sizeof(int),
                     hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  // Size classes (N <= 64, N > 64): with an auxiliary stream and both classes
  // present, the small class's eigen-solve, canon and apply run on `aux` while
  // the large class's (whose N = 128 solves take longest) run on `st`, so the
  // small apply no longer waits for the slowest solve.  Each problem's
  // kernels and arithmetic are those of the one-stream form.
  std::vector<int> cls[2];
  for (int d = 0; d < D; ++d) cls[jobs[d].N > 64].push_back(d);
  const bool split = aux != nullptr && !cls[0].empty() && !cls[1].empty();
  std::vector<JacJob> cjj[2];
  std::vector<WJob> cwj[2];
  std::vector<int> cstarts[2];
  JacJob *cjac_dev[2] = {nullptr, nullptr};
  WJob *cwj_dev[2] = {nullptr, nullptr};
  int *cstarts_dev[2] = {nullptr, nullptr};
  int cn_max[2] = {1, 1};
  if (split) {
    char *q = (char *)gstarts_dev + al256((size_t)W_KINDS * 2 * (D + 1) * sizeof(int));
    for (int c = 0; c < 2; ++c) {
      const int n = (int)cls[c].size();
      for (int d : cls[c]) {
        cjj[c].push_back(jj[d]);
        cwj[c].push_back(wj[d]);
        cn_max[c] = std::max(cn_max[c], jobs[d].N);
      }
      cstarts[c].resize((size_t)W_KINDS * (n + 1));
      job_starts(cwj[c].data(), n, cstarts[c].data());
      cjac_dev[c] = (JacJob *)q;
      q += al256((size_t)D * sizeof(JacJob));
      cwj_dev[c] = (WJob *)q;
      q += al256((size_t)D * sizeof(WJob));
      cstarts_dev[c] = (int *)q;
      q += al256((size_t)W_KINDS * (D + 1) * sizeof(int));
      e = hipMemcpyAsync(cjac_dev[c], cjj[c].data(), (size_t)n * sizeof(JacJob),
                         hipMemcpyHostToDevice, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(cwj_dev[c], cwj[c].data(), (size_t)n * sizeof(WJob),
                           hipMemcpyHostToDevice, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(cstarts_dev[c], cstarts[c].data(), cstarts[c].size() * sizeof(int),
                           hipMemcpyHostToDevice, st);
      if (e != hipSuccess) return e;
    }
  }
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  for (size_t g = 0; g + 1 < groups.size(); ++g) {
    const int d0 = groups[g], n = groups[g + 1] - groups[g];
    const int *gs = gstarts.data() + gofs[g];
    const int *gd = gstarts_dev + gofs[g];
    auto tot = [&](int kind) { return gs[kind * (n + 1) + n]; };
    auto rng = [&](int kind) { return gd + kind * (n + 1); };
    const WJob &j0 = wj[d0];
    hipLaunchKernelGGL(k_mean_part, dim3(tot(W_MEAN)), dim3(256), 0, st, wj_dev + d0, j0,
                       rng(W_MEAN), n);
    hipLaunchKernelGGL(k_mean_final, dim3((tot(W_MEANF) + 3) / 4), dim3(256), 0, st, wj_dev + d0,
                       j0, rng(W_MEANF), n, tot(W_MEANF));
    if (tot(W_COV4) > 0)
      hipLaunchKernelGGL(k_cov_part<4>, dim3(tot(W_COV4)), dim3(256), cov_prepare<4>(64), st,
                         wj_dev + d0, j0, rng(W_COV4), n);
    if (tot(W_COV8) > 0)
      hipLaunchKernelGGL(k_cov_part<8>, dim3(tot(W_COV8)), dim3(256), cov_prepare<8>(NMAX), st,
                         wj_dev + d0, j0, rng(W_COV8), n);
    hipLaunchKernelGGL(k_cov_final, dim3((tot(W_COVF) + 3) / 4), dim3(256), 0, st, wj_dev + d0, j0,
                       rng(W_COVF), n, tot(W_COVF));
  }
  // eigen-solve, canon and apply of a set of problems on one stream
  auto finish = [&](hipStream_t sc, int n, const JacJob *jdev, const JacJob &j1, const WJob *wdev,
                    const WJob &w1, const int *sdev, const int *sh, int nmx) -> hipError_t {
    hipError_t r = launch_jacobi(sc, n, jdev, j1, nmx);
    if (r != hipSuccess) return r;
    hipLaunchKernelGGL(k_canon, dim3(n), dim3(NMAX), 0, sc, wdev, w1);
    const int n_ap4 = sh[W_APPLY4 * (n + 1) + n], n_ap8 = sh[W_APPLY8 * (n + 1) + n];
    if (n_ap4 > 0)
      hipLaunchKernelGGL(k_apply<false>, dim3(n_ap4), dim3(256),
                         apply_prepare<false>(std::min(nmx, 64)), sc, wdev, w1,
                         sdev + W_APPLY4 * (n + 1), n);
    if (n_ap8 > 0)
      hipLaunchKernelGGL(k_apply<true>, dim3(n_ap8), dim3(256), apply_prepare<true>(nmx), sc,
                         wdev, w1, sdev + W_APPLY8 * (n + 1), n);
    return hipGetLastError();
  };
  if (!split)
    return finish(st, D, jac_dev, jj[0], wj_dev, wj[0], starts_dev, starts.data(), n_max);
  e = hipEventRecord(fork, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(aux, fork, 0);
  if (e != hipSuccess) return e;
  const int n0 = (int)cls[0].size(), n1 = (int)cls[1].size();
  e = finish(aux, n0, cjac_dev[0], cjj[0][0], cwj_dev[0], cwj[0][0], cstarts_dev[0],
             cstarts[0].data(), cn_max[0]);
  // the join is recorded whatever happened, so the call's stream never waits
  // on an event of an earlier call
  hipError_t e1 = finish(st, n1, cjac_dev[1], cjj[1][0], cwj_dev[1], cwj[1][0], cstarts_dev[1],
                         cstarts[1].data(), cn_max[1]);
  hipError_t e2 = hipEventRecord(join, aux);
  if (e2 == hipSuccess) e2 = hipStreamWaitEvent(st, join, 0);
  return e != hipSuccess ? e : e1 != hipSuccess ? e1 : e2;
}

}  // namespace oica
