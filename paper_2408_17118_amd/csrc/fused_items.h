// Per-work-item device code of the fused fixed-point pass, shared by the
// single-dataset kernels (fixed_point.hip) and the persistent many-dataset
// kernel (batched.hip).  A work item is one block of active rows over one
// split of the samples: it stages X tiles in LDS, runs GEMM1 -> cube -> GEMM2
// on MFMA and writes the item's partial G and partial sum z^4.
//
// MFMA v_mfma_f32_32x32x2f32 operand layout (wave64, lane l, h = l / 32,
// i = l % 32):  A[i][h], B[h][i]  (one float each);  D[r][i] in vgpr v with
// r = 8 (v / 4) + 4 h + (v % 4).  GEMM1 produces Z^T with the rows of B on the
// lane index, so the same registers are directly the B operand of GEMM2 with
// the samples permuted by r(v, h); GEMM2's A operand reads X with the same
// permutation.
#pragma once

#include "oica_internal.h"

namespace oica {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Global-memory views of the item's pointers.  The items also run inside
// separate (not inlined) functions of the batched kernel, where pointers read
// from a context struct are generic: spelled out as global, their loads and
// stores are global (not flat) instructions, which do not hold up the LDS
// waits of the MFMA loop.
#define OICA_GLOBAL __attribute__((address_space(1)))
typedef OICA_GLOBAL const float g_cf32;
typedef OICA_GLOBAL float g_f32;
typedef OICA_GLOBAL double g_f64;
typedef OICA_GLOBAL const int g_cint;
typedef OICA_GLOBAL const f32x4 g_cf32x4;
typedef OICA_GLOBAL f32x4 g_f32x4;

constexpr int WAVES = WAVES_PER_WG;  // waves per work-group
// FP32 X tile in LDS: tt samples (32-sample sub-tiles) x NP features with an
// odd row stride, so column reads hit distinct banks.  The widest variant
// uses 32-sample tiles to leave registers for the one-tile-ahead prefetch.
template <int NP> struct TileF32 {
  static constexpr int tt = NP <= 96 ? 64 : 32;
  static constexpr int sx = tt + 1;
};
constexpr int MIN_SUB = 8;      // each sample split covers >= 8 sub-tiles (256 samples)
constexpr int GRID = 1024;      // work-groups per fused launch (multiple of 8)
constexpr int SPLIT_GROUP = SPLIT_GROUP_HOST;  // splits per first-stage reduction item
constexpr int RED_GRID = 2048;  // work-groups of the first-stage reduction
constexpr int EPI_ROWS = 16;    // rows per wave in the per-row passes (epilogue, init)

// Everything one (row block, sample split) work item needs.
struct ItemCtx {
  const void *X;       // N rows of T samples, row stride ld elements
  int N;
  long long T;
  long long ld;
  int n_sub;
  int n_sp;
  int rows_pad;
  const float *Bm;
  const int *act;
  int kact;
  float *gpart;
  float *s4part;
  double *s4part64;
};

// ---------------------------------------------------------------------------
// One work item of the FP32 fused pass: the rows kb*KWG .. of the active list
// over the samples of split sp.
//   KURT = false: writes partial G (NP floats per row) and partial sum z^4.
//   KURT = true : skips GEMM2 and writes partial sum z^4 in FP64.
//   PF = true   : prefetches the next X tile into registers during the MFMA
//                 work of the current one (PF = false: load, stage, compute).
// ---------------------------------------------------------------------------
template <int NP, int WK, bool KURT, bool PF = true>
__device__ __forceinline__ void item_f32(const ItemCtx &c, int kb, int sp, float *xs) {
  constexpr int KWG = WAVES * WK * 32;
  constexpr int HALF = NP / 2;
  constexpr int TT = TileF32<NP>::tt;
  constexpr int SX = TileF32<NP>::sx;
  g_cf32 *__restrict__ X = (g_cf32 *)c.X;
  const int N = c.N;
  const long long T = c.T;
  const int n_sp = c.n_sp;
  const int rows_pad = c.rows_pad;
  g_cf32 *__restrict__ Bm = (g_cf32 *)c.Bm;
  g_cint *__restrict__ act = (g_cint *)c.act;
  const int kact = c.kact;
  g_f32 *__restrict__ gpart = (g_f32 *)c.gpart;
  g_f32 *__restrict__ s4part = (g_f32 *)c.s4part;
  g_f64 *__restrict__ s4part64 = (g_f64 *)c.s4part64;
  const int tid = threadIdx.x;
  const int wave = tid / 64;
  const int lane = tid % 64;
  const int h = lane / 32;
  const int li = lane % 32;
  {
    const long long sub0 = (long long)sp * c.n_sub / n_sp;
    const long long sub1 = (long long)(sp + 1) * c.n_sub / n_sp;
    const long long t_begin = sub0 * 32;
    long long t_end = sub1 * 32;
    if (t_end > T) t_end = T;

    // B rows of this wave into registers: column block w covers positions
    // kb*KWG + wave*WK*32 + w*32 + li; feature n = HALF*h + s.
    float breg[WK][HALF];
    int pos[WK];
#pragma unroll
    for (int w = 0; w < WK; ++w) {
      pos[w] = kb * KWG + wave * WK * 32 + w * 32 + li;
      int row = -1;
      if (pos[w] < kact) row = act ? act[pos[w]] : pos[w];
#pragma unroll
      for (int s = 0; s < HALF; ++s) {
        const int n = HALF * h + s;
        breg[w][s] = (row >= 0 && n < N) ? Bm[(size_t)row * N + n] : 0.f;
      }
    }

    f32x16 gacc[WK][NP / 32];
    float s4acc[WK];
    double s4acc64[WK];
#pragma unroll
    for (int w = 0; w < WK; ++w) {
      s4acc[w] = 0.f;
      s4acc64[w] = 0.0;
#pragma unroll
      for (int nb = 0; nb < NP / 32; ++nb) gacc[w][nb] = f32x16{0.f};
    }

    // X tiles go through registers (4 consecutive samples of one feature row
    // per load); with PF they are fetched one tile ahead, so the global-load
    // latency of tile i+1 overlaps the MFMA work of tile i.
    constexpr int F4 = NP * TT / 4 / (WAVES * 64);
    const long long ld = c.ld;
    const bool vec4 = (ld % 4) == 0;  // 16-byte aligned rows
    f32x4 pre[F4];
    auto fetch = [&](long long mt) {
#pragma unroll
      for (int q = 0; q < F4; ++q) {
        const int e = tid + q * WAVES * 64;
        const int n = e / (TT / 4);
        const long long gm = mt + (e % (TT / 4)) * 4;
        g_cf32 *src = X + (size_t)n * (size_t)ld + (size_t)gm;
        if (n < N && vec4 && gm + 4 <= t_end) {
          pre[q] = *reinterpret_cast<g_cf32x4 *>(src);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) pre[q][j] = (n < N && gm + j < t_end) ? src[j] : 0.f;
        }
      }
    };
    if constexpr (PF) fetch(t_begin);
    for (long long m_tile = t_begin; m_tile < t_end; m_tile += TT) {
      __syncthreads();
      if constexpr (!PF) fetch(m_tile);
#pragma unroll
      for (int q = 0; q < F4; ++q) {
        const int e = tid + q * WAVES * 64;
        const int n = e / (TT / 4);
        const int m4 = (e % (TT / 4)) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) xs[n * SX + m4 + j] = pre[q][j];
      }
      __syncthreads();
      if constexpr (PF)
        if (m_tile + TT < t_end) fetch(m_tile + TT);
#pragma unroll
      for (int sub = 0; sub < TT / 32; ++sub) {
        if (m_tile + sub * 32 >= t_end) break;
        const int m0 = sub * 32;
        f32x16 zacc[WK];
#pragma unroll
        for (int w = 0; w < WK; ++w) zacc[w] = f32x16{0.f};
#pragma unroll
        for (int s = 0; s < HALF; ++s) {
          const float a = xs[(HALF * h + s) * SX + m0 + li];
#pragma unroll
          for (int w = 0; w < WK; ++w)
            zacc[w] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, breg[w][s], zacc[w], 0, 0, 0);
        }
        if constexpr (KURT) {
#pragma unroll
          for (int w = 0; w < WK; ++w) {
            float t4 = 0.f;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const float z2 = zacc[w][v] * zacc[w][v];
              t4 = fmaf(z2, z2, t4);
            }
            s4acc64[w] += (double)t4;
          }
        } else {
          f32x16 p3[WK];
#pragma unroll
          for (int w = 0; w < WK; ++w) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const float z = zacc[w][v];
              const float z2 = z * z;
              p3[w][v] = z2 * z;
              s4acc[w] = fmaf(z2, z2, s4acc[w]);
            }
          }
#pragma unroll
          for (int nb = 0; nb < NP / 32; ++nb) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const int m = m0 + 8 * (v / 4) + 4 * h + (v % 4);
              const float a = xs[(nb * 32 + li) * SX + m];
#pragma unroll
              for (int w = 0; w < WK; ++w)
                gacc[w][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, p3[w][v], gacc[w][nb], 0, 0, 0);
            }
          }
        }
      }
    }

    // Write this item's partials.
#pragma unroll
    for (int w = 0; w < WK; ++w) {
      if constexpr (KURT) {
        const double tot = s4acc64[w] + __shfl_xor(s4acc64[w], 32);
        if (h == 0 && pos[w] < kact) s4part64[(size_t)sp * rows_pad + pos[w]] = tot;
      } else {
        const float tot = s4acc[w] + __shfl_xor(s4acc[w], 32);
        if (pos[w] < kact) {
          if (h == 0) s4part[(size_t)sp * rows_pad + pos[w]] = tot;
          g_f32 *dst = gpart + ((size_t)sp * rows_pad + pos[w]) * NP;
#pragma unroll
          for (int nb = 0; nb < NP / 32; ++nb) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              f32x4 v4;
              v4[0] = gacc[w][nb][4 * q + 0];
              v4[1] = gacc[w][nb][4 * q + 1];
              v4[2] = gacc[w][nb][4 * q + 2];
              v4[3] = gacc[w][nb][4 * q + 3];
              *reinterpret_cast<g_f32x4 *>(dst + nb * 32 + 8 * q + 4 * h) = v4;
            }
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// One-wave FP32 item: rows kb*32 .. kb*32+31 of the active list over the
// samples of split sp, computed by one wave alone in its own LDS tile
// (NP x ThinF32::sx floats), so the four waves of a work-group take four
// splits of a problem with at most 32 active rows instead of three of them
// multiplying padding rows.  The arithmetic per row is that of item_f32 on
// the same split: the same 32-sample sub-tiles in the same order and the
// same MFMA sequence on each, so the partials are identical.
// ---------------------------------------------------------------------------
struct ThinF32 {
  static constexpr int tt = 32;
  static constexpr int sx = tt + 1;
};

// Orders this wave's LDS accesses before and after the point (the LDS tile
// is private to the wave, so no work-group barrier is involved).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef __attribute__((address_space(3))) float lds_f32;

template <int NP>
__device__ __forceinline__ void item_f32_wave(const ItemCtx &c, int kb, int sp, float *xs_any) {
  // the tile is in LDS: say so, so the accesses are LDS instructions with
  // 32-bit addresses even when this runs in a separate (not inlined) function
  lds_f32 *xs = (lds_f32 *)xs_any;
  constexpr int HALF = NP / 2;
  constexpr int TT = ThinF32::tt;
  constexpr int SX = ThinF32::sx;
  g_cf32 *__restrict__ X = (g_cf32 *)c.X;
  const int N = c.N;
  const long long T = c.T;
  const int rows_pad = c.rows_pad;
  const int kact = c.kact;
  g_cf32 *__restrict__ Bm = (g_cf32 *)c.Bm;
  g_cint *__restrict__ act = (g_cint *)c.act;
  g_f32 *__restrict__ gpart = (g_f32 *)c.gpart;
  g_f32 *__restrict__ s4part = (g_f32 *)c.s4part;
  const long long ld = c.ld;
  const int lane = threadIdx.x % 64;
  const int h = lane / 32;
  const int li = lane % 32;
  const long long sub0 = (long long)sp * c.n_sub / c.n_sp;
  const long long sub1 = (long long)(sp + 1) * c.n_sub / c.n_sp;
  const long long t_begin = sub0 * 32;
  long long t_end = sub1 * 32;
  if (t_end > T) t_end = T;

  const int pos = kb * 32 + li;
  int row = -1;
  if (pos < kact) row = act ? act[pos] : pos;
  float breg[HALF];
#pragma unroll
  for (int s = 0; s < HALF; ++s) {
    const int n = HALF * h + s;
    breg[s] = (row >= 0 && n < N) ? Bm[(size_t)row * N + n] : 0.f;
  }
  f32x16 gacc[NP / 32];
  float s4acc = 0.f;
#pragma unroll
  for (int nb = 0; nb < NP / 32; ++nb) gacc[nb] = f32x16{0.f};

  constexpr int F4 = NP * TT / 4 / 64;  // 16-byte loads per lane per tile
  constexpr int CH = 4;                 // loads in flight per lane
  const bool vec4 = (ld % 4) == 0;
  for (long long m_tile = t_begin; m_tile < t_end; m_tile += TT) {
    wave_lds_sync();  // the previous tile's reads are done
#pragma unroll 1
    for (int q0 = 0; q0 < F4; q0 += CH) {
      f32x4 pre[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int e = lane + (q0 + u) * 64;
        const int n = e / (TT / 4);
        const long long gm = m_tile + (e % (TT / 4)) * 4;
        g_cf32 *src = X + (size_t)n * (size_t)ld + (size_t)gm;
        if (n < N && vec4 && gm + 4 <= t_end) {
          pre[u] = *reinterpret_cast<g_cf32x4 *>(src);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) pre[u][j] = (n < N && gm + j < t_end) ? src[j] : 0.f;
        }
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int e = lane + (q0 + u) * 64;
        const int n = e / (TT / 4);
        const int m4 = (e % (TT / 4)) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) xs[n * SX + m4 + j] = pre[u][j];
      }
    }
    wave_lds_sync();  // the tile is in LDS
    f32x16 zacc = f32x16{0.f};
#pragma unroll
    for (int s = 0; s < HALF; ++s) {
      const float a = xs[(HALF * h + s) * SX + li];
      zacc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, breg[s], zacc, 0, 0, 0);
    }
    f32x16 p3;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float z = zacc[v];
      const float z2 = z * z;
      p3[v] = z2 * z;
      s4acc = fmaf(z2, z2, s4acc);
    }
#pragma unroll
    for (int nb = 0; nb < NP / 32; ++nb) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int m = 8 * (v / 4) + 4 * h + (v % 4);
        const float a = xs[(nb * 32 + li) * SX + m];
        gacc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, p3[v], gacc[nb], 0, 0, 0);
      }
    }
  }
  const float tot = s4acc + __shfl_xor(s4acc, 32);
  if (pos < kact) {
    if (h == 0) s4part[(size_t)sp * rows_pad + pos] = tot;
    g_f32 *dst = gpart + ((size_t)sp * rows_pad + pos) * NP;
#pragma unroll
    for (int nb = 0; nb < NP / 32; ++nb) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        f32x4 v4;
        v4[0] = gacc[nb][4 * q + 0];
        v4[1] = gacc[nb][4 * q + 1];
        v4[2] = gacc[nb][4 * q + 2];
        v4[3] = gacc[nb][4 * q + 3];
        *reinterpret_cast<g_f32x4 *>(dst + nb * 32 + 8 * q + 4 * h) = v4;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// BF16 pass kernel: X stored in BF16, both contractions on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation; z^3 rounded to BF16
// (nearest even) to feed GEMM2.  Each row b is split once per work item into
// b_hi = bf16(b) and b_lo = bf16(b - b_hi), and GEMM1 runs on both, so z carries
// b to ~2^-17 relative: rounding b itself to BF16 would make the update map
// piecewise constant in b and leave the step stuck near 1e-4.  Operand layout (lane l, h = l / 32, i = l % 32): A[i][8h + j],
// B[8h + j][i] for j = 0..7 (8 bf16 per lane); D as in the FP32 kernel.
// GEMM1 reads the transposed LDS copy xt[m][n] (8 consecutive features, one
// 16-byte read); GEMM2 reads xs[n][m] (two runs of 4 consecutive samples).
// With v = 8q + j for MFMA q of a 32-sample sub-tile, GEMM1's accumulator
// lane holds sample m = 16q + 8(j/4) + 4h + j%4 at k-index 8h + j, so the
// cubed registers are GEMM2's B operand directly.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef OICA_GLOBAL const __bf16 g_cbf16;
typedef OICA_GLOBAL const bf16x8 g_cbf16x8;
constexpr int BT = 64;          // samples per LDS tile
// xs row stride (bf16): 136 bytes = 34 banks, so the 8-byte GEMM2 operand
// reads of 32 consecutive rows hit 32 distinct bank pairs; rows are written
// with 8-byte stores (8-byte aligned)
constexpr int BSX = BT + 4;
template <int NP> struct BfStride { static constexpr int v = NP + 8; };  // xt row stride
// one LDS buffer of the BF16 item: xs (NP x BSX) and xt (BT x (NP + 8)); the
// item uses two of each
template <int NP> struct BfTile {
  static constexpr int xs_elems = NP * BSX;
  static constexpr int xt_elems = BT * BfStride<NP>::v;
};

// S4: also form the per-row sums of z^4 (the kurtosis of the rows before the
// update, recorded only in the passes whose trajectory is kept); without it
// the sums are skipped and a non-null s4part receives zeros.
// NW: waves of the work-group (all stage the shared X tile; each holds its own
// WK x 32 rows).
// LO: rows carried as hi + lo BF16 parts (two GEMM1 MFMAs per step); without
// it each row is rounded once to BF16 (the hi part alone) and the pass is the
// update of that rounded row (the epilogue takes the linear term from the same
// rounding).
template <int NP, int WK, bool S4 = true, int NW = WAVES, bool LO = true>
__device__ __forceinline__ void item_bf16(const ItemCtx &c, int kb, int sp, __bf16 *xs_base,
                                          __bf16 *xt_base) {
  constexpr int KWG = NW * WK * 32;
  constexpr int XTS = BfStride<NP>::v;
  g_cbf16 *__restrict__ X = (g_cbf16 *)c.X;
  const int N = c.N;
  const long long T = c.T;
  const int n_sp = c.n_sp;
  const int rows_pad = c.rows_pad;
  g_cf32 *__restrict__ Bm = (g_cf32 *)c.Bm;
  g_cint *__restrict__ act = (g_cint *)c.act;
  const int kact = c.kact;
  g_f32 *__restrict__ gpart = (g_f32 *)c.gpart;
  g_f32 *__restrict__ s4part = (g_f32 *)c.s4part;
  const int tid = threadIdx.x;
  const int wave = tid / 64;
  const int lane = tid % 64;
  const int h = lane / 32;
  const int li = lane % 32;
  const long long ld = c.ld;
  const bool vec_ok = (ld % 8) == 0;  // 16-byte aligned rows
  {
    const long long sub0 = (long long)sp * c.n_sub / n_sp;
    const long long sub1 = (long long)(sp + 1) * c.n_sub / n_sp;
    const long long t_begin = sub0 * 32;
    long long t_end = sub1 * 32;
    if (t_end > T) t_end = T;

    bf16x8 breg[WK][NP / 16], blo[WK][NP / 16];
    int pos[WK];
#pragma unroll
    for (int w = 0; w < WK; ++w) {
      pos[w] = kb * KWG + wave * WK * 32 + w * 32 + li;
      int row = -1;
      if (pos[w] < kact) row = act ? act[pos[w]] : pos[w];
#pragma unroll
      for (int s = 0; s < NP / 16; ++s) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int n = 16 * s + 8 * h + j;
          const float b = (row >= 0 && n < N) ? Bm[(size_t)row * N + n] : 0.f;
          const __bf16 hi = (__bf16)b;
          breg[w][s][j] = hi;
          blo[w][s][j] = LO ? (__bf16)(b - (float)hi) : (__bf16)0.f;
        }
      }
    }

    f32x16 gacc[WK][NP / 32];
    float s4acc[WK];
#pragma unroll
    for (int w = 0; w < WK; ++w) {
      s4acc[w] = 0.f;
#pragma unroll
      for (int nb = 0; nb < NP / 32; ++nb) gacc[w][nb] = f32x16{0.f};
    }

    // X tiles go through registers, one tile ahead with PF.  A staging unit is
    // one feature pair (2p, 2p+1) over 8 consecutive samples (two 16-byte
    // loads); pairs vary fastest across lanes, so both LDS layouts are written
    // without bank conflicts: xs rows with 16-byte stores, xt with one 32-bit
    // store per sample holding the pair.
    constexpr int PAIRS = NP / 2;
    constexpr int UNITS = PAIRS * (BT / 8);
    constexpr int F8 = (UNITS + NW * 64 - 1) / (NW * 64);
    bf16x8 pre0[F8], pre1[F8];
    auto fetch = [&](long long mt) {
#pragma unroll
      for (int q = 0; q < F8; ++q) {
        const int u = tid + q * NW * 64;
        const int pp = u % PAIRS, c = u / PAIRS;
        const long long gm = mt + c * 8;
        const int n0 = 2 * pp;
        g_cbf16 *src0 = X + (size_t)n0 * (size_t)ld + (size_t)gm;
        g_cbf16 *src1 = src0 + (size_t)ld;
        if (u < UNITS && n0 + 1 < N && vec_ok && gm + 8 <= t_end) {
          pre0[q] = *reinterpret_cast<g_cbf16x8 *>(src0);
          pre1[q] = *reinterpret_cast<g_cbf16x8 *>(src1);
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const bool in = u < UNITS && gm + j < t_end;
            pre0[q][j] = (in && n0 < N) ? src0[j] : (__bf16)0.f;
            pre1[q][j] = (in && n0 + 1 < N) ? src1[j] : (__bf16)0.f;
          }
        }
      }
    };
    auto stage = [&](int b) {
      __bf16 *xs = xs_base + b * BfTile<NP>::xs_elems;
      __bf16 *xt = xt_base + b * BfTile<NP>::xt_elems;
#pragma unroll
      for (int q = 0; q < F8; ++q) {
        const int u = tid + q * NW * 64;
        if (u < UNITS) {
          const int pp = u % PAIRS, c = u / PAIRS;
          bf16x4 *r0 = reinterpret_cast<bf16x4 *>(&xs[(2 * pp) * BSX + c * 8]);
          bf16x4 *r1 = reinterpret_cast<bf16x4 *>(&xs[(2 * pp + 1) * BSX + c * 8]);
          r0[0] = pre0[q].lo;
          r0[1] = pre0[q].hi;
          r1[0] = pre1[q].lo;
          r1[1] = pre1[q].hi;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            bf16x2 two;
            two[0] = pre0[q][j];
            two[1] = pre1[q][j];
            *reinterpret_cast<bf16x2 *>(&xt[(c * 8 + j) * XTS + 2 * pp]) = two;
          }
        }
      }
    };
    // Two LDS buffers: tile i is computed from buffer i % 2 while tile i + 1
    // (already in registers) is written to the other; one barrier per tile.
    // The caller's previous use of the buffers must be finished: barrier first.
    __syncthreads();
    fetch(t_begin);
    stage(0);
    __syncthreads();
    if (t_begin + BT < t_end) fetch(t_begin + BT);
    int cur = 0;
    for (long long m_tile = t_begin; m_tile < t_end; m_tile += BT, cur ^= 1) {
      const __bf16 *xs = xs_base + cur * BfTile<NP>::xs_elems;
      const __bf16 *xt = xt_base + cur * BfTile<NP>::xt_elems;
#pragma unroll
      for (int sub = 0; sub < BT / 32; ++sub) {
        if (m_tile + sub * 32 >= t_end) break;
        const int m0 = sub * 32;
        // Operand reads run three steps ahead of the MFMAs that use them (three
        // register buffers per GEMM, the second GEMM's first reads issued
        // before the cube), so each wait on LDS overlaps two steps of MFMA
        // work.  Scheduling fences keep that order: without them the scheduler
        // moves each read next to its use and every step waits on LDS.
        constexpr int S1 = NP / 16;      // GEMM1 steps (K = 16 features each)
        constexpr int S2 = NP / 16;      // GEMM2 steps (32 features x 16 samples each)
        constexpr int AH = 4;            // reads in flight
        auto ga = [&](int s) {
          return *reinterpret_cast<const bf16x8 *>(&xt[(m0 + li) * XTS + 16 * s + 8 * h]);
        };
        constexpr int NB = NP / 32;      // GEMM2 accumulators; step j: block j % NB, half j / NB
        auto gb = [&](int j) {
          const int nb = j % NB, q = j / NB;
          const __bf16 *src = &xs[(nb * 32 + li) * BSX + m0 + 16 * q + 4 * h];
          const bf16x4 lo = *reinterpret_cast<const bf16x4 *>(src);
          const bf16x4 hi = *reinterpret_cast<const bf16x4 *>(src + 8);
          bf16x8 a;
          a[0] = lo[0]; a[1] = lo[1]; a[2] = lo[2]; a[3] = lo[3];
          a[4] = hi[0]; a[5] = hi[1]; a[6] = hi[2]; a[7] = hi[3];
          return a;
        };
        // GEMM1 at raised wave priority: while one wave of a SIMD runs its
        // dependent MFMA chain, the other's cube and staging instructions do
        // not take its issue slots
        __builtin_amdgcn_s_setprio(1);
        f32x16 zacc[WK];
#pragma unroll
        for (int w = 0; w < WK; ++w) zacc[w] = f32x16{0.f};
        bf16x8 abuf[AH];
        // buffer s holds GEMM1 operand s, or for s >= S1 GEMM2 operand s - S1
#pragma unroll
        for (int s = 0; s < AH; ++s) {
          if (s < S1) abuf[s] = ga(s);
          else if (s - S1 < S2) abuf[s] = gb(s - S1);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < S1; ++s) {
          const bf16x8 a = abuf[s % AH];
#pragma unroll
          for (int w = 0; w < WK; ++w) {
            zacc[w] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, breg[w][s], zacc[w], 0, 0, 0);
            if constexpr (LO)
              zacc[w] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, blo[w][s], zacc[w], 0, 0, 0);
          }
          __builtin_amdgcn_sched_barrier(0);
          if (s + AH < S1) abuf[s % AH] = ga(s + AH);
          else if (s + AH - S1 < S2) abuf[s % AH] = gb(s + AH - S1);
          __builtin_amdgcn_sched_barrier(0);
        }
        __builtin_amdgcn_s_setprio(0);
        bf16x8 p3[WK][2];
#pragma unroll
        for (int w = 0; w < WK; ++w) {
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const float z = zacc[w][v];
            const float z2 = z * z;
            p3[w][v / 8][v % 8] = (__bf16)(z2 * z);
            if constexpr (S4) s4acc[w] = fmaf(z2, z2, s4acc[w]);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
        // GEMM2 operand j sits in abuf[(S1 + j) % AH]
#pragma unroll
        for (int j = 0; j < S2; ++j) {
          const bf16x8 a = abuf[(S1 + j) % AH];
#pragma unroll
          for (int w = 0; w < WK; ++w)
            gacc[w][j % NB] =
                __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, p3[w][j / NB], gacc[w][j % NB], 0, 0, 0);
          __builtin_amdgcn_sched_barrier(0);
          if (j + AH < S2) abuf[(S1 + j) % AH] = gb(j + AH);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      if (m_tile + BT < t_end) stage(cur ^ 1);
      __syncthreads();
      if (m_tile + 2 * BT < t_end) fetch(m_tile + 2 * BT);
    }

#pragma unroll
    for (int w = 0; w < WK; ++w) {
      const float tot = s4acc[w] + __shfl_xor(s4acc[w], 32);
      if (pos[w] < kact) {
        if (h == 0 && s4part) s4part[(size_t)sp * rows_pad + pos[w]] = S4 ? tot : 0.f;
        g_f32 *dst = gpart + ((size_t)sp * rows_pad + pos[w]) * NP;
#pragma unroll
        for (int nb = 0; nb < NP / 32; ++nb) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            f32x4 v4;
            v4[0] = gacc[w][nb][4 * q + 0];
            v4[1] = gacc[w][nb][4 * q + 1];
            v4[2] = gacc[w][nb][4 * q + 2];
            v4[3] = gacc[w][nb][4 * q + 3];
            *reinterpret_cast<g_f32x4 *>(dst + nb * 32 + 8 * q + 4 * h) = v4;
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Wave reductions (64 lanes).
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

}  // namespace oica
