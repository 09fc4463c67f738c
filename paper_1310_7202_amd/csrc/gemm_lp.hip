// Low-precision MFMA GEMM for the mixed-precision form of Algorithm 4.1
// (Shabat et al., Section 4): the two products with A,
//   Step 2   Y = A G        and      Step 5   C = L_y^T P A = Lv^T A,
// run on BF16 (or FP16) matrix cores with FP32 accumulation, while the
// pivoted LUs, the Gram matrix and its inverse stay in FP64.
//
// Operands are read in their storage type (FP32 A and G, FP64 Lv) and
// rounded to the 16-bit type in registers on the way to LDS, so no
// low-precision copy of A is ever written.  The unit-lower factor Lv can be
// carried as a pair hi + lo of 16-bit numbers (hi = round(x),
// lo = round(x - hi)), two MFMAs per fragment: rounding Lv alone to 8
// significant bits perturbs the projection by about u kappa(L_y) sqrt(k/m)
// ||A||, which the pair reduces by another factor u.
//
// Tiles: 64 x 64 outputs per workgroup of four waves (2 x 2, each 32 x 32 =
// 2 x 2 MFMA 16x16x32 tiles), K slices of 32 staged in LDS as [row][k]
// (k contiguous, so each lane fetches its 8 consecutive k with one 16-byte
// LDS read), register prefetch of the next slice, two LDS buffers.
// MFMA 16x16x32 (bf16 / f16) layout: lane i + 16 g holds row i, k 8g..8g+7
// of either operand; lane l, slot v of the result holds D[4(l/16) + v][l%16].
#include "rlu_device.h"
#include "rlu_kernels.h"

#include <climits>

#include <algorithm>
#include <type_traits>

namespace rlu {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <typename LP> struct LpMfma;
template <> struct LpMfma<__bf16> {
  typedef bf16x8 vec;
  static __device__ __forceinline__ f4 mma(vec a, vec b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct LpMfma<_Float16> {
  typedef f16x8 vec;
  static __device__ __forceinline__ f4 mma(vec a, vec b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

constexpr int LBK = 32;      // K slice
constexpr int LPAD = 8;      // row padding (16 bytes keeps rows 16-byte aligned)
constexpr int LLD = LBK + LPAD;

template <typename LP, typename TA, typename TB, typename TO, OpA OA, bool SPLIT, int BM, int BN,
          int WM, int WN>
__device__ __forceinline__ void gemm_lp_tile(int64_t M, int64_t N, int64_t K,
                                             const TA* __restrict__ A, int64_t lda,
                                             const int* __restrict__ astep,
                                             const TB* __restrict__ B, int64_t ldb,
                                             TO* __restrict__ C, int64_t ldc, int ksplit,
                                             TO* __restrict__ partial, int bx, int by, int bz,
                                             const unsigned* __restrict__ amax) {
  // A's range scale (FP16): the FP32 matrix is operand A of Y = A G and
  // operand B of C = Lv^T A; undone on the output
  const float asc = lp_scale(amax);
  const float sa = OA == OpA::Plain ? asc : 1.f, sb = OA == OpA::Plain ? 1.f : asc;
  constexpr int NT = 64 * WM * WN;
  constexpr int WTM = BM / WM, WTN = BN / WN, TM = WTM / 16, TN = WTN / 16;
  constexpr int AE = BM * LBK / NT, BE = BN * LBK / NT;
  constexpr int NS = SPLIT ? 2 : 1;
  static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tile");
  static_assert((BM * LBK) % NT == 0 && (BN * LBK) % NT == 0, "tile vs threads");
  typedef typename LpMfma<LP>::vec vec;
  __shared__ __attribute__((aligned(16))) LP As[2][NS][BM * LLD];
  __shared__ __attribute__((aligned(16))) LP Bs[2][BN * LLD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int64_t m0 = (int64_t)bx * BM, n0 = (int64_t)by * BN;
  const int64_t kchunk = ((K + ksplit - 1) / ksplit + LBK - 1) / LBK * LBK;
  const int64_t kbeg = (int64_t)bz * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;

  // raw (storage-type) prefetch registers: conversion and the Lv mapping
  // are applied at the LDS store, after the MFMAs of the current slice, so
  // that no load of the next slice is waited for early
  static_assert(NT % LBK == 0, "a thread's K row is the same for all its elements");
  TA ra[AE];
  TB rb[BE];
  int sa1 = 0;  // Lv^T A: the step of this thread's K row

  auto a_pos = [&](int q, int& i, int& kk) {
    const int e = tid + q * NT;
    if (OA == OpA::LvT) { kk = e % LBK; i = e / LBK; } else { i = e % BM; kk = e / BM; }
  };
  auto load = [&](int64_t k0) {
    if (OA == OpA::LvT) {
      const int64_t gk = k0 + tid % LBK;
      sa1 = gk < kend ? astep[gk] : 0;
    }
#pragma unroll
    for (int q = 0; q < AE; ++q) {
      int i, kk;
      a_pos(q, i, kk);
      const int64_t gi = m0 + i, gk = k0 + kk;
      TA v = TA(0);
      if (gi < M && gk < kend) v = OA == OpA::Plain ? A[gi + gk * lda] : A[gk + gi * lda];
      ra[q] = v;
    }
#pragma unroll
    for (int q = 0; q < BE; ++q) {
      const int e = tid + q * NT;
      const int kk = e % LBK, j = e / LBK;
      const int64_t gj = n0 + j, gk = k0 + kk;
      rb[q] = (gj < N && gk < kend) ? B[gk + gj * ldb] : TB(0);
    }
  };
  auto store = [&](int buf, int64_t k0) {
#pragma unroll
    for (int q = 0; q < AE; ++q) {
      int i, kk;
      a_pos(q, i, kk);
      double xd;
      if (OA == OpA::Plain) {
        xd = (double)((float)ra[q] * sa);
      } else {
        const int64_t gi = m0 + i, gk = k0 + kk;
        xd = (gi < M && gk < kend) ? (double)lv_value<TA>(ra[q], (int)gi, sa1) : 0.0;
      }
      const float x = (float)xd;
      const LP hi = (LP)x;
      As[buf][0][i * LLD + kk] = hi;
      if (SPLIT) As[buf][NS - 1][i * LLD + kk] = (LP)(float)(xd - (double)(float)hi);
    }
#pragma unroll
    for (int q = 0; q < BE; ++q) {
      const int e = tid + q * NT;
      const int kk = e % LBK, j = e / LBK;
      Bs[buf][j * LLD + kk] = (LP)((float)rb[q] * sb);
    }
  };

  f4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

  int buf = 0;
  if (kbeg < kend) {
    load(kbeg);
    store(0, kbeg);
  }
  __syncthreads();
  for (int64_t kt = kbeg; kt < kend; kt += LBK) {
    const bool more = kt + LBK < kend;
    if (more) load(kt + LBK);
    const int kof = 8 * (lane >> 4);
    vec af[NS][TM], bf[TN];
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      const int row = wm * WTM + a * 16 + (lane & 15);
#pragma unroll
      for (int s2 = 0; s2 < NS; ++s2) af[s2][a] = *(const vec*)&As[buf][s2][row * LLD + kof];
    }
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int col = wn * WTN + b * 16 + (lane & 15);
      bf[b] = *(const vec*)&Bs[buf][col * LLD + kof];
    }
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        acc[a][b] = LpMfma<LP>::mma(af[0][a], bf[b], acc[a][b]);
        if (SPLIT) acc[a][b] = LpMfma<LP>::mma(af[NS - 1][a], bf[b], acc[a][b]);
      }
    if (more) store(buf ^ 1, kt + LBK);
    __syncthreads();
    buf ^= 1;
  }

#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gi = m0 + wm * WTM + a * 16 + 4 * (lane >> 4) + v;
        const int64_t gj = n0 + wn * WTN + b * 16 + (lane & 15);
        if (gi < M && gj < N) {
          const TO val = (TO)((double)acc[a][b][v] / (double)asc);
          if (ksplit > 1) partial[(int64_t)bz * M * N + gi + gj * M] = val;
          else C[gi + gj * ldc] = val;
        }
      }
}

// Workgroup b runs on XCD b mod 8: each XCD takes a contiguous range of
// tiles, ordered so that consecutive tiles share the larger operand (N index
// fastest when A is larger, else M), which is then read from HBM once.
__device__ __forceinline__ int xcd_chunked_lp(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

template <typename LP, typename TA, typename TB, typename TO, OpA OA, bool SPLIT, int BM, int BN,
          int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN)
gemm_lp_kernel(int64_t M, int64_t N, int64_t K, const TA* __restrict__ A, int64_t lda,
               const int* __restrict__ astep, const TB* __restrict__ B, int64_t ldb,
               TO* __restrict__ C, int64_t ldc, int ksplit, TO* __restrict__ partial, int tm,
               int tn, int nfast, const unsigned* __restrict__ amax) {
  const int t = xcd_chunked_lp((int)blockIdx.x, (int)gridDim.x);
  int bx, by, bz;
  if (nfast) {
    by = t % tn; const int rest = t / tn; bx = rest % tm; bz = rest / tm;
  } else {
    bx = t % tm; const int rest = t / tm; by = rest % tn; bz = rest / tn;
  }
  gemm_lp_tile<LP, TA, TB, TO, OA, SPLIT, BM, BN, WM, WN>(M, N, K, A, lda, astep, B, ldb, C, ldc,
                                                          ksplit, partial, bx, by, bz, amax);
}

// Grouped form: workgroup b computes the tile map[b] = (task, bx + tiles_m by)
// of one of many independent products (no split-K).
template <typename LP, typename TA, typename TB, typename TO, OpA OA, bool SPLIT, int BM, int BN,
          int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN)
gemm_lp_grouped_kernel(const GemmTaskDev* __restrict__ tasks, const int2* __restrict__ map) {
  const int2 e = map[blockIdx.x];
  if (e.x < 0) return;  // padding of the XCD layout
  const GemmTaskDev& t = tasks[e.x];
  const int bx = e.y % t.tiles_m, by = e.y / t.tiles_m;
  gemm_lp_tile<LP, TA, TB, TO, OA, SPLIT, BM, BN, WM, WN>(
      t.M, t.N, t.K, (const TA*)t.A, t.lda, t.astep, (const TB*)t.B, t.ldb, (TO*)t.C, t.ldc, 1,
      nullptr, bx, by, 0, t.amax);
}

// ---------------------------------------------------------------------------
// Large-tile form for long products (K >= 1024, thousands of rows or
// columns): 128-row tiles, vectorized global loads (4 consecutive elements
// per load along the operand's contiguous dimension), the 16-bit values
// written to LDS 4 at a time (8 bytes), so the per-element LDS stores and
// scalar loads of the small-tile form no longer bound the kernel.
//   * A of Step 2 (FP32, M contiguous): a thread loads a 4 x 4 block (4 rows
//     at 4 consecutive k, four 16-byte loads) and writes each row's 4 k.
//   * Lv^T of Step 5 (FP64 Y, K contiguous): 4 consecutive k of one output
//     row (two 16-byte loads), masked by the rows' choosing steps, split
//     into hi + lo.
//   * B operands (FP32, K contiguous): 4 consecutive k of one column.
// Vector loads need 16-byte aligned leading dimensions; the launcher falls
// back to the small-tile form otherwise.
// ---------------------------------------------------------------------------
template <typename LP, typename TA, OpA OA, bool SPLIT, int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN)
gemm_lp2_kernel(int64_t M, int64_t N, int64_t K, const TA* __restrict__ A, int64_t lda,
                const int* __restrict__ astep, const float* __restrict__ B, int64_t ldb,
                double* __restrict__ C, int64_t ldc, int ksplit, double* __restrict__ partial,
                int tm, int tn, int nfast, const unsigned* __restrict__ amax) {
  constexpr int NT = 64 * WM * WN;
  // A's range scale (FP16), as in the small-tile form
  const float asc = lp_scale(amax);
  const float sa = OA == OpA::Plain ? asc : 1.f, sb = OA == OpA::Plain ? 1.f : asc;
  constexpr int WTM = BM / WM, WTN = BN / WN, TM = WTM / 16, TN = WTN / 16;
  constexpr int NS = SPLIT ? 2 : 1;
  // loads per thread per K slice
  constexpr int ACH = (OA == OpA::Plain) ? (BM * LBK / 16) / NT : (BM * LBK / 4) / NT;
  constexpr int BCH = (BN * LBK / 4) / NT;
  static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tile");
  static_assert(ACH * NT == ((OA == OpA::Plain) ? BM * LBK / 16 : BM * LBK / 4), "A chunks");
  static_assert(BCH * NT == BN * LBK / 4, "B chunks");
  typedef typename LpMfma<LP>::vec vec;
  typedef LP lp4 __attribute__((ext_vector_type(4)));
  __shared__ __attribute__((aligned(16))) LP As[2][NS][BM * LLD];
  __shared__ __attribute__((aligned(16))) LP Bs[2][BN * LLD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int t = xcd_chunked_lp((int)blockIdx.x, (int)gridDim.x);
  int bx, by, bz;
  if (nfast) {
    by = t % tn; const int rest = t / tn; bx = rest % tm; bz = rest / tm;
  } else {
    bx = t % tm; const int rest = t / tm; by = rest % tn; bz = rest / tn;
  }
  const int64_t m0 = (int64_t)bx * BM, n0 = (int64_t)by * BN;
  const int64_t kchunk = ((K + ksplit - 1) / ksplit + LBK - 1) / LBK * LBK;
  const int64_t kbeg = (int64_t)bz * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;

  // prefetch registers: A as FP32 values (Plain) or FP64 (LvT)
  typedef typename std::conditional<OA == OpA::Plain, float, double>::type RA;
  RA ra[ACH][(OA == OpA::Plain) ? 16 : 4];
  int rs[(OA == OpA::Plain) ? 1 : ACH][4];  // Lv^T: the steps of the loaded K rows
  float rb[BCH][4];

  auto load = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < ACH; ++q) {
      const int e = tid + q * NT;
      if (OA == OpA::Plain) {
        // 4 x 4 block: rows 4 (e % (BM/4)) .., k 4 (e / (BM/4)) ..
        const int i4 = 4 * (e % (BM / 4)), k4 = 4 * (e / (BM / 4));
        const int64_t gi = m0 + i4;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int64_t gk = k0 + k4 + c;
          if (gk < kend && gi + 3 < M) {
            const float4 v = *(const float4*)&A[gi + gk * lda];
            ra[q][4 * c + 0] = v.x; ra[q][4 * c + 1] = v.y;
            ra[q][4 * c + 2] = v.z; ra[q][4 * c + 3] = v.w;
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              ra[q][4 * c + r] = (gk < kend && gi + r < M) ? (float)A[gi + r + gk * lda] : 0.f;
          }
        }
      } else {
        // 4 consecutive k of output row i, as stored, with their steps (the
        // Lv mapping is applied at the LDS store)
        const int kk4 = 4 * (e % (LBK / 4)), i = e / (LBK / 4);
        const int64_t gi = m0 + i, gk = k0 + kk4;
        if (gi < M && gk + 3 < kend) {
          const double2 v0 = *(const double2*)&A[gk + gi * lda];
          const double2 v1 = *(const double2*)&A[gk + 2 + gi * lda];
          const int4 s4 = *(const int4*)&astep[gk];
          ra[q][0] = v0.x; ra[q][1] = v0.y; ra[q][2] = v1.x; ra[q][3] = v1.y;
          rs[q][0] = s4.x; rs[q][1] = s4.y; rs[q][2] = s4.z; rs[q][3] = s4.w;
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const bool in = gi < M && gk + c < kend;
            ra[q][c] = in ? (double)A[gk + c + gi * lda] : 0.0;
            rs[q][c] = in ? astep[gk + c] : INT_MIN;  // INT_MIN: outside, maps to 0
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < BCH; ++q) {
      const int e = tid + q * NT;
      const int kk4 = 4 * (e % (LBK / 4)), j = e / (LBK / 4);
      const int64_t gj = n0 + j, gk = k0 + kk4;
      if (gj < N && gk + 3 < kend) {
        const float4 v = *(const float4*)&B[gk + gj * ldb];
        rb[q][0] = v.x; rb[q][1] = v.y; rb[q][2] = v.z; rb[q][3] = v.w;
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) rb[q][c] = (gj < N && gk + c < kend) ? B[gk + c + gj * ldb] : 0.f;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < ACH; ++q) {
      const int e = tid + q * NT;
      if (OA == OpA::Plain) {
        const int i4 = 4 * (e % (BM / 4)), k4 = 4 * (e / (BM / 4));
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          lp4 h;
          h.x = (LP)(ra[q][r] * sa); h.y = (LP)(ra[q][4 + r] * sa);
          h.z = (LP)(ra[q][8 + r] * sa); h.w = (LP)(ra[q][12 + r] * sa);
          *(lp4*)&As[buf][0][(i4 + r) * LLD + k4] = h;
        }
      } else {
        const int kk4 = 4 * (e % (LBK / 4)), i = e / (LBK / 4);
        const int gi = (int)(m0 + i);
        lp4 h, l;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double xd = lv_value<double>(ra[q][c], gi, rs[q][c]);
          const float x = (float)xd;
          const LP hi = (LP)x;
          h[c] = hi;
          l[c] = (LP)(float)(xd - (double)(float)hi);
        }
        *(lp4*)&As[buf][0][i * LLD + kk4] = h;
        if (SPLIT) *(lp4*)&As[buf][NS - 1][i * LLD + kk4] = l;
      }
    }
#pragma unroll
    for (int q = 0; q < BCH; ++q) {
      const int e = tid + q * NT;
      const int kk4 = 4 * (e % (LBK / 4)), j = e / (LBK / 4);
      lp4 h;
      h.x = (LP)(rb[q][0] * sb); h.y = (LP)(rb[q][1] * sb);
      h.z = (LP)(rb[q][2] * sb); h.w = (LP)(rb[q][3] * sb);
      *(lp4*)&Bs[buf][j * LLD + kk4] = h;
    }
  };

  f4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

  int buf = 0;
  if (kbeg < kend) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  for (int64_t kt = kbeg; kt < kend; kt += LBK) {
    const bool more = kt + LBK < kend;
    if (more) load(kt + LBK);
    const int kof = 8 * (lane >> 4);
    vec af[NS][TM], bf[TN];
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      const int row = wm * WTM + a * 16 + (lane & 15);
#pragma unroll
      for (int s2 = 0; s2 < NS; ++s2) af[s2][a] = *(const vec*)&As[buf][s2][row * LLD + kof];
    }
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int col = wn * WTN + b * 16 + (lane & 15);
      bf[b] = *(const vec*)&Bs[buf][col * LLD + kof];
    }
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        acc[a][b] = LpMfma<LP>::mma(af[0][a], bf[b], acc[a][b]);
        if (SPLIT) acc[a][b] = LpMfma<LP>::mma(af[NS - 1][a], bf[b], acc[a][b]);
      }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gi = m0 + wm * WTM + a * 16 + 4 * (lane >> 4) + v;
        const int64_t gj = n0 + wn * WTN + b * 16 + (lane & 15);
        if (gi < M && gj < N) {
          const double val = (double)acc[a][b][v] / (double)asc;
          if (ksplit > 1) partial[(int64_t)bz * M * N + gi + gj * M] = val;
          else C[gi + gj * ldc] = val;
        }
      }
}

template <typename LP, typename TA, OpA OA, bool SPLIT, int BM, int BN, int WM, int WN>
hipError_t launch_lp2(const GemmDesc& d, hipStream_t s) {
  const int tm = (int)((d.M + BM - 1) / BM), tn = (int)((d.N + BN - 1) / BN);
  const int64_t tiles = (int64_t)tm * tn;
  int ks = 1;
  if (d.partial)
    while (tiles * ks < 512 && d.K / (ks * 2) >= 2048 && ks < 16) ks *= 2;
  if (d.ksplit_out) *d.ksplit_out = ks;
  const int nfast = d.M > d.N ? 1 : 0;
  hipLaunchKernelGGL((gemm_lp2_kernel<LP, TA, OA, SPLIT, BM, BN, WM, WN>),
                     dim3((unsigned)(tiles * ks)), dim3(64 * WM * WN), 0, s, d.M, d.N, d.K,
                     (const TA*)d.A, d.lda, d.astep, (const float*)d.B, d.ldb, (double*)d.C,
                     d.ldc, ks, (double*)d.partial, tm, tn, nfast, d.amax);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ks == 1 || d.no_sum) return e;
  return launch_splitk_sum_f64(d.M, d.N, ks, (const double*)d.partial, (double*)d.C, d.ldc,
                               nullptr, s);
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

template <typename LP, typename TA, typename TB, OpA OA, bool SPLIT>
hipError_t launch_lp(const GemmDesc& d, hipStream_t s) {
  constexpr int BM = 64, BN = 64, WM = 2, WN = 2;
  const int64_t tiles = ((d.M + BM - 1) / BM) * ((d.N + BN - 1) / BN);
  int ks = 1;
  if (d.partial)
    while (tiles * ks < 1024 && d.K / (ks * 2) >= 1024 && ks < 32) ks *= 2;
  const int tm = (int)((d.M + BM - 1) / BM), tn = (int)((d.N + BN - 1) / BN);
  const int nfast = d.M > d.N ? 1 : 0;
  hipLaunchKernelGGL((gemm_lp_kernel<LP, TA, TB, double, OA, SPLIT, BM, BN, WM, WN>),
                     dim3((unsigned)((int64_t)tm * tn * ks)), dim3(64 * WM * WN), 0, s, d.M, d.N,
                     d.K, (const TA*)d.A, d.lda, d.astep, (const TB*)d.B, d.ldb, (double*)d.C,
                     d.ldc, ks, (double*)d.partial, tm, tn, nfast, d.amax);
  if (d.ksplit_out) *d.ksplit_out = ks;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ks == 1 || d.no_sum) return e;
  return launch_splitk_sum_f64(d.M, d.N, ks, (const double*)d.partial, (double*)d.C, d.ldc,
                               nullptr, s);
}

}  // namespace

size_t gemm_lp_partial_elems(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64);
  int ks = 1;
  while (tiles * ks < 1024 && K / (ks * 2) >= 1024 && ks < 32) ks *= 2;
  // the large-tile form: 128-row tiles, fewer tiles, its own split rule
  const int64_t t2 = std::min(((M + 127) / 128) * ((N + 191) / 192),
                              ((M + 127) / 128) * ((N + 127) / 128));
  int ks2 = 1;
  while (t2 * ks2 < 512 && K / (ks2 * 2) >= 2048 && ks2 < 16) ks2 *= 2;
  ks = std::max(ks, ks2);
  size_t elems = ks > 1 ? (size_t)ks * (size_t)M * (size_t)N : 0;
  elems = std::max(elems, stream_sketch_partial_elems(M, N, K));
  return std::max(elems, stream_project_partial_elems(M, N, K));
}

hipError_t launch_gemm_lp(const GemmDesc& d, bool fp16, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0) return hipSuccess;
  if (d.opb != OpB::Plain) return hipErrorInvalidValue;
  if (stream_sketch_applies(d)) return launch_sketch_stream_lp(d, fp16, s);
  if (stream_project_applies(d)) return launch_project_stream_lp(d, fp16, s);
  const bool bvec = d.ldb % 4 == 0 && aligned16(d.B);
  if (d.opa == OpA::Plain && d.K >= 1024 && d.M >= 1024 && bvec && d.lda % 4 == 0 &&
      aligned16(d.A)) {
    return fp16 ? launch_lp2<_Float16, float, OpA::Plain, false, 128, 192, 4, 1>(d, s)
                : launch_lp2<__bf16, float, OpA::Plain, false, 128, 192, 4, 1>(d, s);
  }
  if (d.opa == OpA::LvT && d.K >= 1024 && d.N >= 1024 && bvec && d.lda % 2 == 0 &&
      aligned16(d.A) && aligned16(d.astep)) {
    return fp16 ? launch_lp2<_Float16, double, OpA::LvT, true, 128, 128, 2, 2>(d, s)
                : launch_lp2<__bf16, double, OpA::LvT, true, 128, 128, 2, 2>(d, s);
  }
  if (d.opa == OpA::Plain) {  // Y = A G: FP32 A and G
    return fp16 ? launch_lp<_Float16, float, float, OpA::Plain, false>(d, s)
                : launch_lp<__bf16, float, float, OpA::Plain, false>(d, s);
  }
  if (d.opa == OpA::LvT) {    // C = Lv^T A: FP64 Lv as a hi + lo pair, FP32 A
    return fp16 ? launch_lp<_Float16, double, float, OpA::LvT, true>(d, s)
                : launch_lp<__bf16, double, float, OpA::LvT, true>(d, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gemm_lp_grouped(OpA opa, bool fp16, const GemmTaskDev* tasks, const int2* map,
                                  int nwg, hipStream_t s) {
  if (nwg <= 0) return hipSuccess;
#define RLU_LPG(LP, TA, OA, SPLIT)                                                              \
  hipLaunchKernelGGL((gemm_lp_grouped_kernel<LP, TA, float, double, OA, SPLIT, 64, 64, 2, 2>), \
                     dim3((unsigned)nwg), dim3(256), 0, s, tasks, map)
  if (opa == OpA::Plain) {
    if (fp16) RLU_LPG(_Float16, float, OpA::Plain, false);
    else RLU_LPG(__bf16, float, OpA::Plain, false);
  } else if (opa == OpA::LvT) {
    if (fp16) RLU_LPG(_Float16, double, OpA::LvT, true);
    else RLU_LPG(__bf16, double, OpA::LvT, true);
  } else {
    return hipErrorInvalidValue;
  }
#undef RLU_LPG
  return hipGetLastError();
}

}  // namespace rlu
