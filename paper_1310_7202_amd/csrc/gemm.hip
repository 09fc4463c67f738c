// MFMA GEMM for the dense products of Algorithm 4.1 (Shabat et al.,
// Section 4):
//   Step 2   Y   = A G                      (M = m, N = l, K = n)
//   Step 5   C   = L_y^T P A  computed as Lv^T A in original row order
//            S   = L_y^T L_y  = Lv^T Lv     (Gram matrix of the Remark)
//            B   = S^{-1} C
//   Step 7   L   = L_y L_b    = P (Lv L_b)  (rows scattered to positions)
// where Lv is the unit-lower factor of Step 3 read in place (see
// lv_value in rlu_device.h): the permutation P never touches A.
//
// One kernel template: a workgroup computes a BM x BN tile of C with 16x16x4
// MFMA tiles, staging BK = 16 deep slices of both operands through LDS with
// register double buffering (global loads of slice t+1 overlap the MFMAs of
// slice t).  Operands may be converted on load (TA, TB -> TC), the output is
// written in TO.  Optional split-K writes per-split partial sums that a
// second kernel adds in a fixed order, so results never depend on timing.
#include "rlu_device.h"
#include "rlu_kernels.h"

namespace rlu {
namespace {

constexpr int BK = 16;

template <typename TC, int BM, int BN, int WM, int WN>
struct Tile {
  static constexpr int NT = 64 * WM * WN;
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int TM = WTM / 16, TN = WTN / 16;
  static constexpr int APAD = 2, BPAD = 2;
  static constexpr int AL = BM + APAD, BL = BN + BPAD;
  static constexpr int AE = BM * BK / NT, BE = BN * BK / NT;
  static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tile must be a multiple of 16");
  static_assert((BM * BK) % NT == 0 && (BN * BK) % NT == 0, "tile must divide threads");
};

template <typename TA, typename TB, typename TC, typename TO, int BM, int BN, int WM, int WN,
          OpA OA, OpB OB>
__global__ void __launch_bounds__(64 * WM * WN)
gemm_kernel(int64_t M, int64_t N, int64_t K, const TA* __restrict__ A, int64_t lda,
            const int* __restrict__ astep, const TB* __restrict__ B, int64_t ldb,
            const int* __restrict__ bstep, TO* __restrict__ C, int64_t ldc,
            const int* __restrict__ rowmap, int ksplit, TO* __restrict__ partial) {
  typedef Tile<TC, BM, BN, WM, WN> Tl;
  typedef Mfma<TC> MF;
  __shared__ TC As[2][BK][Tl::AL];
  __shared__ TC Bs[2][BK][Tl::BL];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int64_t m0 = (int64_t)blockIdx.x * BM;
  const int64_t n0 = (int64_t)blockIdx.y * BN;
  // K range of this split (multiples of BK)
  const int64_t kchunk = ((K + ksplit - 1) / ksplit + BK - 1) / BK * BK;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;

  TC ra[Tl::AE], rb[Tl::BE];

  auto load = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < Tl::AE; ++q) {
      const int e = tid + q * Tl::NT;
      int i, kk;
      if (OA == OpA::LvT) { kk = e % BK; i = e / BK; } else { i = e % BM; kk = e / BM; }
      const int64_t gi = m0 + i, gk = k0 + kk;
      TC v = TC(0);
      if (gi < M && gk < kend) {
        if (OA == OpA::Plain) {
          v = (TC)A[gi + gk * lda];
        } else if (OA == OpA::LvT) {
          v = (TC)lv_value<TA>(A[gk + gi * lda], (int)gi, astep[gk]);
        } else {
          v = (TC)lv_value<TA>(A[gi + gk * lda], (int)gk, astep[gi]);
        }
      }
      ra[q] = v;
    }
#pragma unroll
    for (int q = 0; q < Tl::BE; ++q) {
      const int e = tid + q * Tl::NT;
      const int kk = e % BK, j = e / BK;
      const int64_t gj = n0 + j, gk = k0 + kk;
      TC v = TC(0);
      if (gj < N && gk < kend) {
        if (OB == OpB::Plain) v = (TC)B[gk + gj * ldb];
        else v = (TC)lv_value<TB>(B[gk + gj * ldb], (int)gj, bstep[gk]);
      }
      rb[q] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < Tl::AE; ++q) {
      const int e = tid + q * Tl::NT;
      int i, kk;
      if (OA == OpA::LvT) { kk = e % BK; i = e / BK; } else { i = e % BM; kk = e / BM; }
      As[buf][kk][i] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < Tl::BE; ++q) {
      const int e = tid + q * Tl::NT;
      const int kk = e % BK, j = e / BK;
      Bs[buf][kk][j] = rb[q];
    }
  };

  typename MF::acc_t acc[Tl::TM][Tl::TN];
#pragma unroll
  for (int a = 0; a < Tl::TM; ++a)
#pragma unroll
    for (int b = 0; b < Tl::TN; ++b) acc[a][b] = MF::zero();

  int buf = 0;
  if (kbeg < kend) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  for (int64_t kt = kbeg; kt < kend; kt += BK) {
    const bool more = kt + BK < kend;
    if (more) load(kt + BK);
#pragma unroll
    for (int k4 = 0; k4 < BK / 4; ++k4) {
      const int kr = k4 * 4 + (lane >> 4);
      TC af[Tl::TM], bf[Tl::TN];
#pragma unroll
      for (int a = 0; a < Tl::TM; ++a) af[a] = As[buf][kr][wm * Tl::WTM + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < Tl::TN; ++b) bf[b] = Bs[buf][kr][wn * Tl::WTN + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < Tl::TM; ++a)
#pragma unroll
        for (int b = 0; b < Tl::TN; ++b) acc[a][b] = MF::mma(af[a], bf[b], acc[a][b]);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // epilogue
#pragma unroll
  for (int a = 0; a < Tl::TM; ++a)
#pragma unroll
    for (int b = 0; b < Tl::TN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gi = m0 + wm * Tl::WTM + a * 16 + MF::row(lane, v);
        const int64_t gj = n0 + wn * Tl::WTN + b * 16 + (lane & 15);
        if (gi < M && gj < N) {
          const TO val = (TO)acc[a][b][v];
          if (ksplit > 1) {
            partial[(int64_t)blockIdx.z * M * N + gi + gj * M] = val;
          } else {
            const int64_t oi = rowmap ? (int64_t)rowmap[gi] : gi;
            C[oi + gj * ldc] = val;
          }
        }
      }
}

template <typename TO>
__global__ void __launch_bounds__(256) splitk_sum_kernel(int64_t M, int64_t N, int ksplit,
                                                         const TO* __restrict__ partial,
                                                         TO* __restrict__ C, int64_t ldc,
                                                         const int* __restrict__ rowmap) {
  const int64_t total = M * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    TO s = partial[e];
    for (int z = 1; z < ksplit; ++z) s += partial[(int64_t)z * total + e];  // fixed order
    const int64_t i = e % M, j = e / M;
    const int64_t oi = rowmap ? (int64_t)rowmap[i] : i;
    C[oi + j * ldc] = s;
  }
}

struct Cfg { int bm, bn; };

// Pick the tile shape that finishes first on 256 CUs: time ~ (rounds of 256
// tiles) x (tile area); ties go to the shape with more tiles.
Cfg choose_cfg(int64_t M, int64_t N) {
  const Cfg cands[3] = {{64, 64}, {64, 112}, {112, 64}};
  Cfg best = cands[0];
  double best_cost = 1e300, best_tiles = 0;
  for (const Cfg& c : cands) {
    const double tiles = (double)((M + c.bm - 1) / c.bm) * (double)((N + c.bn - 1) / c.bn);
    const double rounds = (double)(((int64_t)tiles + 255) / 256);
    const double cost = rounds * c.bm * c.bn;
    if (cost < best_cost || (cost == best_cost && tiles > best_tiles)) {
      best_cost = cost; best = c; best_tiles = tiles;
    }
  }
  return best;
}

template <typename TA, typename TB, typename TC, typename TO, int BM, int BN, int WM, int WN,
          OpA OA, OpB OB>
hipError_t launch_cfg(const GemmDesc& d, int ksplit, hipStream_t s) {
  dim3 grid((unsigned)((d.M + BM - 1) / BM), (unsigned)((d.N + BN - 1) / BN), (unsigned)ksplit);
  hipLaunchKernelGGL((gemm_kernel<TA, TB, TC, TO, BM, BN, WM, WN, OA, OB>), grid,
                     dim3(64 * WM * WN), 0, s, d.M, d.N, d.K, (const TA*)d.A, d.lda, d.astep,
                     (const TB*)d.B, d.ldb, d.bstep, (TO*)d.C, d.ldc, d.rowmap, ksplit,
                     (TO*)d.partial);
  return hipGetLastError();
}

template <typename TA, typename TB, typename TC, typename TO, OpA OA, OpB OB>
hipError_t launch_ops(const GemmDesc& d, hipStream_t s) {
  const Cfg c = choose_cfg(d.M, d.N);
  const int ks = d.ksplit > 1 ? d.ksplit : 1;
  hipError_t e;
  if (c.bm == 64 && c.bn == 64)
    e = launch_cfg<TA, TB, TC, TO, 64, 64, 2, 2, OA, OB>(d, ks, s);
  else if (c.bm == 64)
    e = launch_cfg<TA, TB, TC, TO, 64, 112, 4, 1, OA, OB>(d, ks, s);
  else
    e = launch_cfg<TA, TB, TC, TO, 112, 64, 1, 4, OA, OB>(d, ks, s);
  if (e != hipSuccess || ks == 1) return e;
  const int64_t total = d.M * d.N;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(splitk_sum_kernel<TO>, dim3((unsigned)blocks), dim3(256), 0, s, d.M, d.N, ks,
                     (const TO*)d.partial, (TO*)d.C, d.ldc, d.rowmap);
  return hipGetLastError();
}

template <typename TA, typename TB, typename TC, typename TO>
hipError_t dispatch(const GemmDesc& d, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0) return hipSuccess;
  if (d.opa == OpA::Plain && d.opb == OpB::Plain)
    return launch_ops<TA, TB, TC, TO, OpA::Plain, OpB::Plain>(d, s);
  if (d.opa == OpA::LvT && d.opb == OpB::Plain)
    return launch_ops<TA, TB, TC, TO, OpA::LvT, OpB::Plain>(d, s);
  if (d.opa == OpA::LvT && d.opb == OpB::Lv)
    return launch_ops<TA, TB, TC, TO, OpA::LvT, OpB::Lv>(d, s);
  if (d.opa == OpA::Lv && d.opb == OpB::Plain)
    return launch_ops<TA, TB, TC, TO, OpA::Lv, OpB::Plain>(d, s);
  return hipErrorInvalidValue;
}

}  // namespace

size_t gemm_partial_elems(int64_t M, int64_t N, int ksplit) {
  return ksplit > 1 ? (size_t)ksplit * (size_t)M * (size_t)N : 0;
}

// FP64 path: every operand and the output in FP64.
template <>
hipError_t launch_gemm<double>(const GemmDesc& d, hipStream_t s) {
  return dispatch<double, double, double, double>(d, s);
}

}  // namespace rlu
