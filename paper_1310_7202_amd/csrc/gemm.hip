// MFMA GEMM for the dense products of Algorithm 4.1 (Shabat et al.,
// Section 4):
//   Step 2   Y   = A G                      (M = m, N = l, K = n)
//   Step 5   C   = L_y^T P A  computed as Lv^T A in original row order
//            S   = L_y^T L_y  = Lv^T Lv     (Gram matrix of the Remark)
//            B   = S^{-1} C
//   Step 7   L   = L_y L_b    = P (Lv L_b)  (rows scattered to positions)
// where Lv is the unit-lower factor of Step 3 read in place (see lv_value in
// rlu_device.h): the permutation P never touches A.
//
// One kernel template: a workgroup computes a BM x BN tile of C with 16x16x4
// MFMA tiles, staging BK-deep slices of both operands through LDS with
// register prefetch (global loads of slice t+1 overlap the MFMAs of slice t).
// Each operand is staged in the LDS layout that matches its contiguous
// dimension in HBM, so global reads stay long and coalesced:
//   * operand contiguous along M/N (A of Step 2): LDS [k][row]
//   * operand contiguous along K (both operands of Step 5): LDS [row][k],
//     and a deep slice (BK = 32) so each column is read in 256-byte runs.
// Operands may be converted on load (TA, TB -> TC), the output is written in
// TO.  Optional split-K writes per-split partial sums that a second kernel
// adds in a fixed order, so results never depend on timing.
#include "rlu_device.h"
#include "rlu_kernels.h"

#include <cstdlib>

namespace rlu {
namespace {

template <int BM, int BN, int BK, int WM, int WN, bool AK, bool BKC, int NBUF>
struct Tile {
  static constexpr int NT = 64 * WM * WN;
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int TM = WTM / 16, TN = WTN / 16;
  // LDS strides: [k][row] layout pads rows, [row][k] layout pads k
  static constexpr int A_LD = AK ? (BK + 2) : (BM + 2);
  static constexpr int B_LD = BKC ? (BK + 2) : (BN + 2);
  static constexpr int A_SZ = AK ? BM * A_LD : BK * A_LD;
  static constexpr int B_SZ = BKC ? BN * B_LD : BK * B_LD;
  static constexpr int AE = BM * BK / NT, BE = BN * BK / NT;
  static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tile must be a multiple of 16");
  static_assert((BM * BK) % NT == 0 && (BN * BK) % NT == 0, "tile must divide threads");
  static_assert(BK % 4 == 0, "BK multiple of the MFMA depth");
  static_assert(NT % BK == 0, "a thread's K row is the same for all its elements");
};

// One BM x BN output tile (bx, by) over K split bz of ksplit.
template <typename TA, typename TB, typename TC, typename TO, int BM, int BN, int BK, int WM,
          int WN, int NBUF, OpA OA, OpB OB>
__device__ __forceinline__ void gemm_tile(
    int64_t M, int64_t N, int64_t K, const TA* __restrict__ A, int64_t lda,
    const int* __restrict__ astep, const TB* __restrict__ B, int64_t ldb,
    const int* __restrict__ bstep, TO* __restrict__ C, int64_t ldc,
    const int* __restrict__ rowmap, int ksplit, TO* __restrict__ partial, int bx, int by,
    int bz, int acol0 = 0, int csub = 0, int blower = 0, int mirror = 0) {
  constexpr bool AK = (OA == OpA::LvT);  // A operand contiguous along K
  constexpr bool BKC = true;             // B operands are contiguous along K
  typedef Tile<BM, BN, BK, WM, WN, AK, BKC, NBUF> Tl;
  typedef Mfma<TC> MF;
  __shared__ TC As[NBUF][Tl::A_SZ];
  __shared__ TC Bs[NBUF][Tl::B_SZ];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int64_t m0 = (int64_t)bx * BM;
  const int64_t n0 = (int64_t)by * BN;
  // K range of this split (multiples of BK)
  const int64_t kchunk = ((K + ksplit - 1) / ksplit + BK - 1) / BK * BK;
  int64_t kbeg = (int64_t)bz * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
  // B lower triangular (B(t, j) = 0 for t < j): the tile's columns start at
  // n0, so the K slices wholly above row n0 add only exact zeros; skip them
  if (blower) {
    const int64_t kb = n0 / BK * BK;
    if (kb > kbeg) kbeg = kb;
  }

  // Prefetch registers hold the operands in their storage type: the
  // conversion, and the Lv mapping of the K-contiguous operands (one step
  // per thread), are applied when the slice is written to LDS, after the
  // MFMAs of the current slice, so that no load of the next slice is waited
  // for early.  (Lv and LvStrict operands, whose step varies per element,
  // are mapped on load.)
  TA ra[Tl::AE];
  TB rb[Tl::BE];
  int sa1 = 0, sb1 = 0;  // Lv^T A / Lv B: the step of this thread's K row

  // element q of this thread in the A tile: (row i, k kk)
  auto a_pos = [&](int q, int& i, int& kk) {
    const int e = tid + q * Tl::NT;
    if (AK) { kk = e % BK; i = e / BK; } else { i = e % BM; kk = e / BM; }
  };
  auto load = [&](int64_t k0) {
    if (OA == OpA::LvT) {
      const int64_t gk = k0 + tid % BK;  // the same K row for every element (NT % BK == 0)
      sa1 = gk < kend ? astep[gk] : 0;
    }
    if (OB == OpB::Lv) {
      const int64_t gk = k0 + tid % BK;
      sb1 = gk < kend ? bstep[gk] : 0;
    }
#pragma unroll
    for (int q = 0; q < Tl::AE; ++q) {
      int i, kk;
      a_pos(q, i, kk);
      const int64_t gi = m0 + i, gk = k0 + kk;
      TA v = TA(0);
      if (gi < M && gk < kend) {
        if (OA == OpA::Plain || OA == OpA::LvT) v = AK ? A[gk + gi * lda] : A[gi + gk * lda];
        else if (OA == OpA::Lv) v = lv_value<TA>(A[gi + gk * lda], (int)gk, astep[gi]);
        else v = (int)(acol0 + gk) < astep[gi] ? A[gi + gk * lda] : TA(0);  // LvStrict
      }
      ra[q] = v;
    }
#pragma unroll
    for (int q = 0; q < Tl::BE; ++q) {
      const int e = tid + q * Tl::NT;
      const int kk = e % BK, j = e / BK;
      const int64_t gj = n0 + j, gk = k0 + kk;
      rb[q] = (gj < N && gk < kend) ? B[gk + gj * ldb] : TB(0);
    }
  };
  auto store = [&](int buf, int64_t k0) {
#pragma unroll
    for (int q = 0; q < Tl::AE; ++q) {
      int i, kk;
      a_pos(q, i, kk);
      const int64_t gi = m0 + i, gk = k0 + kk;
      TC v;
      if (OA == OpA::LvT)
        v = gi < M && gk < kend ? (TC)lv_value<TA>(ra[q], (int)gi, sa1) : TC(0);
      else
        v = (TC)ra[q];
      if (AK) As[buf][i * Tl::A_LD + kk] = v;
      else As[buf][kk * Tl::A_LD + i] = v;
    }
#pragma unroll
    for (int q = 0; q < Tl::BE; ++q) {
      const int e = tid + q * Tl::NT;
      const int kk = e % BK, j = e / BK;
      TC v;
      if (OB == OpB::Plain) {
        v = (TC)rb[q];
      } else {
        const int64_t gj = n0 + j, gk = k0 + kk;
        v = (gj < N && gk < kend) ? (TC)lv_value<TB>(rb[q], (int)gj, sb1) : TC(0);
      }
      Bs[buf][j * Tl::B_LD + kk] = v;
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
    store(0, kbeg);
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
      for (int a = 0; a < Tl::TM; ++a) {
        const int row = wm * Tl::WTM + a * 16 + (lane & 15);
        af[a] = AK ? As[buf][row * Tl::A_LD + kr] : As[buf][kr * Tl::A_LD + row];
      }
#pragma unroll
      for (int b = 0; b < Tl::TN; ++b) {
        const int col = wn * Tl::WTN + b * 16 + (lane & 15);
        bf[b] = Bs[buf][col * Tl::B_LD + kr];
      }
#pragma unroll
      for (int a = 0; a < Tl::TM; ++a)
#pragma unroll
        for (int b = 0; b < Tl::TN; ++b) acc[a][b] = MF::mma(af[a], bf[b], acc[a][b]);
    }
    if (more) {
      if (NBUF == 1) __syncthreads();  // everyone is done reading the only buffer
      store(NBUF == 1 ? 0 : buf ^ 1, kt + BK);
    }
    __syncthreads();
    if (NBUF == 2) buf ^= 1;
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
            partial[(int64_t)bz * M * N + gi + gj * M] = val;
            if (mirror) partial[(int64_t)bz * M * N + gj + gi * M] = val;
          } else if (mirror) {
            C[gi + gj * ldc] = val;
            C[gj + gi * ldc] = val;
          } else {
            const int64_t oi = rowmap ? (int64_t)rowmap[gi] : gi;
            if (csub) C[oi + gj * ldc] -= val;
            else C[oi + gj * ldc] = val;
          }
        }
      }
}

// Workgroup b of a launch runs on XCD b mod 8.  Give each XCD a contiguous
// range of tile indices, so that the workgroups an XCD runs at the same time
// take consecutive tiles.
__device__ __forceinline__ int xcd_chunked(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

// One-dimensional grid of tm x tn x ksplit tiles.  Consecutive tiles share
// the larger operand: with nfast the N index runs fastest (tiles of one row
// block of A, Step 2 and Step 7), otherwise the M index (tiles of one
// column block of B, Step 5), so that operand block is fetched from HBM once
// and reused from the XCD's L2.
template <typename TA, typename TB, typename TC, typename TO, int BM, int BN, int BK, int WM,
          int WN, int NBUF, OpA OA, OpB OB>
__global__ void __launch_bounds__(64 * WM * WN)
gemm_kernel(int64_t M, int64_t N, int64_t K, const TA* __restrict__ A, int64_t lda,
            const int* __restrict__ astep, const TB* __restrict__ B, int64_t ldb,
            const int* __restrict__ bstep, TO* __restrict__ C, int64_t ldc,
            const int* __restrict__ rowmap, int ksplit, TO* __restrict__ partial, int tm, int tn,
            int nfast, int acol0, int csub, int blower, int sym) {
  const int t = xcd_chunked((int)blockIdx.x, (int)gridDim.x);
  int bx, by, bz;
  if (sym) {
    // a symmetric product (tm == tn): tile u of a split is the u-th tile on
    // or below the diagonal, row by row
    const int ntri = tm * (tm + 1) / 2;
    bz = t / ntri;
    const int u = t % ntri;
    int row = 0, first = 0;  // first: index of tile (row, 0)
    while (first + row + 1 <= u) {
      first += row + 1;
      ++row;
    }
    bx = row;
    by = u - first;
  } else if (nfast) {
    by = t % tn; const int rest = t / tn; bx = rest % tm; bz = rest / tm;
  } else {
    bx = t % tm; const int rest = t / tm; by = rest % tn; bz = rest / tn;
  }
  gemm_tile<TA, TB, TC, TO, BM, BN, BK, WM, WN, NBUF, OA, OB>(
      M, N, K, A, lda, astep, B, ldb, bstep, C, ldc, rowmap, ksplit, partial, bx, by, bz, acol0,
      csub, blower, sym && bx != by ? 1 : 0);
}

// Many independent products in one launch: workgroup b computes the tile
// named by map[b] = (task, bx + tiles_m (by + tiles_n bz)).
template <typename TA, typename TB, typename TC, typename TO, int BM, int BN, int BK, int WM,
          int WN, int NBUF, OpA OA, OpB OB>
__global__ void __launch_bounds__(64 * WM * WN)
gemm_grouped_kernel(const GemmTaskDev* __restrict__ tasks, const int2* __restrict__ map) {
  const int2 e = map[blockIdx.x];
  if (e.x < 0) return;  // padding of the XCD layout
  const GemmTaskDev& t = tasks[e.x];
  const int bx = e.y % t.tiles_m, rest = e.y / t.tiles_m;
  const int by = rest % t.tiles_n, bz = rest / t.tiles_n;
  gemm_tile<TA, TB, TC, TO, BM, BN, BK, WM, WN, NBUF, OA, OB>(
      t.M, t.N, t.K, (const TA*)t.A, t.lda, t.astep, (const TB*)t.B, t.ldb, t.bstep, (TO*)t.C,
      t.ldc, t.rowmap, t.ksplit, (TO*)t.partial, bx, by, bz);
}

// Split-K sums of a group: blockIdx.y is the task; tasks without a split
// are skipped.
__global__ void __launch_bounds__(256) splitk_sum_grouped_kernel(
    const GemmTaskDev* __restrict__ tasks) {
  const GemmTaskDev& t = tasks[blockIdx.y];
  if (t.ksplit <= 1) return;
  const int64_t total = t.M * t.N;
  const double* partial = (const double*)t.partial;
  double* C = (double*)t.C;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = partial[e];
    for (int z = 1; z < t.ksplit; ++z) s += partial[(int64_t)z * total + e];  // fixed order
    const int64_t i = e % t.M, j = e / t.M;
    const int64_t oi = t.rowmap ? (int64_t)t.rowmap[i] : i;
    C[oi + j * t.ldc] = s;
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

// Tile shapes compiled in (BM, BN, BK, waves M x N, LDS buffers).
enum CfgId { C64x64x16, C64x112x16, C112x64x16, C64x112x32, C112x64x32, C112x64x64,
             C64x64x32, C128x64x16, C64x128x16, C128x224x16, C224x128x16, CFG_COUNT };
struct CfgInfo { int bm, bn, bk; };
struct GemmShape { int cfg; int ksplit; };
constexpr CfgInfo kCfg[CFG_COUNT] = {{64, 64, 16}, {64, 112, 16}, {112, 64, 16},
                                     {64, 112, 32}, {112, 64, 32}, {112, 64, 64},
                                     {64, 64, 32}, {128, 64, 16}, {64, 128, 16},
                                     {128, 224, 16}, {224, 128, 16}};

int g_force_cfg = -1;  // tuning override (-1: automatic)

// Tile shape and split-K for a product (the tuning table of this library,
// from sweeps of the FP64 and FP32 products of the 8192 x 8192
// configuration on MI355X: 128 x 224 tiles with split-K 4 took the sketch
// from 0.75 to 0.56 ms in FP64, 224 x 128 the projection from 1.31 to 0.84 ms):
//   * the tile shape minimizes (rounds of 256 tiles) x (tile area), ties to
//     more tiles; an A operand streamed along K (Lv^T) uses 64 x 64 tiles,
//     which measured fastest for it;
//   * split-K raises the workgroup count to about four per CU (one
//     workgroup per CU leaves the FP64 MFMA pipe idle at every barrier),
//     keeping at least 256 of K per split (the Gram product of Step 5 went
//     from 55 to 51 us at 8192 x 200 with 256 workgroups instead of 128).
GemmShape choose_shape(int64_t M, int64_t N, int64_t K, bool kcontig_a) {
  GemmShape sh{C64x64x16, 1};
  // Long products with one short side (the two products with A): one
  // 8-wave tile spans the whole short side, so the long operand is read once,
  // and split-K brings the grid to one workgroup per CU.
  if (g_force_cfg < 0 && K >= 4096 && ((N <= 224 && M >= 1024) || (M <= 224 && N >= 1024))) {
    sh.cfg = N <= 224 && M >= 1024 ? C128x224x16 : C224x128x16;
    const CfgInfo& c = kCfg[sh.cfg];
    const int64_t tiles = ((M + c.bm - 1) / c.bm) * ((N + c.bn - 1) / c.bn);
    int ks = 1;
    while (tiles * ks < 256 && K / (ks * 2) >= 1024 && ks < 32) ks *= 2;
    sh.ksplit = ks;
    return sh;
  }
  if (g_force_cfg >= 0) {
    sh.cfg = g_force_cfg;
  } else if (K >= 4096 && ((N <= 672 && M >= 1024) || (M <= 672 && N >= 1024))) {
    // The same long products with a short side of two or three 8-wave tiles
    // (l or k up to 672): 128 x 224 tiles in either orientation (a short M
    // side wastes less in 128-row tiles), split as below.  At 16384^2 with
    // k = 500, l = 520 in FP64 the factorization took 19.6 ms against 21.4 ms
    // with the 64-wide tiles.
    sh.cfg = C128x224x16;
  } else if (kcontig_a) {
    sh.cfg = C64x64x16;
  } else {
    const int cands[3] = {C64x64x16, C64x112x16, C112x64x16};
    double best_cost = 1e300, best_tiles = 0;
    for (int id : cands) {
      const CfgInfo& c = kCfg[id];
      const double tiles = (double)((M + c.bm - 1) / c.bm) * (double)((N + c.bn - 1) / c.bn);
      const double rounds = (double)(((int64_t)tiles + 255) / 256);
      const double cost = rounds * c.bm * c.bn;
      if (cost < best_cost || (cost == best_cost && tiles > best_tiles)) {
        best_cost = cost; sh.cfg = id; best_tiles = tiles;
      }
    }
  }
  const CfgInfo& c = kCfg[sh.cfg];
  const int64_t tiles = ((M + c.bm - 1) / c.bm) * ((N + c.bn - 1) / c.bn);
  int ks = 1;
  while (tiles * ks < 1024 && K / (ks * 2) >= 256 && ks < 32) ks *= 2;
  // A grid still smaller than one workgroup per CU (the products of small
  // problems) is bound by the latency of its chain of K slices, about 1.3 us
  // each: split further, down to 64 of K per split.
  while (tiles * ks < 256 && K / (ks * 2) >= 64 && ks < 32) ks *= 2;
  sh.ksplit = ks;
  return sh;
}

template <typename TA, typename TB, typename TC, typename TO, int BM, int BN, int BK, int WM,
          int WN, int NBUF, OpA OA, OpB OB>
hipError_t launch_cfg(const GemmDesc& d, int ksplit, hipStream_t s) {
  const int tm = (int)((d.M + BM - 1) / BM), tn = (int)((d.N + BN - 1) / BN);
  // a symmetric product computes the tiles on and below the diagonal only
  const int sym = d.sym && BM == BN && d.M == d.N && !d.rowmap && !d.csub ? 1 : 0;
  const int64_t nb = sym ? (int64_t)tm * (tm + 1) / 2 * ksplit : (int64_t)tm * tn * ksplit;
  if (nb >= (1LL << 31)) return hipErrorInvalidValue;
  const int nfast = d.M > d.N ? 1 : 0;  // A is the larger operand
  hipLaunchKernelGGL((gemm_kernel<TA, TB, TC, TO, BM, BN, BK, WM, WN, NBUF, OA, OB>),
                     dim3((unsigned)nb), dim3(64 * WM * WN), 0, s, d.M, d.N, d.K, (const TA*)d.A,
                     d.lda, d.astep, (const TB*)d.B, d.ldb, d.bstep, (TO*)d.C, d.ldc, d.rowmap,
                     ksplit, (TO*)d.partial, tm, tn, nfast, d.acol0, d.csub ? 1 : 0,
                     d.b_lower ? 1 : 0, sym);
  return hipGetLastError();
}

template <typename TA, typename TB, typename TC, typename TO, OpA OA, OpB OB>
hipError_t launch_ops(const GemmDesc& d, hipStream_t s) {
  GemmShape sh = choose_shape(d.M, d.N, d.K, OA == OpA::LvT);
  const int c = sh.cfg;
  // ksplit 0 = automatic (needs the partial workspace); 1 = no split
  const int ks = d.csub ? 1 : (d.ksplit == 0 ? (d.partial ? sh.ksplit : 1) : d.ksplit);
  if (d.ksplit_out) *d.ksplit_out = ks;
  hipError_t e;
  switch (c) {
    case C64x64x16: e = launch_cfg<TA, TB, TC, TO, 64, 64, 16, 2, 2, 2, OA, OB>(d, ks, s); break;
    case C64x112x16: e = launch_cfg<TA, TB, TC, TO, 64, 112, 16, 4, 1, 2, OA, OB>(d, ks, s); break;
    case C112x64x16: e = launch_cfg<TA, TB, TC, TO, 112, 64, 16, 1, 4, 2, OA, OB>(d, ks, s); break;
    case C64x112x32: e = launch_cfg<TA, TB, TC, TO, 64, 112, 32, 4, 1, 2, OA, OB>(d, ks, s); break;
    case C112x64x32: e = launch_cfg<TA, TB, TC, TO, 112, 64, 32, 1, 4, 2, OA, OB>(d, ks, s); break;
    case C112x64x64: e = launch_cfg<TA, TB, TC, TO, 112, 64, 64, 1, 4, 1, OA, OB>(d, ks, s); break;
    case C64x64x32: e = launch_cfg<TA, TB, TC, TO, 64, 64, 32, 2, 2, 2, OA, OB>(d, ks, s); break;
    case C128x64x16: e = launch_cfg<TA, TB, TC, TO, 128, 64, 16, 2, 2, 2, OA, OB>(d, ks, s); break;
    case C128x224x16: e = launch_cfg<TA, TB, TC, TO, 128, 224, 16, 4, 2, 2, OA, OB>(d, ks, s); break;
    case C224x128x16: e = launch_cfg<TA, TB, TC, TO, 224, 128, 16, 2, 4, 2, OA, OB>(d, ks, s); break;
    default: e = launch_cfg<TA, TB, TC, TO, 64, 128, 16, 2, 2, 2, OA, OB>(d, ks, s); break;
  }
  if (e != hipSuccess || ks == 1 || d.no_sum) return e;
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
  if (d.opa == OpA::LvStrict && d.opb == OpB::Plain)
    return launch_ops<TA, TB, TC, TO, OpA::LvStrict, OpB::Plain>(d, s);
  return hipErrorInvalidValue;
}

template <typename TA, typename TB, typename TC, typename TO, OpA OA, OpB OB>
hipError_t launch_grouped_ops(int cfg, const GemmTaskDev* tasks, const int2* map, int nwg,
                              hipStream_t s) {
  if (nwg <= 0) return hipSuccess;
#define RLU_GG(BM, BN, BK, WM, WN, NB)                                                       \
  hipLaunchKernelGGL((gemm_grouped_kernel<TA, TB, TC, TO, BM, BN, BK, WM, WN, NB, OA, OB>), \
                     dim3((unsigned)nwg), dim3(64 * WM * WN), 0, s, tasks, map)
  switch (cfg) {
    case C64x64x16: RLU_GG(64, 64, 16, 2, 2, 2); break;
    case C64x112x16: RLU_GG(64, 112, 16, 4, 1, 2); break;
    case C112x64x16: RLU_GG(112, 64, 16, 1, 4, 2); break;
    case C64x112x32: RLU_GG(64, 112, 32, 4, 1, 2); break;
    case C112x64x32: RLU_GG(112, 64, 32, 1, 4, 2); break;
    case C64x64x32: RLU_GG(64, 64, 32, 2, 2, 2); break;
    case C128x64x16: RLU_GG(128, 64, 16, 2, 2, 2); break;
    case C64x128x16: RLU_GG(64, 128, 16, 2, 2, 2); break;
    default: return hipErrorInvalidValue;
  }
#undef RLU_GG
  return hipGetLastError();
}

}  // namespace

void gemm_group_tile(int cfg, int* bm, int* bn) {
  const int c = (cfg >= 0 && cfg < CFG_COUNT) ? cfg : C64x64x16;
  *bm = kCfg[c].bm;
  *bn = kCfg[c].bn;
}

bool gemm_group_cfg_valid(int cfg) {
  switch (cfg) {
    case C64x64x16: case C64x112x16: case C112x64x16: case C64x112x32: case C112x64x32:
    case C64x64x32: case C128x64x16: case C64x128x16:
      return true;
    default:
      return false;
  }
}

const char* gemm_cfg_name(int cfg) {
  static const char* const names[CFG_COUNT] = {
      "64x64x16", "64x112x16", "112x64x16", "64x112x32", "112x64x32", "112x64x64",
      "64x64x32", "128x64x16", "64x128x16", "128x224x16", "224x128x16"};
  return (cfg >= 0 && cfg < CFG_COUNT) ? names[cfg] : nullptr;
}

// The grouped products of the batched form, by role (operand forms and
// types fixed by the role; f32: FP32 storage of A, G and L).
hipError_t launch_gemm_grouped_role(GemmRole role, bool f32, int cfg, const GemmTaskDev* tasks,
                                    const int2* map, int nwg, hipStream_t s) {
  if (!gemm_group_cfg_valid(cfg)) return hipErrorInvalidValue;
  switch (role) {
    case GemmRole::Sketch:
      return f32 ? launch_grouped_ops<float, float, float, double, OpA::Plain, OpB::Plain>(cfg, tasks, map, nwg, s)
                 : launch_grouped_ops<double, double, double, double, OpA::Plain, OpB::Plain>(cfg, tasks, map, nwg, s);
    case GemmRole::Gram:
      return launch_grouped_ops<double, double, double, double, OpA::LvT, OpB::Lv>(cfg, tasks, map, nwg, s);
    case GemmRole::Project:
      return f32 ? launch_grouped_ops<double, float, float, double, OpA::LvT, OpB::Plain>(cfg, tasks, map, nwg, s)
                 : launch_grouped_ops<double, double, double, double, OpA::LvT, OpB::Plain>(cfg, tasks, map, nwg, s);
    case GemmRole::Solve:
      return launch_grouped_ops<double, double, double, double, OpA::Plain, OpB::Plain>(cfg, tasks, map, nwg, s);
    case GemmRole::FormL:
      return f32 ? launch_grouped_ops<double, double, double, float, OpA::Lv, OpB::Plain>(cfg, tasks, map, nwg, s)
                 : launch_grouped_ops<double, double, double, double, OpA::Lv, OpB::Plain>(cfg, tasks, map, nwg, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_splitk_sum_grouped(const GemmTaskDev* tasks, int count, int64_t max_elems,
                                     hipStream_t s) {
  if (count <= 0 || max_elems <= 0) return hipSuccess;
  int64_t bx = (max_elems + 255) / 256;
  if (bx > 64) bx = 64;
  hipLaunchKernelGGL(splitk_sum_grouped_kernel, dim3((unsigned)bx, (unsigned)count), dim3(256), 0,
                     s, tasks);
  return hipGetLastError();
}

size_t gemm_partial_elems(int64_t M, int64_t N, int ksplit) {
  return ksplit > 1 ? (size_t)ksplit * (size_t)M * (size_t)N : 0;
}

size_t gemm_auto_partial_elems(int64_t M, int64_t N, int64_t K, OpA opa) {
  return gemm_partial_elems(M, N, choose_shape(M, N, K, opa == OpA::LvT).ksplit);
}

hipError_t launch_splitk_sum_f64(int64_t M, int64_t N, int ksplit, const double* partial,
                                 double* C, int64_t ldc, const int* rowmap, hipStream_t s) {
  const int64_t total = M * N;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(splitk_sum_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, M, N,
                     ksplit, partial, C, ldc, rowmap);
  return hipGetLastError();
}

void gemm_force_config(int id) { g_force_cfg = (id >= 0 && id < CFG_COUNT) ? id : -1; }

template <typename TA, typename TB, typename TC, typename TO>
hipError_t launch_gemm_t(const GemmDesc& d, hipStream_t s) {
  return dispatch<TA, TB, TC, TO>(d, s);
}

// FP64 path: every operand and the output in FP64.
template hipError_t launch_gemm_t<double, double, double, double>(const GemmDesc&, hipStream_t);
// FP32 path: FP32 MFMA on FP32 storage (A, G) or on Lv rounded to FP32;
// results widened to FP64 for the pivoted LUs and the Gram solve.
template hipError_t launch_gemm_t<float, float, float, double>(const GemmDesc&, hipStream_t);
template hipError_t launch_gemm_t<double, float, float, double>(const GemmDesc&, hipStream_t);
// FP64 arithmetic, FP32 output (L of the FP32 path).
template hipError_t launch_gemm_t<double, double, double, float>(const GemmDesc&, hipStream_t);

template <>
hipError_t launch_gemm<double>(const GemmDesc& d, hipStream_t s) {
  return dispatch<double, double, double, double>(d, s);
}

}  // namespace rlu
