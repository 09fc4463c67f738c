// Inverse of the k x k Gram matrix S = L_y^T L_y (Step 5 of Algorithm 4.1,
// Shabat et al., Section 4, and the Remark after it: the pseudo-inverse
// (L_y^T L_y)^{-1} L_y^T, with the small k x k inversion done by Gaussian
// elimination).
//
// S is symmetric positive definite (L_y has a unit diagonal, hence full
// column rank), so Gauss-Jordan elimination without pivoting is stable.
#include "rlu_device.h"
#include "rlu_kernels.h"

#include <algorithm>

namespace rlu {
namespace {

// ---------------------------------------------------------------------------
// The symmetric sweep operator, 64 pivots per launch.  Sweeping pivot p of
// a matrix M replaces
//   M[r][s] by M[r][s] - M[r][p] M[p][s] / M[p][p]     (r, s != p)
//   M[r][p] by M[r][p] / M[p][p],  M[p][s] by M[p][s] / M[p][p]
//   M[p][p] by -1 / M[p][p]
// which is Gauss-Jordan elimination written so that a symmetric matrix stays
// symmetric; sweeping every pivot of S once leaves -S^{-1}.  Every pivot met
// is a Schur complement of the SPD matrix S, hence positive.
//
// The new value of an entry (r, s) under the sweep of a pivot set J depends
// only on rows J + {r} and columns J + {s}.  So launch J gives each 64 x 64
// tile (I, c) of S one workgroup, which gathers the augmented matrix
//   [ S_JJ  S_Jc ]
//   [ S_IJ  S_Ic ]      (rows I and columns c left out when I = J or c = J)
// into registers, sweeps the pivots of J in it and writes its (I, c) part.
// Tiles read one buffer and write the other (S and a k x k scratch copy,
// alternating so that the last launch writes S); the last launch also
// negates.
// ---------------------------------------------------------------------------
constexpr int GB = 64;
constexpr int kSwThreads = 256;  // 16 x 16 threads, 8 x 8 entries each

__device__ __forceinline__ int blk_size(int k, int J) { return min(GB, k - GB * J); }
__device__ __forceinline__ int num_blocks(int k) { return (k + GB - 1) / GB; }
// launch J writes S when an even number of launches follow it
__device__ __forceinline__ bool writes_s(int nb, int J) { return ((nb - 1 - J) & 1) == 0; }

// odd block counts start from the copy in scratch (so that the last launch
// still writes S): copy S there first
__global__ void __launch_bounds__(256) sweep_copy_kernel(const SpdTaskDev* __restrict__ tasks,
                                                         SpdTaskDev one) {
  const SpdTaskDev t = tasks ? tasks[blockIdx.y] : one;
  const int nb = num_blocks(t.k);
  if (nb < 2 || !writes_s(nb, 0)) return;
  const int64_t kk = (int64_t)t.k * t.k;
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < kk; e += (int64_t)gridDim.x * 256)
    t.scratch[e] = t.S[e];
}

// One tile: RA = 8 when the augmented matrix has the rows of block I (I != J),
// else 4; RB likewise for the columns of block c.  Thread (ty, tx) holds
// augmented rows ty + 16 a and columns tx + 16 b.  Each pivot costs one
// barrier: the owners of its column and row (and of the next pivot) publish
// them in LDS; every thread then updates its entries and, from the same
// LDS values, the next pivot, so the division leaves the critical path.
template <int RA, int RB>
__device__ __forceinline__ void sweep_tile(const double* __restrict__ in, double* __restrict__ out,
                                           int k, int J, int I, int cb, bool last) {
  const int bj = blk_size(k, J), bi = blk_size(k, I), bc = blk_size(k, cb);
  __shared__ double colb[2][2 * GB];
  __shared__ double rowb[2][2 * GB];
  __shared__ double diagb[2];
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  double M[RA][RB];
#pragma unroll
  for (int a = 0; a < RA; ++a) {
    const int r = ty + 16 * a;
    const bool rin = a < 4 ? r < bj : r - GB < bi;
    const int64_t gr = a < 4 ? (int64_t)GB * J + r : (int64_t)GB * I + (r - GB);
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int c = tx + 16 * b;
      const bool cin = b < 4 ? c < bj : c - GB < bc;
      const int64_t gc = b < 4 ? (int64_t)GB * J + c : (int64_t)GB * cb + (c - GB);
      M[a][b] = (rin && cin) ? in[gr + gc * k] : 0.0;
    }
  }
  double rd = 1.0 / in[(int64_t)GB * J * (k + 1)];  // first pivot

  // pivot p = 16 pa + pt sits in register slot pa of the threads with
  // ty = pt (its row) and tx = pt (its column); pa is unrolled so that every
  // register index is static
#pragma unroll
  for (int pa = 0; pa < 4; ++pa) {
    for (int pt = 0; pt < 16; ++pt) {
      const int p = 16 * pa + pt;
      if (p >= bj) break;
      const int par = p & 1, q = p + 1;
      const bool orow = ty == pt, ocol = tx == pt;
      if (ocol) {
#pragma unroll
        for (int a = 0; a < RA; ++a) colb[par][ty + 16 * a] = M[a][pa];
      }
      if (orow) {
#pragma unroll
        for (int b = 0; b < RB; ++b) rowb[par][tx + 16 * b] = M[pa][b];
      }
      // the next pivot's entry, before this step
      if (q < bj && ty == (q & 15) && tx == (q & 15)) {
        const int pn = pa < 3 ? pa + 1 : 3;
        diagb[par] = pt < 15 ? M[pa][pa] : M[pn][pn];
      }
      __syncthreads();
      double fr[RA], gs[RB];
#pragma unroll
      for (int a = 0; a < RA; ++a) fr[a] = colb[par][ty + 16 * a];
#pragma unroll
      for (int b = 0; b < RB; ++b) gs[b] = rowb[par][tx + 16 * b] * rd;
      // the next pivot after this step, as its owner computes it below
      // (straight-line code, so that the division overlaps the update)
      const double den = q < bj ? __fma_rn(-colb[par][q], rowb[par][q] * rd, diagb[par]) : 1.0;
      const double rd_next = 1.0 / den;
      // The pivot row and column come out of the same fused multiply-add:
      // with its entries cleared, fr = -1 on the pivot row gives M[p][s] / d
      // (= gs), gs = -1/d on the pivot column gives M[r][p] / d, and both
      // together give -1/d on the pivot.
      fr[pa] = orow ? -1.0 : fr[pa];
      gs[pa] = ocol ? -rd : gs[pa];
#pragma unroll
      for (int b = 0; b < RB; ++b) M[pa][b] = orow ? 0.0 : M[pa][b];
#pragma unroll
      for (int a = 0; a < RA; ++a) M[a][pa] = ocol ? 0.0 : M[a][pa];
#pragma unroll
      for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int b = 0; b < RB; ++b) M[a][b] = __fma_rn(-fr[a], gs[b], M[a][b]);
      rd = rd_next;
    }
  }

  // the (I, c) part of the augmented matrix
  constexpr int a0 = RA == 8 ? 4 : 0, b0 = RB == 8 ? 4 : 0;
#pragma unroll
  for (int a = a0; a < RA; ++a) {
    const int i = ty + 16 * (a - a0);
    if (i >= bi) continue;
#pragma unroll
    for (int b = b0; b < RB; ++b) {
      const int j = tx + 16 * (b - b0);
      if (j >= bc) continue;
      out[(int64_t)GB * I + i + ((int64_t)GB * cb + j) * k] = last ? -M[a][b] : M[a][b];
    }
  }
}

__global__ void __launch_bounds__(kSwThreads) sweep_step_kernel(const SpdTaskDev* __restrict__ tasks,
                                                               SpdTaskDev one, int J) {
  const SpdTaskDev t = tasks ? tasks[blockIdx.y] : one;
  const int k = t.k, nb = num_blocks(k);
  if (J >= nb || (int)blockIdx.x >= nb * nb) return;
  const int I = blockIdx.x % nb, cb = blockIdx.x / nb;
  const double* in;
  double* out;
  if (nb == 1) {
    in = out = t.S;  // a single tile: in place
  } else {
    const bool ws = writes_s(nb, J);
    in = ws ? t.scratch : t.S;
    out = ws ? t.S : t.scratch;
  }
  const bool last = J == nb - 1;
  if (I != J) {
    if (cb != J) sweep_tile<8, 8>(in, out, k, J, I, cb, last);
    else sweep_tile<8, 4>(in, out, k, J, I, cb, last);
  } else {
    if (cb != J) sweep_tile<4, 8>(in, out, k, J, I, cb, last);
    else sweep_tile<4, 4>(in, out, k, J, I, cb, last);
  }
}

}  // namespace

bool spd_inverse_supported(int64_t k) { return k >= 1 && k <= kSpdMaxK; }

size_t spd_inverse_scratch_elems(int64_t k) { return (size_t)k * (size_t)k; }

namespace {
hipError_t sweep_steps(const SpdTaskDev* tasks, SpdTaskDev one, int count, int64_t kmax,
                       hipStream_t s) {
  const int nb = (int)((kmax + GB - 1) / GB);
  if (nb >= 2) {
    const unsigned g = (unsigned)std::min<int64_t>((kmax * kmax + 255) / 256, 1024);
    hipLaunchKernelGGL(sweep_copy_kernel, dim3(g, (unsigned)count), dim3(256), 0, s, tasks, one);
  }
  for (int J = 0; J < nb; ++J)
    hipLaunchKernelGGL(sweep_step_kernel, dim3((unsigned)(nb * nb), (unsigned)count),
                       dim3(kSwThreads), 0, s, tasks, one, J);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_spd_inverse_scratch(double* S, int64_t k, double* scratch, hipStream_t s) {
  if (!spd_inverse_supported(k)) return hipErrorInvalidValue;
  if (k > GB && !scratch) return hipErrorInvalidValue;
  return sweep_steps(nullptr, SpdTaskDev{S, (int)k, scratch}, 1, k, s);
}

hipError_t launch_spd_inverse_batched(const SpdTaskDev* tasks, int count, int64_t kmax,
                                     hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (!spd_inverse_supported(kmax)) return hipErrorInvalidValue;
  return sweep_steps(tasks, SpdTaskDev{nullptr, 0, nullptr}, count, kmax, s);
}

}  // namespace rlu
