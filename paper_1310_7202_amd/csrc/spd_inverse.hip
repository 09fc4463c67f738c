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
// The symmetric sweep operator, GB pivots per launch.  Sweeping pivot p of
// a matrix M replaces
//   M[r][s] by M[r][s] - M[r][p] M[p][s] / M[p][p]     (r, s != p)
//   M[r][p] by M[r][p] / M[p][p],  M[p][s] by M[p][s] / M[p][p]
//   M[p][p] by -1 / M[p][p]
// which is Gauss-Jordan elimination written so that a symmetric matrix stays
// symmetric; sweeping every pivot of S once leaves -S^{-1}.  Every pivot met
// is a Schur complement of the SPD matrix S, hence positive.
//
// The new value of an entry (r, s) under the sweep of a pivot set J depends
// only on rows J + {r} and columns J + {s}.  So launch J gives each GB x GB
// tile (I, c) of S one workgroup, which gathers the augmented matrix
//   [ S_JJ  S_Jc ]
//   [ S_IJ  S_Ic ]      (rows I and columns c left out when I = J or c = J)
// into registers, sweeps the pivots of J in it and writes its (I, c) part.
// Tiles read one buffer and write the other (S and a k x k scratch copy,
// alternating so that the last launch writes S); the last launch also
// negates.
// ---------------------------------------------------------------------------
// The block size GB is 64 for k <= 64 (one launch in place) and 32 above:
// a 32-block launch gives each workgroup a quarter of the work (a 64 x 64
// augmented matrix) on four times as many CUs, at the cost of twice as many
// launches.
constexpr int kSwThreads = 256;  // 16 x 16 threads, (2 GB / 16)^2 entries each

template <int GB>
__device__ __forceinline__ int blk_size(int k, int J) { return min(GB, k - GB * J); }
template <int GB>
__device__ __forceinline__ int num_blocks(int k) { return (k + GB - 1) / GB; }
// launch J writes S when an even number of launches follow it
__device__ __forceinline__ bool writes_s(int nb, int J) { return ((nb - 1 - J) & 1) == 0; }

// odd block counts start from the copy in scratch (so that the last launch
// still writes S): copy S there first
template <int GB>
__global__ void __launch_bounds__(256) sweep_copy_kernel(const SpdTaskDev* __restrict__ tasks,
                                                         SpdTaskDev one) {
  const SpdTaskDev t = tasks ? tasks[blockIdx.y] : one;
  const int nb = num_blocks<GB>(t.k);
  if (nb < 2 || !writes_s(nb, 0)) return;
  const int64_t kk = (int64_t)t.k * t.k;
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < kk; e += (int64_t)gridDim.x * 256)
    t.scratch[e] = t.S[e];
}

// One tile: RA = 2 S (S = GB / 16 register slots per block) when the
// augmented matrix has the rows of block I (I != J), else S; RB likewise for
// the columns of block c.  Thread (ty, tx) holds augmented rows ty + 16 a and
// columns tx + 16 b.
//
// Pivots are swept two at a time: sweeping the pair J2 = {p, p + 1} at once
// is the same as sweeping p and then p + 1 (the sweep of a block replaces
// M_rs by M_rs - M_rJ2 D^{-1} M_J2s, M_rJ2 by M_rJ2 D^{-1}, M_J2s by
// D^{-1} M_J2s and D by -D^{-1}, D = M_J2J2, symmetric positive definite),
// so each pair costs one barrier.  The owners of the pair's two columns and
// two rows publish them in LDS, and the owners of the next pair's 2 x 2
// block publish it; every thread then applies the rank-2 update and, from
// the same LDS values, forms the next pair's block and its inverse, so the
// division leaves the critical path.  An odd last pivot is a pair whose
// second member is absent (zero row and column, D = diag(d, 1)).
template <int GB, int RA, int RB>
__device__ __forceinline__ void sweep_tile(const double* __restrict__ in, double* __restrict__ out,
                                           int k, int J, int I, int cb, bool last) {
  constexpr int S = GB / 16;
  const int bj = blk_size<GB>(k, J), bi = blk_size<GB>(k, I), bc = blk_size<GB>(k, cb);
  __shared__ double colb[2][2][2 * GB];  // [parity][member of the pair][augmented row]
  __shared__ double rowb[2][2][2 * GB];
  __shared__ double dnx[2][3];           // next pair's block before this step
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  double M[RA][RB];
#pragma unroll
  for (int a = 0; a < RA; ++a) {
    const int r = ty + 16 * a;
    const bool rin = a < S ? r < bj : r - GB < bi;
    const int64_t gr = a < S ? (int64_t)GB * J + r : (int64_t)GB * I + (r - GB);
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int c = tx + 16 * b;
      const bool cin = b < S ? c < bj : c - GB < bc;
      const int64_t gc = b < S ? (int64_t)GB * J + c : (int64_t)GB * cb + (c - GB);
      M[a][b] = (rin && cin) ? in[gr + gc * k] : 0.0;
    }
  }
  // inverse of the first pair's block: [e11 e12; e12 e22]
  double e11, e12, e22;
  {
    const int64_t o = (int64_t)GB * J;
    const double d11 = in[o + o * k];
    if (bj >= 2) {
      const double d12 = in[o + (o + 1) * k], d22 = in[(o + 1) + (o + 1) * k];
      const double r = 1.0 / __fma_rn(d11, d22, -d12 * d12);
      e11 = d22 * r; e12 = -d12 * r; e22 = d11 * r;
    } else {
      e11 = 1.0 / d11; e12 = 0.0; e22 = 0.0;
    }
  }

  // pair (p, p + 1), p = 16 pa + pt with pt even: both sit in register slot
  // pa of the threads with ty (rows) or tx (columns) = pt, pt + 1; pa is
  // unrolled so that every register index is static
#pragma unroll
  for (int pa = 0; pa < S; ++pa) {
    const int pn = pa < S - 1 ? pa + 1 : S - 1;
    for (int pt = 0; pt < 16; pt += 2) {
      const int p = 16 * pa + pt;
      if (p >= bj) break;
      const int par = (pt >> 1) & 1;
      const bool two = p + 1 < bj;
      const bool orow0 = ty == pt, orow1 = two && ty == pt + 1;
      const bool ocol0 = tx == pt, ocol1 = two && tx == pt + 1;
      if (ocol0 || ocol1) {
#pragma unroll
        for (int a = 0; a < RA; ++a) colb[par][tx - pt][ty + 16 * a] = M[a][pa];
      }
      if (orow0 || orow1) {
#pragma unroll
        for (int b = 0; b < RB; ++b) rowb[par][ty - pt][tx + 16 * b] = M[pa][b];
      }
      // the next pair (q0, q1) = (p + 2, p + 3): its block before this step
      // sits in slot pa, or pa + 1 when pt = 14
      const int q0 = p + 2, qt = q0 & 15;
      const bool nxt = q0 < bj, nxt2 = q0 + 1 < bj;
      if (nxt && ty >= qt && ty <= qt + 1 && tx >= qt && tx <= qt + 1 && ty <= tx) {
        const int slot = (ty - qt) + (tx - qt);  // 0: (q0, q0), 1: (q0, q1), 2: (q1, q1)
        if (slot == 0 || nxt2) dnx[par][slot] = pt < 14 ? M[pa][pa] : M[pn][pn];
      }
      __syncthreads();
      double f0[RA], f1[RA], g0[RB], g1[RB];
#pragma unroll
      for (int a = 0; a < RA; ++a) {
        f0[a] = colb[par][0][ty + 16 * a];
        f1[a] = two ? colb[par][1][ty + 16 * a] : 0.0;
      }
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const double r0 = rowb[par][0][tx + 16 * b];
        const double r1 = two ? rowb[par][1][tx + 16 * b] : 0.0;
        g0[b] = __fma_rn(e12, r1, e11 * r0);
        g1[b] = __fma_rn(e22, r1, e12 * r0);
      }
      // the next pair's block after this step and its inverse (straight-line
      // code, so that the division overlaps the update)
      double n11 = 1.0, n12 = 0.0, n22 = 1.0;
      if (nxt) {
        const int q1 = nxt2 ? q0 + 1 : q0;
        const double c00 = colb[par][0][q0], c01 = two ? colb[par][1][q0] : 0.0;
        const double c10 = colb[par][0][q1], c11 = two ? colb[par][1][q1] : 0.0;
        const double s00 = rowb[par][0][q0], s01 = two ? rowb[par][1][q0] : 0.0;
        const double s10 = rowb[par][0][q1], s11 = two ? rowb[par][1][q1] : 0.0;
        // D^{-1} M_J2,q for the columns q0 and q1
        const double h00 = __fma_rn(e12, s01, e11 * s00), h01 = __fma_rn(e22, s01, e12 * s00);
        const double h10 = __fma_rn(e12, s11, e11 * s10), h11 = __fma_rn(e22, s11, e12 * s10);
        n11 = dnx[par][0] - __fma_rn(c00, h00, c01 * h01);
        if (nxt2) {
          n12 = dnx[par][1] - __fma_rn(c00, h10, c01 * h11);
          n22 = dnx[par][2] - __fma_rn(c10, h10, c11 * h11);
        }
      }
      const double rn = 1.0 / (nxt2 ? __fma_rn(n11, n22, -n12 * n12) : n11);
      // rows and columns of the pair come out of the same multiply-adds: with
      // their entries cleared, f = -e_i on pivot row i and g = -D^{-1} e_j on
      // pivot column j give D^{-1} M_J2s, M_rJ2 D^{-1} and -D^{-1}
      f0[pa] = orow0 ? -1.0 : (orow1 ? 0.0 : f0[pa]);
      f1[pa] = orow0 ? 0.0 : (orow1 ? -1.0 : f1[pa]);
      g0[pa] = ocol0 ? -e11 : (ocol1 ? -e12 : g0[pa]);
      g1[pa] = ocol0 ? -e12 : (ocol1 ? -e22 : g1[pa]);
#pragma unroll
      for (int b = 0; b < RB; ++b) M[pa][b] = (orow0 || orow1) ? 0.0 : M[pa][b];
#pragma unroll
      for (int a = 0; a < RA; ++a) M[a][pa] = (ocol0 || ocol1) ? 0.0 : M[a][pa];
#pragma unroll
      for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int b = 0; b < RB; ++b)
          M[a][b] = __fma_rn(-f1[a], g1[b], __fma_rn(-f0[a], g0[b], M[a][b]));
      if (nxt2) {
        e11 = n22 * rn; e12 = -n12 * rn; e22 = n11 * rn;
      } else {
        e11 = rn; e12 = 0.0; e22 = 0.0;
      }
    }
  }

  // the (I, c) part of the augmented matrix
  constexpr int a0 = RA == 2 * S ? S : 0, b0 = RB == 2 * S ? S : 0;
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

template <int GB>
__global__ void __launch_bounds__(kSwThreads) sweep_step_kernel(const SpdTaskDev* __restrict__ tasks,
                                                               SpdTaskDev one, int J) {
  constexpr int S = GB / 16;
  const SpdTaskDev t = tasks ? tasks[blockIdx.y] : one;
  const int k = t.k, nb = num_blocks<GB>(k);
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
    if (cb != J) sweep_tile<GB, 2 * S, 2 * S>(in, out, k, J, I, cb, last);
    else sweep_tile<GB, 2 * S, S>(in, out, k, J, I, cb, last);
  } else {
    if (cb != J) sweep_tile<GB, S, 2 * S>(in, out, k, J, I, cb, last);
    else sweep_tile<GB, S, S>(in, out, k, J, I, cb, last);
  }
}

}  // namespace

bool spd_inverse_supported(int64_t k) { return k >= 1 && k <= kSpdMaxK; }

size_t spd_inverse_scratch_elems(int64_t k) { return (size_t)k * (size_t)k; }

namespace {
template <int GB>
hipError_t sweep_steps_gb(const SpdTaskDev* tasks, SpdTaskDev one, int count, int64_t kmax,
                          hipStream_t s) {
  const int nb = (int)((kmax + GB - 1) / GB);
  if (nb >= 2) {
    const unsigned g = (unsigned)std::min<int64_t>((kmax * kmax + 255) / 256, 1024);
    hipLaunchKernelGGL(sweep_copy_kernel<GB>, dim3(g, (unsigned)count), dim3(256), 0, s, tasks,
                       one);
  }
  for (int J = 0; J < nb; ++J)
    hipLaunchKernelGGL(sweep_step_kernel<GB>, dim3((unsigned)(nb * nb), (unsigned)count),
                       dim3(kSwThreads), 0, s, tasks, one, J);
  return hipGetLastError();
}

hipError_t sweep_steps(const SpdTaskDev* tasks, SpdTaskDev one, int count, int64_t kmax,
                       hipStream_t s) {
  return kmax > 64 ? sweep_steps_gb<32>(tasks, one, count, kmax, s)
                   : sweep_steps_gb<64>(tasks, one, count, kmax, s);
}
}  // namespace

hipError_t launch_spd_inverse_scratch(double* S, int64_t k, double* scratch, hipStream_t s) {
  if (!spd_inverse_supported(k)) return hipErrorInvalidValue;
  if (k > 64 && !scratch) return hipErrorInvalidValue;
  return sweep_steps(nullptr, SpdTaskDev{S, (int)k, scratch}, 1, k, s);
}

hipError_t launch_spd_inverse_batched(const SpdTaskDev* tasks, int count, int64_t kmax,
                                     hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (!spd_inverse_supported(kmax)) return hipErrorInvalidValue;
  return sweep_steps(tasks, SpdTaskDev{nullptr, 0, nullptr}, count, kmax, s);
}

}  // namespace rlu
