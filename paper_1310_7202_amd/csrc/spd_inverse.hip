// Inverse of the k x k Gram matrix S = L_y^T L_y (Step 5 of Algorithm 4.1,
// Shabat et al., Section 4, and the Remark after it: the pseudo-inverse
// (L_y^T L_y)^{-1} L_y^T, with the small k x k inversion done by Gaussian
// elimination).
//
// S is symmetric positive definite (L_y has a unit diagonal, hence full
// column rank), so Gauss-Jordan elimination without pivoting is stable and
// turns S into S^{-1} in place: at step j the pivot row is scaled by the
// reciprocal pivot and eliminated from every other row.
//
// One workgroup of 32 TY threads holds the whole matrix in registers: thread
// (ty, tx) = (t / 32, t % 32) owns rows ty + TY a and columns tx + 32 b.  The
// pivot row and column of each step pass through LDS (two buffers alternating
// by step, so one barrier per step suffices).
#include "rlu_device.h"
#include "rlu_kernels.h"

namespace rlu {
namespace {


template <int TY, int NA, int NB>
__device__ __forceinline__ void spd_inverse_body(double* __restrict__ S, int k) {
  constexpr int KR = TY * NA, KC = 32 * NB;
  __shared__ double rowj[2][KC];
  __shared__ double colj[2][KR];
  const int t = threadIdx.x, ty = t >> 5, tx = t & 31;
  double a[NA][NB];
#pragma unroll
  for (int ia = 0; ia < NA; ++ia)
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) {
      const int i = ty + TY * ia, c = tx + 32 * ib;
      a[ia][ib] = (i < k && c < k) ? S[i + (int64_t)c * k] : (i == c ? 1.0 : 0.0);
    }
  for (int j = 0; j < k; ++j) {
    const int par = j & 1;
    const int ja = j / TY, jb = j >> 5;  // register slots of row j / column j (uniform)
    const bool own_row = (j % TY) == ty, own_col = (j & 31) == tx;
    if (own_row) {
#pragma unroll
      for (int x = 0; x < NA; ++x)
        if (x == ja)
#pragma unroll
          for (int ib = 0; ib < NB; ++ib) rowj[par][tx + 32 * ib] = a[x][ib];
    }
    if (own_col) {
#pragma unroll
      for (int y = 0; y < NB; ++y)
        if (y == jb)
#pragma unroll
          for (int ia = 0; ia < NA; ++ia) colj[par][ty + TY * ia] = a[ia][y];
    }
    __syncthreads();
    const double d = 1.0 / rowj[par][j];
    // rank-one elimination of row j from every other row, written so that
    // row j and column j are left untouched (their factors are zero) ...
    double r[NB];
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) {
      const int c = tx + 32 * ib;
      r[ib] = (c == j) ? 0.0 : rowj[par][c] * d;  // scaled pivot row
    }
#pragma unroll
    for (int ia = 0; ia < NA; ++ia) {
      const int i = ty + TY * ia;
      const double f = (i == j) ? 0.0 : colj[par][i];
#pragma unroll
      for (int ib = 0; ib < NB; ++ib) a[ia][ib] = __fma_rn(-f, r[ib], a[ia][ib]);
    }
    // ... and then set explicitly: row j becomes the scaled pivot row (with
    // 1/pivot on the diagonal), column j becomes -column/pivot
    if (own_row) {
#pragma unroll
      for (int x = 0; x < NA; ++x)
        if (x == ja)
#pragma unroll
          for (int ib = 0; ib < NB; ++ib) {
            const int c = tx + 32 * ib;
            a[x][ib] = (c == j) ? d : rowj[par][c] * d;
          }
    }
    if (own_col) {
#pragma unroll
      for (int y = 0; y < NB; ++y)
        if (y == jb)
#pragma unroll
          for (int ia = 0; ia < NA; ++ia) {
            const int i = ty + TY * ia;
            if (i != j) a[ia][y] = -colj[par][i] * d;
          }
    }
  }
#pragma unroll
  for (int ia = 0; ia < NA; ++ia)
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) {
      const int i = ty + TY * ia, c = tx + 32 * ib;
      if (i < k && c < k) S[i + (int64_t)c * k] = a[ia][ib];
    }
}

template <int TY, int NA, int NB>
__global__ void __launch_bounds__(32 * TY) spd_inverse_kernel(double* __restrict__ S, int k) {
  spd_inverse_body<TY, NA, NB>(S, k);
}

// One workgroup per matrix of a batch.
template <int TY, int NA, int NB>
__global__ void __launch_bounds__(32 * TY)
spd_inverse_batched_kernel(const SpdTaskDev* __restrict__ tasks) {
  const SpdTaskDev t = tasks[blockIdx.x];
  spd_inverse_body<TY, NA, NB>(t.S, t.k);
}

}  // namespace

bool spd_inverse_supported(int64_t k) { return k >= 1 && k <= 208; }

hipError_t launch_spd_inverse(double* S, int64_t k, hipStream_t s) {
  if (!spd_inverse_supported(k)) return hipErrorInvalidValue;
  const int kk = (int)k;
#define RLU_SPD(TY, NA, NB) \
  hipLaunchKernelGGL((spd_inverse_kernel<TY, NA, NB>), dim3(1), dim3(32 * TY), 0, s, S, kk)
  if (k <= 64) RLU_SPD(32, 2, 2);
  else if (k <= 128) RLU_SPD(32, 4, 4);
  else if (k <= 160) RLU_SPD(32, 5, 5);
  else if (k <= 192) RLU_SPD(32, 6, 6);
  else RLU_SPD(16, 13, 7);  // 208 x 224
#undef RLU_SPD
  return hipGetLastError();
}

hipError_t launch_spd_inverse_batched(const SpdTaskDev* tasks, int count, int64_t kmax,
                                     hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (!spd_inverse_supported(kmax)) return hipErrorInvalidValue;
#define RLU_SPD(TY, NA, NB)                                                                 \
  hipLaunchKernelGGL((spd_inverse_batched_kernel<TY, NA, NB>), dim3((unsigned)count),      \
                     dim3(32 * TY), 0, s, tasks)
  if (kmax <= 64) RLU_SPD(32, 2, 2);
  else if (kmax <= 128) RLU_SPD(32, 4, 4);
  else if (kmax <= 160) RLU_SPD(32, 5, 5);
  else if (kmax <= 192) RLU_SPD(32, 6, 6);
  else RLU_SPD(16, 13, 7);
#undef RLU_SPD
  return hipGetLastError();
}

}  // namespace rlu
