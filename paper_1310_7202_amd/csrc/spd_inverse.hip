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
// One workgroup of 512 threads holds the whole matrix in registers: thread
// (ty, tx) = (t / 32, t % 32) owns rows ty + 16 a and columns tx + 32 b.  The
// pivot row and column of each step pass through LDS (two buffers alternating
// by step, so one barrier per step suffices).
#include "rlu_device.h"
#include "rlu_kernels.h"

namespace rlu {
namespace {

constexpr int kSpdThreads = 512;

template <int NA, int NB>
__global__ void __launch_bounds__(kSpdThreads) spd_inverse_kernel(double* __restrict__ S, int k) {
  constexpr int KR = 16 * NA, KC = 32 * NB;
  __shared__ double rowj[2][KC];
  __shared__ double colj[2][KR];
  const int t = threadIdx.x, ty = t >> 5, tx = t & 31;
  double a[NA][NB];
#pragma unroll
  for (int ia = 0; ia < NA; ++ia)
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) {
      const int i = ty + 16 * ia, c = tx + 32 * ib;
      a[ia][ib] = (i < k && c < k) ? S[i + (int64_t)c * k] : (i == c ? 1.0 : 0.0);
    }
  for (int j = 0; j < k; ++j) {
    const int par = j & 1;
    if ((j & 15) == ty) {
      const int ia = j >> 4;
#pragma unroll
      for (int x = 0; x < NA; ++x)
        if (x == ia)
#pragma unroll
          for (int ib = 0; ib < NB; ++ib) rowj[par][tx + 32 * ib] = a[x][ib];
    }
    if ((j & 31) == tx) {
      const int ib = j >> 5;
#pragma unroll
      for (int y = 0; y < NB; ++y)
        if (y == ib)
#pragma unroll
          for (int ia = 0; ia < NA; ++ia) colj[par][ty + 16 * ia] = a[ia][y];
    }
    __syncthreads();
    const double d = 1.0 / rowj[par][j];
#pragma unroll
    for (int ia = 0; ia < NA; ++ia) {
      const int i = ty + 16 * ia;
      const double f = colj[par][i];
#pragma unroll
      for (int ib = 0; ib < NB; ++ib) {
        const int c = tx + 32 * ib;
        const double rc = rowj[par][c] * d;  // scaled pivot row
        double v;
        if (i == j) v = (c == j) ? d : rc;
        else v = (c == j) ? -f * d : a[ia][ib] - f * rc;
        a[ia][ib] = v;
      }
    }
  }
#pragma unroll
  for (int ia = 0; ia < NA; ++ia)
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) {
      const int i = ty + 16 * ia, c = tx + 32 * ib;
      if (i < k && c < k) S[i + (int64_t)c * k] = a[ia][ib];
    }
}

}  // namespace

bool spd_inverse_supported(int64_t k) { return k >= 1 && k <= 208; }

hipError_t launch_spd_inverse(double* S, int64_t k, hipStream_t s) {
  if (!spd_inverse_supported(k)) return hipErrorInvalidValue;
  const int kk = (int)k;
  if (k <= 64)
    hipLaunchKernelGGL((spd_inverse_kernel<4, 2>), dim3(1), dim3(kSpdThreads), 0, s, S, kk);
  else if (k <= 128)
    hipLaunchKernelGGL((spd_inverse_kernel<8, 4>), dim3(1), dim3(kSpdThreads), 0, s, S, kk);
  else
    hipLaunchKernelGGL((spd_inverse_kernel<13, 7>), dim3(1), dim3(kSpdThreads), 0, s, S, kk);
  return hipGetLastError();
}

}  // namespace rlu
