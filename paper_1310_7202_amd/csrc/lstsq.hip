// Rank-deficient least squares on the factors of the randomized LU
// (Shabat et al., Section 4.4, Algorithm 4.3): x = Q (U_1^{-1} L^+ P b; 0).
//
// The launch sequence (rlu_api.cpp, rlu_lstsq) folds P into the rows of L
// (lstsq_scatter_rows: L_P = P^T L, so L^T P b = L_P^T b), applies L^+
// through the Gram matrix with the products and the SPD inverse of Step 5,
// and ends with lstsq_back: back substitution with U_1 (the leading k x k
// block of U) for each right-hand side, and the scatter x[q[j]] = z[j].
#include "rlu_device.h"
#include "rlu_kernels.h"

#include <hip/hip_runtime.h>

namespace rlu {
namespace {

constexpr int kLsThreads = 256;
constexpr int kLsPer = kLsMaxK / kLsThreads;  // rows of U_1 per thread

// Ld (m x k, FP64, ld m): row p[i] of Ld = row i of L.  Entries of p outside
// [0, m) are skipped (p is a permutation for the factors of rlu_factor).
template <typename T>
__global__ void __launch_bounds__(256) lstsq_scatter_rows_kernel(const T* __restrict__ L,
                                                                 int64_t ldl,
                                                                 const int64_t* __restrict__ p,
                                                                 int64_t m, int64_t k,
                                                                 double* __restrict__ Ld) {
  const int64_t total = m * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % m, j = e / m;
    const int64_t dst = p[i];
    if ((uint64_t)dst < (uint64_t)m) Ld[dst + j * m] = (double)L[i + j * ldl];
  }
}

// One workgroup per right-hand side r: z_1 = U_1^{-1} y (column r of Y,
// k x nrhs), then x(:, r) = Q (z_1; 0).  Column j of U_1 is loaded while
// column j + 1 is applied; the working right-hand side, the solution and
// the diagonal live in LDS.  A zero diagonal entry leaves its unknown 0.
template <typename TU, typename TX>
__global__ void __launch_bounds__(kLsThreads) lstsq_back_kernel(
    const TU* __restrict__ U, int64_t ldu, const double* __restrict__ Y, int k,
    const int64_t* __restrict__ q, int64_t n, TX* __restrict__ X, int64_t ldx) {
  __shared__ double z[kLsMaxK];
  __shared__ double zf[kLsMaxK];
  __shared__ double dg[kLsMaxK];
  const int t = threadIdx.x;
  const int64_t r = blockIdx.x;
  for (int i = t; i < k; i += kLsThreads) {
    z[i] = Y[i + r * k];
    dg[i] = (double)U[i + (int64_t)i * ldu];
  }
  double u[kLsPer], un[kLsPer];
  auto load = [&](int j, double* dst) {
#pragma unroll
    for (int c = 0; c < kLsPer; ++c) {
      const int i = t + kLsThreads * c;
      dst[c] = i < j ? (double)U[i + (int64_t)j * ldu] : 0.0;  // j < 0 loads nothing
    }
  };
  load(k - 1, u);
  __syncthreads();
  for (int j = k - 1; j >= 0; --j) {
    load(j - 1, un);
    const double d = dg[j];
    const double zj = d != 0.0 ? z[j] / d : 0.0;
    if (t == 0) zf[j] = zj;
#pragma unroll
    for (int c = 0; c < kLsPer; ++c) {
      const int i = t + kLsThreads * c;
      if (i < j) z[i] = __fma_rn(-u[c], zj, z[i]);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kLsPer; ++c) u[c] = un[c];
  }
  for (int64_t j = t; j < n; j += kLsThreads) {
    const int64_t dst = q[j];
    if ((uint64_t)dst < (uint64_t)n) X[dst + r * ldx] = (TX)(j < k ? zf[j] : 0.0);
  }
}

inline unsigned grid_elems(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

}  // namespace

template <typename T>
hipError_t launch_lstsq_scatter_rows(const T* L, int64_t ldl, const int64_t* p, int64_t m,
                                     int64_t k, double* Ld, hipStream_t s) {
  if (m <= 0 || k <= 0) return hipSuccess;
  hipLaunchKernelGGL((lstsq_scatter_rows_kernel<T>), dim3(grid_elems(m * k)), dim3(256), 0, s, L,
                     ldl, p, m, k, Ld);
  return hipGetLastError();
}
template hipError_t launch_lstsq_scatter_rows<double>(const double*, int64_t, const int64_t*,
                                                      int64_t, int64_t, double*, hipStream_t);
template hipError_t launch_lstsq_scatter_rows<float>(const float*, int64_t, const int64_t*,
                                                     int64_t, int64_t, double*, hipStream_t);

template <typename T>
hipError_t launch_lstsq_back(const T* U, int64_t ldu, const double* Y, int64_t k,
                             const int64_t* q, int64_t n, int64_t nrhs, T* X, int64_t ldx,
                             hipStream_t s) {
  if (nrhs <= 0) return hipSuccess;
  if (k < 1 || k > kLsMaxK || nrhs >= (1LL << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((lstsq_back_kernel<T, T>), dim3((unsigned)nrhs), dim3(kLsThreads), 0, s, U,
                     ldu, Y, (int)k, q, n, X, ldx);
  return hipGetLastError();
}
template hipError_t launch_lstsq_back<double>(const double*, int64_t, const double*, int64_t,
                                              const int64_t*, int64_t, int64_t, double*, int64_t,
                                              hipStream_t);
template hipError_t launch_lstsq_back<float>(const float*, int64_t, const double*, int64_t,
                                             const int64_t*, int64_t, int64_t, float*, int64_t,
                                             hipStream_t);

}  // namespace rlu
