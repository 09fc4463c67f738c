// Steps 5-6 of Algorithm 4.4, fast randomized LU (Shabat et al., Section
// 4.5): the full-rank interpolative decomposition Y = X Y(J, :) of the
// sketch and B = L_y^+ P X A(J, :).
//
// The ID comes from the partial-pivot LU of Step 3 (Section 3.4 allows an
// LU-based ID): with rows never moved, Lv (m x l) is that LU's unit-lower
// factor in original row order, J = the rows its steps chose (in step
// order) and L11 = Lv(J, :) (l x l unit lower triangular), so
//   X = Y Y(J, :)^{-1} = Lv L11^{-1}.
// With L_y = P Lv(:, 0:k) and S = Lv(:, 0:k)^T Lv(:, 0:k),
//   L_y^+ P X = S^{-1} Lv(:, 0:k)^T Lv L11^{-1} = [I_k, T] L11^{-1} = W,
//   T = S^{-1} Lv(:, 0:k)^T Lv(:, k:l),
// and B = W A(J, :) reads l rows of A instead of all of it.  The products
// (S, T, B) run on the matrix-core GEMM; this file holds the two kernels
// between them: W from [I_k, T] by a right-hand triangular solve with L11,
// and the gather of A(J, :).
#include "rlu_device.h"
#include "rlu_kernels.h"

namespace rlu {
namespace {

// W L11 = V = [I_k, T]: rows of W are independent.  One wave per block of
// `rows` rows of W, held in LDS (row stride l + 1), solved from the last
// column to the first: W(r, c) = V(r, c) - sum_{c' > c} W(r, c') L11(c', c),
// L11(c', c) = Y[J[c'] + c ldy] (the multiplier row J[c'] stored at step c).
__global__ void __launch_bounds__(64) id_solve_kernel(const double* __restrict__ T, int64_t ldt,
                                                      const double* __restrict__ Y, int64_t ldy,
                                                      const int* __restrict__ J, int k, int l,
                                                      int rows, double* __restrict__ W,
                                                      int64_t ldw) {
  extern __shared__ double sm[];
  const int ld = l + 1;
  double* Ws = sm;                       // rows x ld
  double* col = sm + (int64_t)rows * ld; // column c of L11 below the diagonal
  const int lane = threadIdx.x;
  const int r0 = blockIdx.x * rows;
  // V = [I_k, T] into LDS
  for (int e = lane; e < rows * l; e += 64) {
    const int rr = e / l, c = e % l, r = r0 + rr;
    double v = 0.0;
    if (r < k) v = c < k ? (c == r ? 1.0 : 0.0) : T[r + (int64_t)(c - k) * ldt];
    Ws[rr * ld + c] = v;
  }
  const int r = r0 + lane;
  const bool act = lane < rows && r < k;
  for (int c = l - 1; c >= 0; --c) {
    for (int cp = c + 1 + lane; cp < l; cp += 64) col[cp] = Y[J[cp] + (int64_t)c * ldy];
    __syncthreads();
    if (act) {
      double acc = Ws[lane * ld + c];
      for (int cp = c + 1; cp < l; ++cp) acc = __fma_rn(-Ws[lane * ld + cp], col[cp], acc);
      Ws[lane * ld + c] = acc;
    }
    __syncthreads();
  }
  for (int e = lane; e < rows * l; e += 64) {
    const int rr = e / l, c = e % l, rw = r0 + rr;
    if (rw < k) W[rw + (int64_t)c * ldw] = Ws[rr * ld + c];
  }
}

// AJ(c, j) = A(J[c], j), c < l, j < n
template <typename T>
__global__ void __launch_bounds__(256) gather_rows_kernel(const T* __restrict__ A, int64_t lda,
                                                          const int* __restrict__ J, int l,
                                                          int64_t n, T* __restrict__ AJ,
                                                          int64_t ldaj) {
  const int64_t total = (int64_t)l * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e % l, j = e / l;
    AJ[c + j * ldaj] = A[(int64_t)J[c] + j * lda];
  }
}

}  // namespace

int id_solve_rows(int l) {
  const int64_t budget = 160 * 1024 - 1024;
  int64_t rows = (budget / 8 - l) / (l + 1);
  if (rows > 64) rows = 64;
  return rows < 1 ? 0 : (int)rows;
}

hipError_t launch_id_solve(const double* T, int64_t ldt, const double* Y, int64_t ldy,
                           const int* J, int k, int l, double* W, int64_t ldw, hipStream_t s) {
  if (k <= 0 || l <= 0) return hipSuccess;
  const int rows = id_solve_rows(l);
  if (rows < 1) return hipErrorInvalidValue;
  const size_t lds = ((size_t)rows * (l + 1) + (size_t)l) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)id_solve_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const unsigned blocks = (unsigned)((k + rows - 1) / rows);
  hipLaunchKernelGGL(id_solve_kernel, dim3(blocks), dim3(64), lds, s, T, ldt, Y, ldy, J, k, l,
                     rows, W, ldw);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_rows(const T* A, int64_t lda, const int* J, int l, int64_t n, T* AJ,
                              int64_t ldaj, hipStream_t s) {
  if (l <= 0 || n <= 0) return hipSuccess;
  int64_t blocks = ((int64_t)l * n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(gather_rows_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, A, lda, J, l,
                     n, AJ, ldaj);
  return hipGetLastError();
}
template hipError_t launch_gather_rows<double>(const double*, int64_t, const int*, int, int64_t,
                                               double*, int64_t, hipStream_t);
template hipError_t launch_gather_rows<float>(const float*, int64_t, const int*, int, int64_t,
                                              float*, int64_t, hipStream_t);

}  // namespace rlu
