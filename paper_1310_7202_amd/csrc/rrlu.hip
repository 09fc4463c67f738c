// The rank-revealing Step 3 of Algorithm 4.1 as listed (Shabat et al.,
// Section 4, with the RRLU of Section 3.1, Theorem 3.1): P Y Q_y = L_y U_y.
//
// Q_y is the column order of a column-pivoted QR of the sketch Y (m x l):
// at each step the remaining column with the largest norm orthogonal to the
// columns already chosen.  That norm is the diagonal of the Schur complement
// of the Gram matrix S = Y^T Y, so the same order comes from a pivoted
// Cholesky factorization S(q, q) = R^T R, which needs only the l x l Gram
// matrix (one product on the matrix cores) and runs in one workgroup.  Then
// the columns are gathered into Y Q_y and the partial-pivot LU of Step 3 runs
// on it unchanged.
//
// Pivoted Cholesky, one workgroup of 1024 threads, l <= 1024 (left-looking):
//   step j: the remaining column c* with the largest Schur diagonal d(c*)
//           (lowest current position on ties, as the positions move by the
//           exchanges of a column-pivoted QR) takes position j;
//           R(j, c*) = sqrt(d(c*)), and for every remaining column c
//           R(j, c) = (S(c*, c) - sum_{t<j} R(t, c*) R(t, c)) / R(j, c*),
//           d(c) -= R(j, c)^2.
// R is stored by step and original column, R[t l + c], so the sums read
// consecutive addresses across the threads of a wave; G = 1024 / l'
// threads (l' = l rounded up to a power of two) share each column's sum.
#include "rlu_device.h"
#include "rlu_kernels.h"

#include <climits>

namespace rlu {
namespace {

constexpr int kCpThreads = 1024;
constexpr int kCpWaves = kCpThreads / 64;

__device__ __forceinline__ bool cp_better(double a, int pa, double b, int pb) {
  return a > b || (a == b && pa < pb);
}

__global__ void __launch_bounds__(kCpThreads)
colpiv_gram_kernel(const double* __restrict__ S, int64_t lds, int l, int group,
                   double* __restrict__ R, int* __restrict__ qy) {
  __shared__ double d[kSpdColPivMax];     // Schur diagonal, by original column
  __shared__ int pos[kSpdColPivMax];      // current position of each column
  __shared__ int col_at[kSpdColPivMax];   // column at each position
  __shared__ double rp[kSpdColPivMax];    // R(0:j, c*) of the current pivot
  __shared__ double wbest[kCpWaves];
  __shared__ int wpos[kCpWaves], wcol[kCpWaves];
  __shared__ int s_win;
  __shared__ double s_rjj;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = tid / group, sub = tid % group;  // column handled, share of its sum
  for (int i = tid; i < l; i += kCpThreads) {
    d[i] = S[i + (int64_t)i * lds];
    pos[i] = i;
    col_at[i] = i;
  }
  __syncthreads();
  for (int j = 0; j < l; ++j) {
    // ---- the remaining column with the largest Schur diagonal -------------
    double best = -1.0;
    int bp = INT_MAX, bc = -1;
    if (sub == 0 && c < l && pos[c] >= j) {
      const double v = d[c];
      if (!(v != v)) { best = v; bp = pos[c]; bc = c; }  // a NaN never wins
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(best, off, 64);
      const int op = __shfl_xor(bp, off, 64), oc = __shfl_xor(bc, off, 64);
      if (oc >= 0 && (bc < 0 || cp_better(ov, op, best, bp))) { best = ov; bp = op; bc = oc; }
    }
    if (lane == 0) { wbest[wave] = best; wpos[wave] = bp; wcol[wave] = bc; }
    __syncthreads();
    if (tid == 0) {
      double b = -1.0;
      int p = INT_MAX, w = -1;
      for (int q = 0; q < kCpWaves; ++q)
        if (wcol[q] >= 0 && (w < 0 || cp_better(wbest[q], wpos[q], b, p))) {
          b = wbest[q]; p = wpos[q]; w = wcol[q];
        }
      if (w < 0) w = col_at[j];  // every remaining diagonal is NaN: keep the order
      // exchange positions j and pos[w]
      const int cj = col_at[j], pw = pos[w];
      col_at[pw] = cj; pos[cj] = pw;
      col_at[j] = w; pos[w] = j;
      qy[j] = w;
      s_win = w;
      const double dj = d[w];
      s_rjj = dj > 0.0 ? sqrt(dj) : 0.0;
    }
    __syncthreads();
    const int win = s_win;
    const double rjj = s_rjj;
    for (int t = tid; t < j; t += kCpThreads) rp[t] = R[(int64_t)t * l + win];
    __syncthreads();
    // ---- row j of R over the remaining columns -----------------------------
    const bool act = c < l && pos[c] > j;
    double acc = 0.0;
    if (act) {
      const double* Rc = R + c;
      int t = sub;
      for (; t + 3 * group < j; t += 4 * group) {
        const double r0 = Rc[(int64_t)t * l], r1 = Rc[(int64_t)(t + group) * l];
        const double r2 = Rc[(int64_t)(t + 2 * group) * l], r3 = Rc[(int64_t)(t + 3 * group) * l];
        acc = __fma_rn(rp[t], r0, acc);
        acc = __fma_rn(rp[t + group], r1, acc);
        acc = __fma_rn(rp[t + 2 * group], r2, acc);
        acc = __fma_rn(rp[t + 3 * group], r3, acc);
      }
      for (; t < j; t += group) acc = __fma_rn(rp[t], Rc[(int64_t)t * l], acc);
    }
    // the group's partial sums (consecutive lanes), in a fixed order
    for (int off = 1; off < group; off <<= 1) acc += __shfl_down(acc, off, 64);
    if (act && sub == 0) {
      const double v = S[win + (int64_t)c * lds] - acc;
      const double r = rjj > 0.0 ? v / rjj : 0.0;
      R[(int64_t)j * l + c] = r;
      d[c] = d[c] - r * r;
    }
    if (tid == 0) R[(int64_t)j * l + win] = rjj;
    __syncthreads();
  }
}

// Yq(:, j) = Y(:, qy[j])
__global__ void __launch_bounds__(256) gather_cols_kernel(const double* __restrict__ Y, int64_t ldy,
                                                          const int* __restrict__ qy,
                                                          double* __restrict__ Yq, int64_t ldq,
                                                          int64_t m, int l) {
  const int j = blockIdx.y;
  const int64_t src = (int64_t)qy[j];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    Yq[i + (int64_t)j * ldq] = Y[i + src * ldy];
}

}  // namespace

hipError_t launch_colpiv_gram(const double* S, int64_t lds, int l, double* R, int* qy,
                              hipStream_t s) {
  if (l <= 0) return hipSuccess;
  if (l > kSpdColPivMax) return hipErrorInvalidValue;
  int lp = 1;
  while (lp < l) lp <<= 1;
  const int group = lp >= kCpThreads ? 1 : kCpThreads / lp;   // a power of two <= 64
  hipLaunchKernelGGL(colpiv_gram_kernel, dim3(1), dim3(kCpThreads), 0, s, S, lds, l,
                     group > 64 ? 64 : group, R, qy);
  return hipGetLastError();
}

hipError_t launch_gather_cols(const double* Y, int64_t ldy, const int* qy, double* Yq,
                              int64_t ldq, int64_t m, int l, hipStream_t s) {
  if (m <= 0 || l <= 0) return hipSuccess;
  if (l > 65535) return hipErrorInvalidValue;
  int64_t bx = (m + 255) / 256;
  if (bx > 64) bx = 64;
  hipLaunchKernelGGL(gather_cols_kernel, dim3((unsigned)bx, (unsigned)l), dim3(256), 0, s, Y, ldy,
                     qy, Yq, ldq, m, l);
  return hipGetLastError();
}

}  // namespace rlu
