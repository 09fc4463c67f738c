// Assembly of the outputs of Algorithm 4.1 (Shabat et al., Section 4) from
// the two pivoted LUs, plus small utility kernels.
//
// Step 6 is computed as the partial-pivot LU of B^T (n x k), held in the
// storage of B (k x n): Q^T B^T = L' U' with L' unit lower (n x k) and U'
// upper (k x k).  Transposing, B Q = U'^T L'^T, and with D = diag(U'):
//   L_b = U'^T D^{-1}   (unit lower, k x k)
//   U_b = D L'^T        (upper, k x n)
// which is the column-pivoted LU of B with the unit diagonal on L_b, the
// form Step 7 needs (L = L_y L_b stays unit lower trapezoidal).  A zero pivot
// D(r) = 0 leaves column r of L_b below the diagonal zero; row r of U_b is
// then zero as well (its multipliers were never scaled and are all zero).
#include "rlu_device.h"
#include "rlu_kernels.h"

namespace rlu {
namespace {

template <typename TI, typename TO>
__global__ void __launch_bounds__(256) convert2d_kernel(const TI* __restrict__ src, int64_t lds,
                                                        TO* __restrict__ dst, int64_t ldd,
                                                        int64_t rows, int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % rows, j = e / rows;
    dst[i + j * ldd] = (TO)src[i + j * lds];
  }
}

// Dense copy of the unit-lower factor that a pivoted LU left in place (rows
// never moved): out(i, c) = Lv(i, c) for c < cols, converted to TO.
template <typename TO>
__global__ void __launch_bounds__(256) lv_dense_kernel(const double* __restrict__ X, int64_t ldx,
                                                       const int* __restrict__ rstep,
                                                       TO* __restrict__ out, int64_t ldo,
                                                       int64_t rows, int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % rows, c = e / rows;
    out[i + c * ldo] = (TO)lv_value<double>(X[i + c * ldx], (int)c, rstep[i]);
  }
}

// Batched form of lv_dense_kernel over strided panels: out(i, c) =
// Lv(i, c) of the panel whose entry (i, c) is X[i rs + c cs].
template <typename TO>
__global__ void __launch_bounds__(256) lv_dense_batched_kernel(
    const LvDenseTaskDev* __restrict__ tasks) {
  const LvDenseTaskDev t = tasks[blockIdx.y];
  const int64_t total = t.rows * t.cols;
  TO* out = (TO*)t.out;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % t.rows, c = e / t.rows;
    out[i + c * t.ldo] = (TO)lv_value<double>(t.X[i * t.rs + c * t.cs], (int)c, t.rstep[i]);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) copy2d_kernel(const T* __restrict__ src, int64_t lds,
                                                     T* __restrict__ dst, int64_t ldd,
                                                     int64_t rows, int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % rows, j = e / rows;
    dst[i + j * ldd] = src[i + j * lds];
  }
}

__global__ void __launch_bounds__(256) fill_u32_kernel(uint32_t* __restrict__ p, size_t count,
                                                       uint32_t v) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (size_t)gridDim.x * blockDim.x)
    p[e] = v;
}

__global__ void __launch_bounds__(256) copy_i32_kernel(const int* __restrict__ src,
                                                       int32_t* __restrict__ dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

// Steps 7-8 assembly (blockIdx.y = problem of a batch, or the one task
// passed by value): the permutations p and q from the row positions, U = U_b
// scattered by column position, L_b, and the info words.
template <typename TO>
__global__ void __launch_bounds__(256) assemble_batched_kernel(const AsmTaskDev* __restrict__ tasks,
                                                               AsmTaskDev one) {
  const AsmTaskDev t = tasks ? tasks[blockIdx.y] : one;
  const int64_t m = t.m, n = t.n, k = t.k;
  const int64_t e_q = m, e_u = m + n, e_lb = m + n + k * n, total = e_lb + k * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < e_q) {
      t.p[t.pos_y[e]] = e;
    } else if (e < e_u) {
      const int64_t o = e - e_q;
      t.q[t.pos_b[o]] = o;
    } else if (e < e_lb) {
      const int64_t x = e - e_u, r = x % k, o = x / k;
      const double d = t.Bst[r + (int64_t)t.piv_b[r] * k];
      const double lv = lv_value<double>(t.Bst[r + o * k], (int)r, t.rstep_b[o]);
      ((TO*)t.U)[r + (int64_t)t.pos_b[o] * t.ldu] = (TO)(d * lv);
    } else {
      const int64_t x = e - e_lb, i = x % k, r = x / k;
      double v = 0.0;
      if (i == r) {
        v = 1.0;
      } else if (i > r) {
        const int64_t o = t.piv_b[r];
        const double d = t.Bst[r + o * k];
        const double u = t.Bst[i + o * k];
        v = d != 0.0 ? u / d : 0.0;
      }
      t.Lb[i + r * k] = v;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    t.info[0] = t.flags[0];
    t.info[1] = t.flags[1];
    // bit 0: the pivot exchange failed; bit 1: a non-finite value was found
    // in the sketch (the check the caller asked for)
    t.info[2] = (t.flags[2] != 0 ? 1 : 0) | (t.flags[4] != 0 ? 2 : 0);
  }
}

// Non-finite scan of a sketch (blockIdx.y = task): any NaN or infinity in
// A or G reaches every entry of its row of Y = A G (x * 0 and inf - inf are
// NaN), so scanning Y finds it without another pass over A.  A wave that
// finds one stores 1 into the task's flag word (every writer stores the same
// value).
__global__ void __launch_bounds__(256) check_finite_kernel(const FiniteTaskDev* __restrict__ tasks,
                                                           FiniteTaskDev one) {
  const FiniteTaskDev t = tasks ? tasks[blockIdx.y] : one;
  bool bad = false;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < t.count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long b = __double_as_longlong(t.Y[e]);
    bad |= (b & 0x7ff0000000000000ull) == 0x7ff0000000000000ull;
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) *t.flag = 1;
}

// dst (cols x rows) = src (rows x cols)^T through 32 x 32 LDS tiles.
__global__ void __launch_bounds__(256) transpose_kernel(const double* __restrict__ src,
                                                        int64_t lds, double* __restrict__ dst,
                                                        int64_t ldd, int64_t rows, int64_t cols) {
  __shared__ double t[32][33];
  const int64_t r0 = 32 * (int64_t)blockIdx.x, c0 = 32 * (int64_t)blockIdx.y;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int y = ty; y < 32; y += 8) {
    const int64_t r = r0 + tx, c = c0 + y;
    t[y][tx] = (r < rows && c < cols) ? src[r + c * lds] : 0.0;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t c = c0 + tx, r = r0 + y;  // dst(c, r) = src(r, c)
    if (r < rows && c < cols) dst[c + r * ldd] = t[tx][y];
  }
}

inline unsigned grid_for(int64_t n, int64_t cap = 8192) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

}  // namespace

template <typename TI, typename TO>
hipError_t launch_convert2d(const TI* src, int64_t lds, TO* dst, int64_t ldd, int64_t rows,
                            int64_t cols, hipStream_t s) {
  hipLaunchKernelGGL((convert2d_kernel<TI, TO>), dim3(grid_for(rows * cols)), dim3(256), 0, s,
                     src, lds, dst, ldd, rows, cols);
  return hipGetLastError();
}
template hipError_t launch_convert2d<double, float>(const double*, int64_t, float*, int64_t,
                                                    int64_t, int64_t, hipStream_t);
template hipError_t launch_convert2d<float, double>(const float*, int64_t, double*, int64_t,
                                                    int64_t, int64_t, hipStream_t);

template <typename TO>
hipError_t launch_lv_dense(const double* X, int64_t ldx, const int* rstep, TO* out, int64_t ldo,
                           int64_t rows, int64_t cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL((lv_dense_kernel<TO>), dim3(grid_for(rows * cols)), dim3(256), 0, s, X, ldx,
                     rstep, out, ldo, rows, cols);
  return hipGetLastError();
}
template hipError_t launch_lv_dense<double>(const double*, int64_t, const int*, double*, int64_t,
                                            int64_t, int64_t, hipStream_t);
template hipError_t launch_lv_dense<float>(const double*, int64_t, const int*, float*, int64_t,
                                           int64_t, int64_t, hipStream_t);

template <typename TO>
hipError_t launch_lv_dense_batched(const LvDenseTaskDev* tasks, int count, int64_t max_elems,
                                   hipStream_t s) {
  if (count <= 0 || max_elems <= 0) return hipSuccess;
  if (count > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL((lv_dense_batched_kernel<TO>), dim3(grid_for(max_elems, 2048), (unsigned)count),
                     dim3(256), 0, s, tasks);
  return hipGetLastError();
}
template hipError_t launch_lv_dense_batched<double>(const LvDenseTaskDev*, int, int64_t,
                                                    hipStream_t);
template hipError_t launch_lv_dense_batched<float>(const LvDenseTaskDev*, int, int64_t,
                                                   hipStream_t);

template <typename T>
hipError_t launch_copy2d(const T* src, int64_t lds, T* dst, int64_t ldd, int64_t rows,
                         int64_t cols, hipStream_t s) {
  hipLaunchKernelGGL(copy2d_kernel<T>, dim3(grid_for(rows * cols)), dim3(256), 0, s, src, lds, dst,
                     ldd, rows, cols);
  return hipGetLastError();
}
template hipError_t launch_copy2d<double>(const double*, int64_t, double*, int64_t, int64_t,
                                          int64_t, hipStream_t);
template hipError_t launch_copy2d<float>(const float*, int64_t, float*, int64_t, int64_t, int64_t,
                                         hipStream_t);

hipError_t launch_fill_u32(uint32_t* p, size_t count, uint32_t v, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for((int64_t)count, 1024)), dim3(256), 0, s, p,
                     count, v);
  return hipGetLastError();
}

hipError_t launch_copy_i32(const int* src, int32_t* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(copy_i32_kernel, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

template <typename TO>
hipError_t launch_assemble_batched(const AsmTaskDev* tasks, int count, int64_t max_elems,
                                   hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t bx = (max_elems + 255) / 256;
  if (bx < 1) bx = 1;
  if (bx > 128) bx = 128;
  hipLaunchKernelGGL(assemble_batched_kernel<TO>, dim3((unsigned)bx, (unsigned)count), dim3(256),
                     0, s, tasks, AsmTaskDev{});
  return hipGetLastError();
}
template hipError_t launch_assemble_batched<double>(const AsmTaskDev*, int, int64_t, hipStream_t);
template hipError_t launch_assemble_batched<float>(const AsmTaskDev*, int, int64_t, hipStream_t);

template <typename TO>
hipError_t launch_assemble_one(const AsmTaskDev& t, hipStream_t s) {
  const int64_t total = t.m + t.n + t.k * t.n + t.k * t.k;
  hipLaunchKernelGGL(assemble_batched_kernel<TO>, dim3(grid_for(total, 1024)), dim3(256), 0, s,
                     (const AsmTaskDev*)nullptr, t);
  return hipGetLastError();
}
template hipError_t launch_assemble_one<double>(const AsmTaskDev&, hipStream_t);
template hipError_t launch_assemble_one<float>(const AsmTaskDev&, hipStream_t);

hipError_t launch_check_finite(const FiniteTaskDev& t, hipStream_t s) {
  if (t.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(check_finite_kernel, dim3(grid_for(t.count, 2048)), dim3(256), 0, s,
                     (const FiniteTaskDev*)nullptr, t);
  return hipGetLastError();
}

hipError_t launch_check_finite_batched(const FiniteTaskDev* tasks, int count, int64_t max_elems,
                                       hipStream_t s) {
  if (count <= 0 || max_elems <= 0) return hipSuccess;
  if (count > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(check_finite_kernel, dim3(grid_for(max_elems, 256), (unsigned)count),
                     dim3(256), 0, s, tasks, FiniteTaskDev{});
  return hipGetLastError();
}

hipError_t launch_transpose(const double* src, int64_t lds, double* dst, int64_t ldd,
                            int64_t rows, int64_t cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)((rows + 31) / 32), (unsigned)((cols + 31) / 32)),
                     dim3(256), 0, s, src, lds, dst, ldd, rows, cols);
  return hipGetLastError();
}

}  // namespace rlu
