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
__device__ __forceinline__ void spd_inverse_body(const double* __restrict__ S, int lds,
                                                 double* __restrict__ Out, int ldo, int k) {
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
      a[ia][ib] = (i < k && c < k) ? S[i + (int64_t)c * lds] : (i == c ? 1.0 : 0.0);
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
      if (i < k && c < k) Out[i + (int64_t)c * ldo] = a[ia][ib];
    }
}

template <int TY, int NA, int NB>
__global__ void __launch_bounds__(32 * TY) spd_inverse_kernel(double* __restrict__ S, int k) {
  spd_inverse_body<TY, NA, NB>(S, k, S, k, k);
}

// One workgroup per matrix of a batch.
template <int TY, int NA, int NB>
__global__ void __launch_bounds__(32 * TY)
spd_inverse_batched_kernel(const SpdTaskDev* __restrict__ tasks) {
  const SpdTaskDev t = tasks[blockIdx.x];
  spd_inverse_body<TY, NA, NB>(t.S, t.k, t.S, t.k, t.k);
}

// ---------------------------------------------------------------------------
// Blocked Gauss-Jordan for larger k.  With 64-wide blocks and J the pivot
// block of a step (D = S_JJ, its inverse Di):
//   S_Ic <- S_Ic - S_IJ Di S_Jc   (I, c != J)
//   S_Jc <- Di S_Jc               (c != J)
//   S_IJ <- -S_IJ Di              (I != J)
//   S_JJ <- Di
// (the elementwise step above, taken 64 pivots at a time; every D is a
// Schur complement of the SPD matrix S, hence SPD).  A step is three
// launches: Di by the register kernel (one workgroup), then R = Di S_J. and
// a copy C = S_.J of the old column block, then every 64 x 64 tile of S
// from Di, R and C only, so tiles never read what another tile writes.
// Scratch per matrix: Di (64 x 64), R (64 x k), C (k x 64).
// ---------------------------------------------------------------------------
constexpr int GB = 64;

__device__ __forceinline__ int blk_size(int k, int J) { return min(GB, k - GB * J); }

// step 1: Di = (S_JJ)^{-1}, one workgroup of 32 TY threads per matrix
template <int TY, int NA, int NB>
__global__ void __launch_bounds__(32 * TY) gj_diag_kernel(const SpdTaskDev* __restrict__ tasks,
                                                          SpdTaskDev one, int J) {
  const SpdTaskDev t = tasks ? tasks[blockIdx.x] : one;
  if (GB * J >= t.k) return;
  const int bj = blk_size(t.k, J);
  const double* src = t.S + (int64_t)GB * J * (t.k + 1);
  spd_inverse_body<TY, NA, NB>(src, t.k, t.scratch, GB, bj);
}

int g_diag_variant = 0;

// step 2: R = Di S_J. (64 x k) and C = S_.J (k x 64); blockIdx.x = column
// tile of 64, blockIdx.y = matrix
__global__ void __launch_bounds__(256) gj_panel_kernel(const SpdTaskDev* __restrict__ tasks,
                                                       SpdTaskDev one, int J) {
  const SpdTaskDev t = tasks ? tasks[blockIdx.y] : one;
  const int k = t.k;
  const int c0 = GB * blockIdx.x;
  if (GB * J >= k || c0 >= k) return;
  const int bj = blk_size(k, J), bc = blk_size(k, blockIdx.x);
  const double* Di = t.scratch;
  double* R = t.scratch + GB * GB;              // ld 64
  double* C = R + (int64_t)GB * k;              // ld k
  __shared__ double sD[GB][GB + 1];
  __shared__ double sS[GB][GB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < GB * GB; e += 256) {
    const int i = e % GB, j = e / GB;
    sD[i][j] = (i < bj && j < bj) ? Di[i + j * GB] : 0.0;
    sS[i][j] = (i < bj && j < bc) ? t.S[(GB * J + i) + (int64_t)(c0 + j) * k] : 0.0;
  }
  // the old column block J, rows of this tile
  for (int e = tid; e < GB * GB; e += 256) {
    const int i = e % GB, j = e / GB;
    if (i < bc && j < bj) C[(c0 + i) + (int64_t)j * k] = t.S[(c0 + i) + (int64_t)(GB * J + j) * k];
  }
  __syncthreads();
  if ((int)blockIdx.x == J) return;              // R is not needed for the pivot columns
  for (int e = tid; e < GB * GB; e += 256) {
    const int i = e % GB, j = e / GB;
    if (i >= bj || j >= bc) continue;
    double acc = 0.0;
    for (int q = 0; q < bj; ++q) acc = __fma_rn(sD[i][q], sS[q][j], acc);
    R[i + (int64_t)(c0 + j) * GB] = acc;
  }
}

// step 3: every tile (I, c) of S from Di, R and C; blockIdx.x = I + nb c,
// blockIdx.y = matrix
__global__ void __launch_bounds__(256) gj_update_kernel(const SpdTaskDev* __restrict__ tasks,
                                                        SpdTaskDev one, int J) {
  const SpdTaskDev t = tasks ? tasks[blockIdx.y] : one;
  const int k = t.k;
  const int nb = (k + GB - 1) / GB;
  if (GB * J >= k || (int)blockIdx.x >= nb * nb) return;
  const int I = blockIdx.x % nb, cb = blockIdx.x / nb;
  const int bj = blk_size(k, J), bi = blk_size(k, I), bc = blk_size(k, cb);
  const int r0 = GB * I, c0 = GB * cb;
  const double* Di = t.scratch;
  const double* R = t.scratch + GB * GB;
  const double* C = R + (int64_t)GB * k;
  __shared__ double sA[GB][GB + 1];   // rows of C (or Di)
  __shared__ double sB[GB][GB + 1];   // columns of R (or Di)
  const int tid = threadIdx.x;
  const bool rowJ = I == J, colJ = cb == J;
  if (rowJ && colJ) {
    for (int e = tid; e < GB * GB; e += 256) {
      const int i = e % GB, j = e / GB;
      if (i < bi && j < bc) t.S[(r0 + i) + (int64_t)(c0 + j) * k] = Di[i + j * GB];
    }
    return;
  }
  if (rowJ) {
    for (int e = tid; e < GB * GB; e += 256) {
      const int i = e % GB, j = e / GB;
      if (i < bi && j < bc) t.S[(r0 + i) + (int64_t)(c0 + j) * k] = R[i + (int64_t)(c0 + j) * GB];
    }
    return;
  }
  for (int e = tid; e < GB * GB; e += 256) {
    const int i = e % GB, q = e / GB;
    sA[i][q] = (i < bi && q < bj) ? C[(r0 + i) + (int64_t)q * k] : 0.0;
    if (colJ) sB[i][q] = (i < bj && q < bj) ? Di[i + q * GB] : 0.0;          // sB[q'][j]
    else sB[i][q] = (i < bj && q < bc) ? R[i + (int64_t)(c0 + q) * GB] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < GB * GB; e += 256) {
    const int i = e % GB, j = e / GB;
    if (i >= bi || j >= bc) continue;
    double acc = 0.0;
    for (int q = 0; q < bj; ++q) acc = __fma_rn(sA[i][q], sB[q][j], acc);
    double* out = &t.S[(r0 + i) + (int64_t)(c0 + j) * k];
    *out = colJ ? -acc : *out - acc;
  }
}

}  // namespace

bool spd_inverse_supported(int64_t k) { return k >= 1 && k <= kSpdMaxK; }

size_t spd_inverse_scratch_elems(int64_t k) {
  return (size_t)GB * GB + 2 * (size_t)GB * (size_t)k;
}

namespace {
hipError_t blocked_steps(const SpdTaskDev* tasks, SpdTaskDev one, int count, int64_t kmax,
                         hipStream_t s) {
  const int nb = (int)((kmax + GB - 1) / GB);
  for (int J = 0; J < nb; ++J) {
    switch (g_diag_variant) {
      case 1: hipLaunchKernelGGL((gj_diag_kernel<8, 8, 2>), dim3((unsigned)count), dim3(256), 0, s, tasks, one, J); break;
      case 2: hipLaunchKernelGGL((gj_diag_kernel<4, 16, 2>), dim3((unsigned)count), dim3(128), 0, s, tasks, one, J); break;
      case 3: hipLaunchKernelGGL((gj_diag_kernel<2, 32, 2>), dim3((unsigned)count), dim3(64), 0, s, tasks, one, J); break;
      default: hipLaunchKernelGGL((gj_diag_kernel<32, 2, 2>), dim3((unsigned)count), dim3(1024), 0, s, tasks, one, J); break;
    }
    hipLaunchKernelGGL(gj_panel_kernel, dim3((unsigned)nb, (unsigned)count), dim3(256), 0, s,
                       tasks, one, J);
    hipLaunchKernelGGL(gj_update_kernel, dim3((unsigned)(nb * nb), (unsigned)count), dim3(256),
                       0, s, tasks, one, J);
  }
  return hipGetLastError();
}
}  // namespace

void spd_force_diag_variant(int v) { g_diag_variant = v; }

hipError_t launch_spd_inverse_blocked(const SpdTaskDev* tasks, int count, int64_t kmax,
                                      hipStream_t s) {
  if (count <= 0) return hipSuccess;
  return blocked_steps(tasks, SpdTaskDev{nullptr, 0, nullptr}, count, kmax, s);
}

hipError_t launch_spd_inverse_scratch(double* S, int64_t k, double* scratch, hipStream_t s) {
  if (!spd_inverse_supported(k)) return hipErrorInvalidValue;
  if (k <= 64) return launch_spd_inverse(S, k, s);
  if (!scratch) return hipErrorInvalidValue;
  return blocked_steps(nullptr, SpdTaskDev{S, (int)k, scratch}, 1, k, s);
}

hipError_t launch_spd_inverse(double* S, int64_t k, hipStream_t s) {
  if (!spd_inverse_supported(k) || k > 208) return hipErrorInvalidValue;
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
  if (kmax > 64) return launch_spd_inverse_blocked(tasks, count, kmax, s);
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
