// Step 1 of Algorithm 4.1 (Shabat et al., Section 4): the n x l test matrix G
// of i.i.d. zero-mean, unit-variance Gaussian entries; and Step 1 of
// Algorithm 4.4 (Section 4.5): the SRFT R = D F S of Section 3.3.
//
// Generator (the paper names none): Philox4x32-10 (Salmon, Moraes, Dror and
// Shaw, SC'11) keyed by the 64-bit seed, one counter per pair of elements in
// column-major order, followed by the Box-Muller transform (Box and Muller,
// 1958) in FP64.  The exact convention is documented in include/rlu.h.
#include "rlu_device.h"
#include "rlu_kernels.h"

namespace rlu {
namespace {

struct Words { uint32_t x0, x1, x2, x3; };

__device__ __forceinline__ Words philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    const uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
    const uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return Words{c0, c1, c2, c3};
}

template <typename T>
__device__ __forceinline__ void gaussian_body(T* __restrict__ G, int64_t ldg, int64_t n,
                                              int64_t l, uint32_t k0, uint32_t k1) {
  const int64_t total = n * l;
  const int64_t npairs = (total + 1) >> 1;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npairs;
       t += (int64_t)gridDim.x * blockDim.x) {
    const Words w = philox10((uint32_t)t, (uint32_t)((uint64_t)t >> 32), 0u, 0u, k0, k1);
    const uint64_t a = ((uint64_t)w.x1 << 32) | w.x0;
    const uint64_t b = ((uint64_t)w.x3 << 32) | w.x2;
    const double u1 = (double)((a >> 11) + 1ull) * 0x1.0p-53;  // (0, 1]
    const double u2 = (double)(b >> 11) * 0x1.0p-53;           // [0, 1)
    const double r = sqrt(-2.0 * log(u1));
    const double theta = (2.0 * M_PI) * u2;
    const double z0 = r * cos(theta), z1 = r * sin(theta);
    const int64_t e0 = 2 * t;
    {
      const int64_t i = e0 % n, j = e0 / n;
      G[i + j * ldg] = (T)z0;
    }
    if (e0 + 1 < total) {
      const int64_t e1 = e0 + 1;
      const int64_t i = e1 % n, j = e1 / n;
      G[i + j * ldg] = (T)z1;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) gaussian_kernel(T* __restrict__ G, int64_t ldg, int64_t n,
                                                       int64_t l, uint32_t k0, uint32_t k1,
                                                       uint32_t* __restrict__ clear) {
  if (clear && blockIdx.x == 0 && threadIdx.x < 16) clear[threadIdx.x] = 0u;
  gaussian_body<T>(G, ldg, n, l, k0, k1);
}

// blockIdx.y selects the matrix of a batch
template <typename T>
__global__ void __launch_bounds__(256) gaussian_batched_kernel(const GaussTaskDev* __restrict__ tasks) {
  const GaussTaskDev t = tasks[blockIdx.y];
  gaussian_body<T>((T*)t.G, t.ldg, t.n, t.l, (uint32_t)(t.seed & 0xffffffffu),
                   (uint32_t)(t.seed >> 32));
}

// ---------------------------------------------------------------------------
// The SRFT R = D F S (n x l) of Algorithm 4.4, with F the orthonormal
// discrete Hartley transform, F(i, c) = (cos + sin)(2 pi i c / n) / sqrt(n),
// D = diag(+1 / -1) and S selecting l distinct columns in a random order.
// Draws (same generator and key as Step 1, third counter word 1 and 2):
//   sign of row i: bit i mod 128 of the four words of counter
//     (i div 128, 0, 1, 0), as bit (i mod 32) of word ((i mod 128) div 32);
//     the bit 0 gives +1.
//   selection: a partial Fisher-Yates shuffle of 0..n-1; step j takes u =
//     (x1:x0) of counter (j, 0, 2, 0) and exchanges positions j and
//     j + (u mod (n - j)); S's column j is the index left at position j.
// ---------------------------------------------------------------------------
constexpr int kSelMax = 1024;          // largest l of the selection kernel
constexpr int kSelSlots = 4 * kSelMax; // open-addressing map of moved positions (<= l used)

__device__ __forceinline__ int sel_find(const int* keys, int pos) {
  unsigned h = ((unsigned)pos * 2654435761u) & (kSelSlots - 1);
  while (keys[h] != pos && keys[h] != -1) h = (h + 1) & (kSelSlots - 1);
  return (int)h;
}

// One wave: the lanes draw the l words, lane 0 runs the shuffle over a map
// of the (at most l) positions beyond the current step that it has moved;
// untouched positions hold themselves.  Position j is final once step j is
// done (later steps only touch positions above it), so it is never stored.
__global__ void __launch_bounds__(64) srft_select_kernel(int64_t n, int l, uint32_t k0,
                                                         uint32_t k1, int* __restrict__ sel) {
  __shared__ unsigned long long u[kSelMax];
  __shared__ int keys[kSelSlots];
  __shared__ int vals[kSelSlots];
  const int lane = threadIdx.x;
  for (int j = lane; j < l; j += 64) {
    const Words w = philox10((uint32_t)j, 0u, 2u, 0u, k0, k1);
    u[j] = ((unsigned long long)w.x1 << 32) | w.x0;
  }
  for (int h = lane; h < kSelSlots; h += 64) keys[h] = -1;
  __syncthreads();
  if (lane == 0) {
    for (int j = 0; j < l; ++j) {
      const int t = j + (int)(u[j] % (unsigned long long)(n - j));
      const int hj = sel_find(keys, j);
      const int vj = keys[hj] == j ? vals[hj] : j;
      const int ht = sel_find(keys, t);
      const int vt = keys[ht] == t ? vals[ht] : t;
      keys[ht] = t; vals[ht] = vj;   // position j is never read again: not stored
      sel[j] = vt;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) srft_matrix_kernel(int64_t n, int l, uint32_t k0,
                                                          uint32_t k1, const int* __restrict__ sel,
                                                          T* __restrict__ R, int64_t ldr) {
  const double scale = 1.0 / sqrt((double)n);
  const int64_t total = n * (int64_t)l;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % n, j = e / n;
    const Words w = philox10((uint32_t)(i >> 7), 0u, 1u, 0u, k0, k1);
    const int t = (int)(i & 127);
    const uint32_t word = t < 32 ? w.x0 : t < 64 ? w.x1 : t < 96 ? w.x2 : w.x3;
    const double d = ((word >> (t & 31)) & 1u) ? -1.0 : 1.0;
    const int64_t r = (i * (int64_t)sel[j]) % n;
    double sn, cs;
    sincospi(2.0 * (double)r / (double)n, &sn, &cs);
    R[i + j * ldr] = (T)(d * (cs + sn) * scale);
  }
}

}  // namespace

template <typename T>
hipError_t launch_srft(T* R, int64_t ldr, int64_t n, int l, uint64_t seed, int* sel,
                       hipStream_t s) {
  if (n <= 0 || l <= 0) return hipSuccess;
  if (l > kSelMax || l > n || n >= (1LL << 31)) return hipErrorInvalidValue;
  const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  hipLaunchKernelGGL(srft_select_kernel, dim3(1), dim3(64), 0, s, n, l, k0, k1, sel);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t blocks = (n * l + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(srft_matrix_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, n, l, k0, k1,
                     sel, R, ldr);
  return hipGetLastError();
}
template hipError_t launch_srft<double>(double*, int64_t, int64_t, int, uint64_t, int*,
                                        hipStream_t);
template hipError_t launch_srft<float>(float*, int64_t, int64_t, int, uint64_t, int*, hipStream_t);

template <typename T>
hipError_t launch_gaussian(T* G, int64_t ldg, int64_t n, int64_t l, uint64_t seed,
                           hipStream_t s, uint32_t* clear) {
  const int64_t npairs = (n * l + 1) / 2;
  int64_t blocks = (npairs + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(gaussian_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, G, ldg, n, l,
                     (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), clear);
  return hipGetLastError();
}

template hipError_t launch_gaussian<double>(double*, int64_t, int64_t, int64_t, uint64_t,
                                            hipStream_t, uint32_t*);
template hipError_t launch_gaussian<float>(float*, int64_t, int64_t, int64_t, uint64_t,
                                           hipStream_t, uint32_t*);

template <typename T>
hipError_t launch_gaussian_batched(const GaussTaskDev* tasks, int count, int64_t max_elems,
                                   hipStream_t s) {
  if (count <= 0 || max_elems <= 0) return hipSuccess;
  int64_t bx = ((max_elems + 1) / 2 + 255) / 256;
  if (bx > 256) bx = 256;
  hipLaunchKernelGGL(gaussian_batched_kernel<T>, dim3((unsigned)bx, (unsigned)count), dim3(256),
                     0, s, tasks);
  return hipGetLastError();
}
template hipError_t launch_gaussian_batched<double>(const GaussTaskDev*, int, int64_t,
                                                    hipStream_t);
template hipError_t launch_gaussian_batched<float>(const GaussTaskDev*, int, int64_t,
                                                   hipStream_t);

}  // namespace rlu
