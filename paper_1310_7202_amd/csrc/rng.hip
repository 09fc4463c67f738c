// Step 1 of Algorithm 4.1 (Shabat et al., Section 4): the n x l test matrix G
// of i.i.d. zero-mean, unit-variance Gaussian entries.
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
                                                       int64_t l, uint32_t k0, uint32_t k1) {
  gaussian_body<T>(G, ldg, n, l, k0, k1);
}

// blockIdx.y selects the matrix of a batch
template <typename T>
__global__ void __launch_bounds__(256) gaussian_batched_kernel(const GaussTaskDev* __restrict__ tasks) {
  const GaussTaskDev t = tasks[blockIdx.y];
  gaussian_body<T>((T*)t.G, t.ldg, t.n, t.l, (uint32_t)(t.seed & 0xffffffffu),
                   (uint32_t)(t.seed >> 32));
}

}  // namespace

template <typename T>
hipError_t launch_gaussian(T* G, int64_t ldg, int64_t n, int64_t l, uint64_t seed,
                           hipStream_t s) {
  const int64_t npairs = (n * l + 1) / 2;
  int64_t blocks = (npairs + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(gaussian_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, G, ldg, n, l,
                     (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  return hipGetLastError();
}

template hipError_t launch_gaussian<double>(double*, int64_t, int64_t, int64_t, uint64_t,
                                            hipStream_t);
template hipError_t launch_gaussian<float>(float*, int64_t, int64_t, int64_t, uint64_t,
                                           hipStream_t);

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
