// Device-side building blocks shared by the HIP kernels of librlu.
//
// gfx950 (CDNA4) only: 64-lane wavefronts, MFMA matrix cores.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rlu {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// MFMA 16x16x4 tiles (one wavefront).
//
// Operand layout (both precisions): lane = i + 16*kk holds A[i][kk] and
// lane = j + 16*kk holds B[kk][j], i, j in [0,16), kk in [0,4).
// Result layout differs:
//   f64 (v_mfma_f64_16x16x4_f64): lane l, slot v holds D[l/16 + 4v][l%16]
//   f32 (v_mfma_f32_16x16x4_f32): lane l, slot v holds D[4(l/16) + v][l%16]
// ---------------------------------------------------------------------------
template <typename T> struct Mfma;

template <> struct Mfma<double> {
  typedef d4 acc_t;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <> struct Mfma<float> {
  typedef f4 acc_t;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// ---------------------------------------------------------------------------
// Unit-lower factor of Step 3 read in place (rows never move).
//
// After the pivoted LU of Y, row `row` of the packed storage holds its
// multipliers for the steps at which it was still active and, if it was
// chosen as the pivot of step s = rstep[row], the U_y row from column s on.
// The unit-lower factor in original row order is therefore
//   Lv(row, r) = Y(row, r)  if r < rstep[row]
//              = 1          if r == rstep[row]
//              = 0          if r > rstep[row]
// (rstep = number of columns for a row never chosen).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T lv_value(T stored, int r, int s) {
  return r < s ? stored : (r == s ? T(1) : T(0));
}

// FP16 range of the mixed form: the products round s A to 16 bits with s a
// power of two that puts max|A| s in [2^13, 2^14) (FP16 then keeps 11
// significant bits from the largest entry down to 2^-24 of it, far from
// 65504), and their FP64 results are multiplied by 1/s: both exact.  s = 1
// without a maximum (BF16 has FP32's exponent range), or when it is zero or
// not finite.  amax holds max|A| as FP32 bits.
__device__ __forceinline__ float lp_scale(const unsigned* amax) {
  if (!amax) return 1.f;
  const float m = __uint_as_float(*amax);
  if (!(m > 0.f) || m > 3.0e38f) return 1.f;
  int e;
  (void)frexpf(m, &e);  // m = f 2^e, f in [1/2, 1)
  const int sh = min(max(14 - e, -100), 100);
  return ldexpf(1.f, sh);
}

// ---------------------------------------------------------------------------
// Wall clock (100 MHz constant clock on gfx9) for bounded waits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long now_ticks() { return (long long)wall_clock64(); }

// Agent-scope (whole device) relaxed load / store of 64-bit words.
__device__ __forceinline__ unsigned long long ld_agent(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_agent_i(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent_i(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-level reductions (64 lanes) through cross-lane shuffles.
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

}  // namespace rlu
