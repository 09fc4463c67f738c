// Streaming low-precision products of the mixed form of Algorithm 4.1
// (Shabat et al., Section 4): the two passes over A at HBM speed.
//
//   Step 2   Y (m x l) = A G     A: FP32, column-major; G pre-converted once
//                                to 16 bits, one row per output column
//   Step 5   C (k x n) = Lv^T A  Lv: FP64 in place in the packed LU of Y,
//                                pre-converted once to a 16-bit hi + lo pair
//
// Both run on BF16 (or FP16) MFMA 16x16x32 with FP32 accumulation.  A, the
// only large operand, is read from HBM exactly once: a workgroup owns a
// block of A (64 rows for Step 2, 64 columns for Step 5) across the whole
// product's other dimension, so no other workgroup reads it.  The small
// operand (G, or the Lv pair) is read by every workgroup; all workgroups
// start at the beginning of K and advance together, so the slice they need
// is in their XCD's L2 when they need it.
//
// MFMA 16x16x32 layout: lane i + 16 g holds row i (A operand) or column i
// (B operand) at k = 8g..8g+7; lane l, slot v of the result is
// D[4 (l / 16) + v][l % 16].
#include "rlu_device.h"
#include "rlu_kernels.h"

#include <climits>

namespace rlu {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <typename LP> struct Mma16;
template <> struct Mma16<__bf16> {
  typedef bf16x8 vec;
  static __device__ __forceinline__ f4 mma(vec a, vec b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct Mma16<_Float16> {
  typedef f16x8 vec;
  static __device__ __forceinline__ f4 mma(vec a, vec b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

constexpr int kBK = 32;           // K per step (one MFMA deep)
constexpr int kLd = kBK + 8;      // LDS row stride in 16-bit elements (80 bytes)
// Loads in flight: kDepth* steps of A, kPre* steps of the small operand (one
// register set per step, refilled right after the step's MFMAs).  The
// vector-memory counter retires loads in issue order, so a wait for the
// small operand of a step also waits for every A load issued before it: the
// small operand's distance bounds how far ahead A effectively runs, and the
// two distances are raised together.  Every load in the loop is
// unconditional (addresses clamped into the matrix, out-of-range values
// zeroed when they are rounded into LDS), so the body is one basic block and
// the counter waits count exactly how many loads may stay in flight.  The
// loop is unrolled kDepth* times (a multiple of kPre* and of 2, the LDS
// buffers).  The widest tiles keep the shallower distances their registers
// allow.
template <int TN> struct SketchDepth {
  static constexpr int kDepth = TN >= 12 ? 4 : 8, kPre = TN >= 12 ? 2 : 4;
};
template <int TR> struct ProjectDepth {  // the Lv pair takes twice the registers
  static constexpr int kDepth = TR >= 9 ? 4 : 6, kPre = TR >= 9 ? 2 : 3;
};

// ---------------------------------------------------------------------------
// Step 2.  Workgroup of NW waves (4, or 8 = two per SIMD when the columns
// split evenly): 64 rows of A x all N_pad = 64 TN columns; wave w owns
// columns [16 TNW w, 16 TNW (w + 1)), TNW = 4 TN / NW, for all 64 rows
// (4 x TNW MFMA tiles).  Per step the workgroup loads A(64 rows, 32 k),
// rounds it to 16 bits and stores it as [row][k] in LDS, and each wave
// reads its G fragments straight from the pre-converted Gb (row = output
// column, K contiguous).  A thread loads either four rows at consecutive k
// (VEC: 16-byte loads, for 16-byte aligned columns) or one row at several
// k (dword loads): a wave may have only so many loads in flight, so the
// wide form keeps more of A in flight per load issued.
// ---------------------------------------------------------------------------
template <typename LP, int TN, bool VEC, int NW>
__global__ void __launch_bounds__(64 * NW, 1)
sketch_stream_kernel(int64_t M, int64_t N, int64_t K, const float* __restrict__ A, int64_t lda,
                     const LP* __restrict__ Gs, double* __restrict__ C, int64_t ldc, int ksplit,
                     double* __restrict__ partial, int tiles_m, const unsigned* __restrict__ amax) {
  typedef typename Mma16<LP>::vec vec;
  constexpr int kDepthS = SketchDepth<TN>::kDepth, kPreS = SketchDepth<TN>::kPre;
  const float asc = lp_scale(amax);  // A's range scale (FP16), undone on the output
  const double ainv = 1.0 / (double)asc;
  constexpr int NP = 64 * TN;       // padded columns of Y
  constexpr int TNW = 4 * TN / NW;  // 16-column tiles of Y per wave
  constexpr int NT = 64 * NW;       // threads
  constexpr int RA = 2048 / NT;     // A values per thread and step (8 or 4)
  constexpr int VK = RA / 4;        // VEC: consecutive k per thread (2 or 1)
  __shared__ __attribute__((aligned(16))) LP As[2][64 * kLd];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bx = (int)(blockIdx.x % tiles_m), bz = (int)(blockIdx.x / tiles_m);
  const int64_t m0 = (int64_t)bx * 64;
  const int64_t kchunk = ((K + ksplit - 1) / ksplit + kBK - 1) / kBK * kBK;
  const int64_t kbeg = (int64_t)bz * kchunk;
  const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;
  const int nsteps = kbeg < kend ? (int)((kend - kbeg + kBK - 1) / kBK) : 0;
  const int64_t kstep0 = kbeg / kBK;

  f4 acc[4][TNW];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int t = 0; t < TNW; ++t) acc[a][t] = f4{0.f, 0.f, 0.f, 0.f};

  if (nsteps > 0) {
    // this thread's A row (clamped); its k group (RA consecutive k) is the
    // wave's, so the k offsets and their clamps are wave-uniform
    const int ar = tid & 63, ag = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool row_ok = m0 + ar < M;
    const int arow = (int)(row_ok ? m0 + ar : M - 1);
    const int64_t kend_t = row_ok ? kend : kbeg;  // no valid k on a row past M
    // VEC: rows 4 vi .. 4 vi + 3 (the group clamped into the matrix; rows
    // past M are zeroed when stored) at k VK vp .. VK vp + VK - 1
    const int vi = tid & 15, vp = tid >> 4;
    const int64_t vrow = m0 + 4 * vi < M ? m0 + 4 * vi : M - 4;
    float ring[kDepthS][RA];
    auto load_a = [&](int step, float* r) {
      if (VEC) {
        const int64_t k0 = kbeg + (int64_t)step * kBK + VK * vp;
#pragma unroll
        for (int e = 0; e < VK; ++e) {
          const int64_t kk = k0 + e < K ? k0 + e : K - 1;
          const float4 x = *(const float4*)(A + kk * lda + vrow);
          r[4 * e] = x.x; r[4 * e + 1] = x.y; r[4 * e + 2] = x.z; r[4 * e + 3] = x.w;
        }
      } else {
        const int64_t k0 = kbeg + (int64_t)step * kBK + RA * ag;
#pragma unroll
        for (int e = 0; e < RA; ++e) {
          const int64_t kk = k0 + e < K ? k0 + e : K - 1;
          r[e] = (A + kk * lda)[arow];
        }
      }
    };
    auto store_a = [&](int buf, int step, const float* r) {
      if (VEC) {
        typedef LP lpv __attribute__((ext_vector_type(VK)));
        const int64_t k0 = kbeg + (int64_t)step * kBK + VK * vp;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bool ok = m0 + 4 * vi + q < M;
          lpv v;
#pragma unroll
          for (int e = 0; e < VK; ++e) v[e] = (LP)((ok && k0 + e < kend ? r[4 * e + q] : 0.f) * asc);
          *(lpv*)&As[buf][(4 * vi + q) * kLd + VK * vp] = v;
        }
      } else {
        typedef LP lpv __attribute__((ext_vector_type(RA)));
        const int64_t k0 = kbeg + (int64_t)step * kBK + RA * ag;
        lpv v;
#pragma unroll
        for (int e = 0; e < RA; ++e) v[e] = (LP)((k0 + e < kend_t ? r[e] : 0.f) * asc);
        *(lpv*)&As[buf][ar * kLd + RA * ag] = v;
      }
    };
    // this wave's G fragments: column n0w + 16 t + (lane & 15), k 8 (lane >> 4);
    // steps past the end re-read the last step (their A is zero)
    // (16-byte units: a step block is NP rows x 4; a 16-row tile is 64)
    const int gv = (wave * 16 * TNW + (lane & 15)) * 4 + (lane >> 4);
    auto load_g = [&](int step, vec* g) {
      const int st = step < nsteps ? step : nsteps - 1;
      const vec* blk = (const vec*)Gs + (kstep0 + st) * (int64_t)(NP * 4);
#pragma unroll
      for (int t = 0; t < TNW; ++t) g[t] = blk[gv + 64 * t];
    };

    vec gset[kPreS][TNW];
#pragma unroll
    for (int d = 0; d < kDepthS; ++d) load_a(d, ring[d]);
#pragma unroll
    for (int d = 0; d < kPreS; ++d) {
      __builtin_amdgcn_sched_barrier(0);
      load_g(d, gset[d]);
    }
    __builtin_amdgcn_sched_barrier(0);
    store_a(0, 0, ring[0]);
    load_a(kDepthS, ring[0]);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    const int kof = 8 * (lane >> 4);
    const int nloop = (nsteps + kDepthS - 1) / kDepthS * kDepthS;
    for (int s0 = 0; s0 < nloop; s0 += kDepthS) {
#pragma unroll
      for (int u = 0; u < kDepthS; ++u) {
        const int s = s0 + u, buf = u & 1;
        vec af[4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
          af[a] = *(const vec*)&As[buf][(16 * a + (lane & 15)) * kLd + kof];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int t = 0; t < TNW; ++t) acc[a][t] = Mma16<LP>::mma(af[a], gset[u % kPreS][t], acc[a][t]);
        // program order is kept (the fences stop the scheduler from moving
        // the refills, and with them the counter waits, across the MFMAs)
        __builtin_amdgcn_sched_barrier(0);
        load_g(s + kPreS, gset[u % kPreS]);
        __builtin_amdgcn_sched_barrier(0);
        // step s+1's A (loaded kDepthS - 1 steps ago) into the other buffer,
        // then that ring slot takes step s+1+kDepthS
        store_a(buf ^ 1, s + 1, ring[(u + 1) % kDepthS]);
        load_a(s + 1 + kDepthS, ring[(u + 1) % kDepthS]);
        __builtin_amdgcn_sched_barrier(0);
        __syncthreads();
      }
    }
  }

  double* out = ksplit > 1 ? partial + (int64_t)bz * M * N : C;
  const int64_t ldo = ksplit > 1 ? M : ldc;
  const int64_t n0w = (int64_t)wave * 16 * TNW;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int t = 0; t < TNW; ++t) {
      const int64_t col = n0w + 16 * t + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + 16 * a + 4 * (lane >> 4) + v;
        if (row < M && col < N) out[row + col * ldo] = (double)acc[a][t][v] * ainv;
      }
    }
}

// Gs (step-major, NP padded columns): for each step of 32 k, row j holds
// G(32 step .. 32 step + 31, j) rounded to 16 bits; zero padding.
template <typename LP>
__global__ void __launch_bounds__(256) convert_g_kernel(const float* __restrict__ G, int64_t ldg,
                                                        int64_t K, int64_t N, LP* __restrict__ Gs,
                                                        int64_t np, int64_t ksteps) {
  const int64_t total = ksteps * np * kBK;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t kq = e % kBK, j = (e / kBK) % np, kk = (e / (kBK * np)) * kBK + kq;
    Gs[e] = (LP)((j < N && kk < K) ? G[kk + j * ldg] : 0.f);
  }
}

template <typename LP>
hipError_t launch_sketch_stream(const GemmDesc& d, hipStream_t s) {
  const int64_t npad = stream_sketch_npad(d.N), ksteps = (d.K + kBK - 1) / kBK;
  LP* Gs = (LP*)d.lp_ws;
  {
    int64_t blocks = (npad * ksteps * kBK + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(convert_g_kernel<LP>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const float*)d.B, d.ldb, d.K, d.N, Gs, npad, ksteps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int tiles_m = (int)((d.M + 63) / 64);
  int ks = 1;
  if (d.partial)
    while (tiles_m * ks < 256 && d.K / (ks * 2) >= 1024 && ks < 16) ks *= 2;
  if (d.ksplit_out) *d.ksplit_out = ks;
  const int tn = (int)(npad / 64);
  const dim3 grid((unsigned)(tiles_m * ks));
  const bool vec = d.M % 4 == 0 && d.lda % 4 == 0 && ((uintptr_t)d.A & 15) == 0;
#define RLU_SKS1(TN, V, NW)                                                                   \
  hipLaunchKernelGGL((sketch_stream_kernel<LP, TN, V, NW>), grid, dim3(64 * NW), 0, s, d.M,    \
                     d.N, d.K, (const float*)d.A, d.lda, (const LP*)Gs, (double*)d.C, d.ldc,  \
                     ks, (double*)d.partial, tiles_m, d.amax)
  // eight waves (two per SIMD) where the columns split evenly over them
#define RLU_SKS(TN)                              \
  if (vec)                                       \
    RLU_SKS1(TN, true, (TN % 2 == 0 ? 8 : 4));   \
  else                                           \
    RLU_SKS1(TN, false, (TN % 2 == 0 ? 8 : 4))
  switch (tn) {
    case 1: RLU_SKS(1); break;
    case 2: RLU_SKS(2); break;
    case 4: RLU_SKS(4); break;
    case 6: RLU_SKS(6); break;
    case 8: RLU_SKS(8); break;
    case 9: RLU_SKS(9); break;
    case 12: RLU_SKS(12); break;
    default: return hipErrorInvalidValue;
  }
#undef RLU_SKS
#undef RLU_SKS1
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ks == 1 || d.no_sum) return e;
  return launch_splitk_sum_f64(d.M, d.N, ks, (const double*)d.partial, (double*)d.C, d.ldc,
                               nullptr, s);
}

// ---------------------------------------------------------------------------
// Step 5.  C (R x N) = Lv^T A.  Workgroup of NW waves (4, or 8 = two per
// SIMD when the rows split evenly): 64 columns of A x all R_pad = 64 TR rows
// of C; wave w owns rows [16 TRW w, 16 TRW (w + 1)), TRW = 4 TR / NW, for
// all 64 columns (TRW x 4 MFMA tiles, two MFMAs each for the hi and lo parts
// of Lv).  Per step the workgroup loads A(32 k, 64 columns) (a wave: 8
// columns x 128 contiguous bytes per float4 load), rounds it to 16 bits into
// LDS as [column][k] (the B-fragment layout), and each wave reads its Lv
// fragments straight from the pre-converted pair (row i of Lv^T, K
// contiguous).
// ---------------------------------------------------------------------------
template <typename LP, int TR, bool VEC, int NW>
__global__ void __launch_bounds__(64 * NW, 1)
project_stream_kernel(int64_t M, int64_t N, int64_t K, const LP* __restrict__ Ls,
                      const float* __restrict__ A, int64_t lda, double* __restrict__ C,
                      int64_t ldc, int ksplit, double* __restrict__ partial, int tiles_n,
                      const unsigned* __restrict__ amax) {
  typedef typename Mma16<LP>::vec vec;
  constexpr int kDepthP = ProjectDepth<TR>::kDepth, kPreP = ProjectDepth<TR>::kPre;
  const float asc = lp_scale(amax);  // A's range scale (FP16), undone on the output
  const double ainv = 1.0 / (double)asc;
  constexpr int RP = 64 * TR;      // padded rows of C
  constexpr int TRW = 4 * TR / NW;  // 16-row tiles of C per wave
  constexpr int NT = 64 * NW;       // threads
  constexpr int AJ = 512 / NT;      // float4 of A per thread and step
  typedef LP lp4 __attribute__((ext_vector_type(4)));
  __shared__ __attribute__((aligned(16))) LP Bs[2][64 * kLd];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bx = (int)(blockIdx.x % tiles_n), bz = (int)(blockIdx.x / tiles_n);
  const int64_t n0 = (int64_t)bx * 64;
  const int64_t kchunk = ((K + ksplit - 1) / ksplit + kBK - 1) / kBK * kBK;
  const int64_t kbeg = (int64_t)bz * kchunk;
  const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;
  const int nsteps = kbeg < kend ? (int)((kend - kbeg + kBK - 1) / kBK) : 0;
  const int64_t kstep0 = kbeg / kBK;
  const int64_t r0w = (int64_t)wave * 16 * TRW;

  f4 acc[TRW][4];
#pragma unroll
  for (int a = 0; a < TRW; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = f4{0.f, 0.f, 0.f, 0.f};

  if (nsteps > 0) {
    // this thread's two float4 of A per step: column f >> 3 (clamped), k 4 (f & 7)
    int bcol[AJ], bk[AJ];
    int64_t kend_t[AJ];  // kbeg on a column past N: no valid k there
    const float* Acol[AJ];
#pragma unroll
    for (int j = 0; j < AJ; ++j) {
      const int f = tid + NT * j;
      bcol[j] = f >> 3;
      bk[j] = 4 * (f & 7);
      const bool col_ok = n0 + bcol[j] < N;
      kend_t[j] = col_ok ? kend : kbeg;
      Acol[j] = A + (col_ok ? n0 + bcol[j] : N - 1) * lda;
    }
    const int64_t kmax4 = (K - 4) & ~(int64_t)3;  // last aligned float4 inside a column
    float4 ring[kDepthP][AJ];
    auto load_a = [&](int step, float4* r) {
      const int64_t k0 = kbeg + (int64_t)step * kBK;
#pragma unroll
      for (int j = 0; j < AJ; ++j) {
        const int64_t kk = k0 + bk[j];
        if (VEC) {
          r[j] = *(const float4*)(Acol[j] + (kk < kmax4 ? kk : kmax4));
        } else {
          float t[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) t[e] = Acol[j][kk + e < K ? kk + e : K - 1];
          r[j] = float4{t[0], t[1], t[2], t[3]};
        }
      }
    };
    auto store_a = [&](int buf, int step, const float4* r) {
      const int64_t k0 = kbeg + (int64_t)step * kBK;
#pragma unroll
      for (int j = 0; j < AJ; ++j) {
        const int64_t kk = k0 + bk[j];
        const float x[4] = {r[j].x, r[j].y, r[j].z, r[j].w};
        lp4 v;
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (LP)((kk + e < kend_t[j] ? x[e] : 0.f) * asc);
        *(lp4*)&Bs[buf][bcol[j] * kLd + bk[j]] = v;
      }
    };
    // this wave's Lv fragments: row r0w + 16 a + (lane & 15), k 8 (lane >> 4);
    // steps past the end re-read the last step (their A is zero)
    // (16-byte units: a step block is 2 x RP rows x 4, hi then lo; a
    // 16-row tile is 64)
    const int lv = (wave * 16 * TRW + (lane & 15)) * 4 + (lane >> 4);
    auto load_l = [&](int step, vec* h, vec* lo) {
      const int st = step < nsteps ? step : nsteps - 1;
      const vec* blk = (const vec*)Ls + (kstep0 + st) * (int64_t)(2 * RP * 4);
#pragma unroll
      for (int a = 0; a < TRW; ++a) {
        h[a] = blk[lv + 64 * a];
        lo[a] = blk[RP * 4 + lv + 64 * a];
      }
    };

    vec hset[kPreP][TRW], lset[kPreP][TRW];
#pragma unroll
    for (int d = 0; d < kDepthP; ++d) load_a(d, ring[d]);
#pragma unroll
    for (int d = 0; d < kPreP; ++d) {
      __builtin_amdgcn_sched_barrier(0);
      load_l(d, hset[d], lset[d]);
    }
    __builtin_amdgcn_sched_barrier(0);
    store_a(0, 0, ring[0]);
    load_a(kDepthP, ring[0]);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    const int kof = 8 * (lane >> 4);
    const int nloop = (nsteps + kDepthP - 1) / kDepthP * kDepthP;
    for (int s0 = 0; s0 < nloop; s0 += kDepthP) {
#pragma unroll
      for (int u = 0; u < kDepthP; ++u) {
        const int s = s0 + u, buf = u & 1;
        vec bf[4];
#pragma unroll
        for (int c = 0; c < 4; ++c)
          bf[c] = *(const vec*)&Bs[buf][(16 * c + (lane & 15)) * kLd + kof];
#pragma unroll
        for (int a = 0; a < TRW; ++a)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            acc[a][c] = Mma16<LP>::mma(hset[u % kPreP][a], bf[c], acc[a][c]);
            acc[a][c] = Mma16<LP>::mma(lset[u % kPreP][a], bf[c], acc[a][c]);
          }
        __builtin_amdgcn_sched_barrier(0);
        load_l(s + kPreP, hset[u % kPreP], lset[u % kPreP]);
        __builtin_amdgcn_sched_barrier(0);
        store_a(buf ^ 1, s + 1, ring[(u + 1) % kDepthP]);
        load_a(s + 1 + kDepthP, ring[(u + 1) % kDepthP]);
        __builtin_amdgcn_sched_barrier(0);
        __syncthreads();
      }
    }
  }

  double* out = ksplit > 1 ? partial + (int64_t)bz * M * N : C;
  const int64_t ldo = ksplit > 1 ? M : ldc;
#pragma unroll
  for (int a = 0; a < TRW; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t col = n0 + 16 * c + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0w + 16 * a + 4 * (lane >> 4) + v;
        if (row < M && col < N) out[row + col * ldo] = (double)acc[a][c][v] * ainv;
      }
    }
}

// Ls (step-major, RP padded rows): for each step of 32 k, the hi parts of
// rows 0..RP-1 of Lv^T, then their lo parts, 32 k contiguous per row.  Row i
// is column i of Lv (m x R, read in place from the packed LU with row steps
// rstep) as a 16-bit hi + lo pair; zero padding.
template <typename LP>
__global__ void __launch_bounds__(256) convert_lv_kernel(const double* __restrict__ Y, int64_t ldy,
                                                         const int* __restrict__ rstep, int64_t K,
                                                         int64_t R, LP* __restrict__ Ls, int64_t rp,
                                                         int64_t ksteps) {
  const int64_t total = ksteps * rp * kBK;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t kq = e % kBK, i = (e / kBK) % rp, ks = e / (kBK * rp), kk = ks * kBK + kq;
    double x = 0.0;
    if (i < R && kk < K) x = lv_value<double>(Y[kk + i * ldy], (int)i, rstep[kk]);
    const float xf = (float)x;
    const LP hi = (LP)xf;
    LP* blk = Ls + ks * 2 * rp * kBK;
    blk[i * kBK + kq] = hi;
    blk[(rp + i) * kBK + kq] = (LP)(float)(x - (double)(float)hi);
  }
}

template <typename LP>
hipError_t launch_project_stream(const GemmDesc& d, hipStream_t s) {
  const int64_t rpad = stream_project_rpad(d.M), ksteps = (d.K + kBK - 1) / kBK;
  LP* Ls = (LP*)d.lp_ws;
  {
    int64_t blocks = (rpad * ksteps * kBK + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(convert_lv_kernel<LP>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const double*)d.A, d.lda, d.astep, d.K, d.M, Ls, rpad, ksteps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int tiles_n = (int)((d.N + 63) / 64);
  int ks = 1;
  if (d.partial)
    while (tiles_n * ks < 256 && d.K / (ks * 2) >= 1024 && ks < 16) ks *= 2;
  if (d.ksplit_out) *d.ksplit_out = ks;
  const int tr = (int)(rpad / 64);
  const dim3 grid((unsigned)(tiles_n * ks));
  const bool vec = d.ldb % 4 == 0 && ((uintptr_t)d.B & 15) == 0;
#define RLU_PJS1(TR, V, NW)                                                                   \
  hipLaunchKernelGGL((project_stream_kernel<LP, TR, V, NW>), grid, dim3(64 * NW), 0, s, d.M,  \
                     d.N, d.K, (const LP*)Ls, (const float*)d.B, d.ldb, (double*)d.C, d.ldc,  \
                     ks, (double*)d.partial, tiles_n, d.amax)
  // eight waves (two per SIMD) where the rows of C split evenly over them
#define RLU_PJS(TR)                                 \
  if (vec)                                          \
    RLU_PJS1(TR, true, (TR % 2 == 0 ? 8 : 4));      \
  else                                              \
    RLU_PJS1(TR, false, (TR % 2 == 0 ? 8 : 4))
  switch (tr) {
    case 1: RLU_PJS(1); break;
    case 2: RLU_PJS(2); break;
    case 4: RLU_PJS(4); break;
    case 6: RLU_PJS(6); break;
    case 8: RLU_PJS(8); break;
    case 9: RLU_PJS(9); break;
    default: return hipErrorInvalidValue;
  }
#undef RLU_PJS
#undef RLU_PJS1
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ks == 1 || d.no_sum) return e;
  return launch_splitk_sum_f64(d.M, d.N, ks, (const double*)d.partial, (double*)d.C, d.ldc,
                               nullptr, s);
}

}  // namespace

int64_t stream_sketch_npad(int64_t N) {
  static const int kTn[] = {1, 2, 4, 6, 8, 9, 12};
  for (int t : kTn)
    if (N <= 64 * t) return 64 * t;
  return -1;
}

size_t stream_sketch_ws_bytes(int64_t K, int64_t N) {
  const int64_t npad = stream_sketch_npad(N);
  if (npad < 0) return 0;
  return (size_t)npad * (size_t)((K + kBK - 1) / kBK * kBK) * 2;
}

size_t stream_sketch_partial_elems(int64_t M, int64_t N, int64_t K) {
  const int tiles_m = (int)((M + 63) / 64);
  int ks = 1;
  while (tiles_m * ks < 256 && K / (ks * 2) >= 1024 && ks < 16) ks *= 2;
  return ks > 1 ? (size_t)ks * (size_t)M * (size_t)N : 0;
}

int64_t stream_project_rpad(int64_t R) {
  static const int kTr[] = {1, 2, 4, 6, 8, 9};
  for (int t : kTr)
    if (R <= 64 * t) return 64 * t;
  return -1;
}

size_t stream_project_ws_bytes(int64_t K, int64_t R) {
  const int64_t rpad = stream_project_rpad(R);
  if (rpad < 0) return 0;
  return 2 * (size_t)rpad * (size_t)((K + kBK - 1) / kBK * kBK) * 2;
}

size_t stream_project_partial_elems(int64_t R, int64_t N, int64_t K) {
  const int tiles_n = (int)((N + 63) / 64);
  int ks = 1;
  while (tiles_n * ks < 256 && K / (ks * 2) >= 1024 && ks < 16) ks *= 2;
  return ks > 1 ? (size_t)ks * (size_t)R * (size_t)N : 0;
}

bool stream_project_applies(const GemmDesc& d) {
  return d.opa == OpA::LvT && d.opb == OpB::Plain && d.lp_ws && d.K >= 1024 &&
         stream_project_rpad(d.M) > 0;
}

hipError_t launch_project_stream_lp(const GemmDesc& d, bool fp16, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0) return hipSuccess;
  return fp16 ? launch_project_stream<_Float16>(d, s) : launch_project_stream<__bf16>(d, s);
}

bool stream_sketch_applies(const GemmDesc& d) {
  return d.opa == OpA::Plain && d.opb == OpB::Plain && d.lp_ws && d.K >= 1024 &&
         stream_sketch_npad(d.N) > 0;
}

hipError_t launch_sketch_stream_lp(const GemmDesc& d, bool fp16, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0) return hipSuccess;
  return fp16 ? launch_sketch_stream<_Float16>(d, s) : launch_sketch_stream<__bf16>(d, s);
}

// ---------------------------------------------------------------------------
// max|A| of FP32 matrices, as FP32 bits by atomic maximum (non-negative
// floats order like their bits; a NaN ranks above every number and makes the
// scale 1, see lp_scale).
// ---------------------------------------------------------------------------
namespace {

__device__ __forceinline__ void absmax_block(const float* __restrict__ A, int64_t lda, int64_t m,
                                             int64_t n, unsigned* word, int64_t b0, int64_t bstep) {
  __shared__ unsigned red[4];
  unsigned best = 0;
  for (int64_t j = b0; j < n; j += bstep)  // a column per workgroup, rows over its threads
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
      const unsigned b = __float_as_uint(A[i + j * lda]) & 0x7fffffffu;
      best = b > best ? b : best;
    }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned x = (unsigned)__shfl_xor((int)best, o);
    best = x > best ? x : best;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned t = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) t = red[w] > t ? red[w] : t;
    if (t) atomicMax(word, t);
  }
}

__global__ void __launch_bounds__(256) absmax_kernel(const float* __restrict__ A, int64_t lda,
                                                     int64_t m, int64_t n, unsigned* word) {
  absmax_block(A, lda, m, n, word, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(256) absmax_batched_kernel(const AbsmaxTaskDev* __restrict__ tasks) {
  const AbsmaxTaskDev t = tasks[blockIdx.y];
  absmax_block(t.A, t.lda, t.m, t.n, t.word, blockIdx.x, gridDim.x);
}

}  // namespace

hipError_t launch_absmax(const float* A, int64_t lda, int64_t m, int64_t n, unsigned* word,
                         hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int64_t blocks = n < 4096 ? n : 4096;
  hipLaunchKernelGGL(absmax_kernel, dim3((unsigned)blocks), dim3(256), 0, s, A, lda, m, n, word);
  return hipGetLastError();
}

hipError_t launch_absmax_batched(const AbsmaxTaskDev* tasks, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(absmax_batched_kernel, dim3(64u, (unsigned)count), dim3(256), 0, s, tasks);
  return hipGetLastError();
}

}  // namespace rlu
