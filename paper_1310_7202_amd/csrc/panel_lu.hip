// LU with partial pivoting of a tall matrix X (nrows x ncols, ncols <= nrows),
// all ncols columns factored, as used twice by Algorithm 4.1 (Shabat et al.,
// Section 4):
//   Step 3  P Y = L_y U_y                 X = Y   (m x l)
//   Step 6  B Q = L_b U_b  via  Q^T B^T = L' U'   X = B^T (n x k), whose rows
//           are the columns of B: row pivoting of B^T is column pivoting of
//           B and produces the same pivot sequence.
// The Remark after Algorithm 4.1 allows partial pivoting in Step 3.
//
// Two kernels: panel_lu_kernel below for panels spread over workgroups, and
// panel_small_kernel (further down) for panels of at most 32 columns whose
// rows fit one workgroup's registers; both make the same choices and give
// the same bits.
//
// Design of the spread kernel (one persistent launch, no host round trip):
//   * workgroup w keeps rows [w R, (w+1) R) of X resident in LDS for the whole
//     factorization; rows never move ("virtual" pivoting): each row records
//     its current position (to reproduce LAPACK's swap bookkeeping and its
//     lowest-position tie break) and the step that chose it.
//   * step j: wave 0 brings column j up to date, finds the workgroup's best
//     candidate (largest magnitude, lowest current position on ties) and
//     publishes its key: the candidate's value in column j (whose magnitude
//     ranks it), position and row, its multiplier of step j-1 and its value
//     in column j+1 *one update behind* (through step j-2); the bulk waves
//     publish the rest of the candidate's row, also one update behind.
//     Every workgroup polls the dense array of keys, selects the same
//     winner (whose key already carries everything the step needs from it,
//     so one device round trip decides the step); at the next step the bulk
//     waves fetch the winner's row and complete it themselves,
//         U(j, c) = row(c) - l(j-1) U(j-1, c),
//     with the same fused multiply-add the winner's own workgroup applies to
//     its copy, so all copies agree bitwise.  Publishing the row one update
//     behind lets the bulk waves apply the rank-one update of step j-1 while
//     wave 0 waits on the exchange: only the exchange latency and
//     O(R/64 + nwg/64) work per lane sit on the critical path.
//   * exchange protocol: every 64-bit word of a record carries the step tag
//     in its upper half and 32 bits of payload in its lower half (a double
//     takes two words).  Words are written and read with device-coherent
//     (agent-scope) relaxed atomic accesses, whose 64-bit single-copy
//     atomicity is all the protocol relies on: a reader accepts a key
//     or row entry only when every word it needs shows the current tag, so no
//     store ordering, fence or cache maintenance is needed and the writer
//     never waits.  Buffers rotate by step mod 3: a workgroup publishes step
//     j+3 only after the exchange of step j+2, which needs every workgroup's
//     step j+2 key, which each publishes only after it finished reading the
//     buffers of step j (the keys in its exchange, the winner's row in
//     its bulk update of step j+1).
//   * every wait is bounded by a wall-clock limit of its own (the clock
//     starts at the wait's first unsuccessful poll, so a long batched launch
//     whose later rounds start late never eats into a wait's budget); on
//     expiry the kernel sets a failure flag and all workgroups leave.
#include "rlu_device.h"
#include "rlu_kernels.h"

#include <algorithm>
#include <climits>
#include <cstdlib>

namespace rlu {
namespace {

// Threads per workgroup: 16 waves (one pivot wave, 15 bulk waves) when a
// lane holds one row (four waves per SIMD fit the registers), else 8 (two
// per SIMD, room for a whole poll of the exchange in flight).
template <int RPL>
constexpr int threads_for() { return RPL <= 1 ? 1024 : 512; }
inline int threads_for_rows(int R) { return R <= 64 ? 1024 : 512; }
constexpr int kNone = INT_MAX;

// Exchange buffer of a step: first a dense key area, 8 words per workgroup
// ([0,1] the candidate's value in column j, [2] its current position, [3]
// its original row or -1 for none, [4,5] its multiplier of step j-1, [6,7]
// its value in column j+1, one update behind like the row), which every
// workgroup polls; then one record per workgroup: 2 words per column of the
// candidate's row (entries from column j+2 on, written at step j by the
// bulk waves), read for the winner only.
constexpr int kKeyWords = 8;
constexpr int kHdrWords = 0;

__host__ __device__ __forceinline__ int64_t key_area_bytes(int nwg) {
  return (8 * (int64_t)kKeyWords * nwg + 127) / 128 * 128;
}

// Two tagged words (16 bytes, word index w) of an exchange buffer, moved
// with one device-coherent (sc1) buffer access, as the relaxed agent-scope
// 8-byte accesses are: half the requests.  Each 8-byte half is moved whole
// and carries its own tag, so a reader may pair halves of different steps
// only to reject them.  In a loaded value, .x/.y are the first word's
// payload and tag, .z/.w the second's.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr int kCoherent = 16;  // sc1
__device__ __forceinline__ Rsrc rsrc_of(const void* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0,
                                           (int)(bytes < INT_MAX ? bytes : INT_MAX), 0x00020000);
}
__device__ __forceinline__ u32x4 ld_words2(Rsrc r, int w) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, w * 8, 0, kCoherent);
}
__device__ __forceinline__ void st_words2(Rsrc r, int w, unsigned tag, unsigned p0, unsigned p1) {
  __builtin_amdgcn_raw_buffer_store_b128(u32x4{p0, tag, p1, tag}, r, w * 8, 0, kCoherent);
}
__device__ __forceinline__ bool tagged2(u32x4 v, unsigned tag) { return v.y == tag && v.w == tag; }
__device__ __forceinline__ unsigned long long payload2(u32x4 v) {
  return ((unsigned long long)v.z << 32) | v.x;
}

__device__ __forceinline__ unsigned long long dbits(double x) {
  return (unsigned long long)__double_as_longlong(x);
}
__device__ __forceinline__ double bitsd(unsigned long long x) {
  return __longlong_as_double((long long)x);
}
// Workgroup barrier that orders LDS only.  __syncthreads() also drains every
// outstanding global store of the wave first, which would put a full memory
// round trip (the exchange record just published) in front of each barrier;
// workgroup members here communicate through LDS alone.
__device__ __forceinline__ void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): LDS (and scalar) ops done
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// larger magnitude wins; equal magnitudes go to the lower current position
__device__ __forceinline__ bool better(double a2, int p2, double a, int p) {
  return a2 > a || (a2 == a && p2 < p);
}

// max(v, v of the lane selected by CTRL) through DPP; lanes without a source
// keep their own value (old operand = own value).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_max(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROW_MASK, 0xF, false);
  const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROW_MASK, 0xF, false);
  return fmax(v, __hiloint2double(hi2, lo2));
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_min(int v) {
  return min(v, __builtin_amdgcn_update_dpp(v, v, CTRL, ROW_MASK, 0xF, false));
}

// The lane (uniform) holding the best (a, p) of the wave: largest key a, then
// lowest position p.  Keys are never NaN, so max is exact: an inclusive max
// scan inside each row of 16 lanes (row_shr 1, 2, 4, 8), then row_bcast 15
// and 31 carry rows 0-1 and 0-3 into lane 63; a ballot finds the lanes that
// hold the maximum, and only when there are several does a second scan take
// the lowest position among them.
__device__ __forceinline__ int wave_best_lane(double a, int p) {
  double m = a;
  m = dpp_max<0x111, 0xF>(m);  // row_shr:1
  m = dpp_max<0x112, 0xF>(m);  // row_shr:2
  m = dpp_max<0x114, 0xF>(m);  // row_shr:4
  m = dpp_max<0x118, 0xF>(m);  // row_shr:8
  m = dpp_max<0x142, 0xA>(m);  // row_bcast:15 into rows 1 and 3
  m = dpp_max<0x143, 0xC>(m);  // row_bcast:31 into rows 2 and 3
  const double mx = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(m), 63),
                                     __builtin_amdgcn_readlane(__double2loint(m), 63));
  const unsigned long long hit = __ballot(a == mx);
  if (__popcll(hit) == 1) return __ffsll((long long)hit) - 1;
  int q = a == mx ? p : INT_MAX;
  q = dpp_min<0x111, 0xF>(q);
  q = dpp_min<0x112, 0xF>(q);
  q = dpp_min<0x114, 0xF>(q);
  q = dpp_min<0x118, 0xF>(q);
  q = dpp_min<0x142, 0xA>(q);
  q = dpp_min<0x143, 0xC>(q);
  const int qmin = __builtin_amdgcn_readlane(q, 63);
  return __ffsll((long long)__ballot(a == mx && p == qmin)) - 1;
}

// Value of lane `src` (uniform) in every lane.
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// RPL = rows per lane: lane l of a wave handles rows l, l+64, ..., so the
// workgroup holds at most 64 * RPL rows.
//
// Step j, with U(i, .) the U row of step i (the winner's row through step
// i-1) kept in a two-slot ring urow[i & 1]:
//   wave 0      U(j-1, j) from the step j-1 key; column j brought up to
//               date; local candidate; its key published          | B1 |
//               wait for all keys, select the winner (its key holds
//               everything wave 0 needs from it), bookkeeping,
//               multipliers of step j                                 | B0 |
//   bulk waves  start loading their columns of the step j-1 winner's
//               row                                                   | B1 |
//               publish their columns of the local candidate's row,
//               complete U(j-1, c) for their own columns c > j from
//               the loaded row, then the rank-one update of step j-1
//               on them                                               | B0 |
// so the only device round trip on wave 0's path is the key exchange; the
// bulk waves' own round trip (the winner's row) overlaps wave 0's work
// before B1 and its exchange after it.
// A bound on one wait: its clock starts at the wait's first unsuccessful
// poll (so a wait that succeeds at once never reads the clock) and the wait
// gives up once more than `tmo` ticks have passed since then.
struct WaitLimit {
  long long t0 = -1;
  // True when the wait should end: its own limit has passed, or another
  // workgroup has raised the failure word.  The word is read only once the
  // wait has lasted kFailCheckTicks (20 us): a normal wait ends well before
  // and pays no extra device round trip per poll for it.
  static constexpr long long kFailCheckTicks = 2000;
  __device__ __forceinline__ bool give_up(long long tmo, const int* fail) {
    const long long now = now_ticks();
    if (t0 < 0) {
      t0 = now;
      return false;
    }
    const long long waited = now - t0;
    if (waited > tmo) return true;
    return waited > kFailCheckTicks && ld_agent_i(fail) != 0;
  }
};

template <int RPL, int kThreads>
__device__ __forceinline__ void panel_body(
    double* __restrict__ X, int64_t rs, int64_t cs, int nrows, int ncols, int R, int nwg,
    int* __restrict__ pos_out, int* __restrict__ rstep_out, int* __restrict__ piv_row_out,
    int* __restrict__ ipiv_out, int* __restrict__ info_out, int* __restrict__ fail,
    char* __restrict__ xch, int64_t rec_stride, long long timeout_ticks, int w, double* smem,
    int step0, int total_cols, const int* __restrict__ pos_in,
    const int* __restrict__ rstep_in) {
  double* Ts = smem;                        // R x ncols, column-major (ld R)
  double* urow = Ts + (int64_t)R * ncols;   // 2 x ncols: U rows by step parity
  double* lbody = urow + 2 * ncols;         // 2 x ncols: single-workgroup "records"
  int* pos_s = (int*)(lbody + 2 * ncols);   // R: final positions (written at the end)
  int* step_s = pos_s + R;                  // R: step that chose the row, kNone if none
  int* pivrow_s = step_s + R;               // ncols: row chosen at each step
  int* ipiv_s = pivrow_s + ncols;           // ncols: its position before the swap
  __shared__ int sh_stop, sh_bw[2];
  __shared__ double sh_piv[2], sh_lm[2], sh_v1[2];   // winner header, by step parity
  __shared__ int sh_cr, sh_cp;                        // local candidate (one workgroup)
  __shared__ double sh_cpiv, sh_clm, sh_cv1;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row0 = w * R;
  // wave 0 carries the critical path and shares its SIMD with a bulk wave:
  // let it issue first
  if (wave == 0) __builtin_amdgcn_s_setprio(3);
  const int nr = min(R, nrows - row0);

  // ---- load the workgroup's rows into LDS ---------------------------------
  if (rs == 1) {
    for (int idx = tid; idx < R * ncols; idx += kThreads) {
      const int r = idx % R, c = idx / R;
      Ts[idx] = r < nr ? X[(int64_t)(row0 + r) + (int64_t)c * cs] : 0.0;
    }
  } else {
    for (int idx = tid; idx < R * ncols; idx += kThreads) {
      const int c = idx % ncols, r = idx / ncols;
      Ts[(int64_t)c * R + r] = r < nr ? X[(int64_t)(row0 + r) * rs + (int64_t)c * cs] : 0.0;
    }
  }
  // rows chosen by an earlier block of columns (global step < step0) stay
  // inactive: they hold U rows
  for (int r = tid; r < R; r += kThreads) {
    int st = kNone;
    if (rstep_in && r < nr) {
      const int s0 = rstep_in[row0 + r];
      if (s0 < step0) st = s0;
    }
    step_s[r] = st;
  }
  // the pivot row and position of every step start as valid indices (the
  // step's own row and position), so that a factorization that stops early
  // (an exchange failure) still hands its consumers, the assembly and the
  // column blocks' triangular solves, in-range rows
  for (int c = tid; c < ncols; c += kThreads) {
    pivrow_s[c] = c;
    ipiv_s[c] = step0 + c;
  }
  if (tid == 0) {
    sh_stop = 0;
    for (int t = 0; t < 2; ++t) { sh_bw[t] = -1; sh_piv[t] = 0.0; sh_lm[t] = 0.0; sh_v1[t] = 0.0; }
  }
  // wave 0's per-row state, in registers: position, choosing step, current
  // pivot-column value and the multiplier of the previous step
  int pos_q[RPL], st_q[RPL];
  double val_q[RPL], mlt_q[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int r = lane + 64 * q;
    pos_q[q] = (pos_in && r < nr) ? pos_in[row0 + r] : row0 + r;
    st_q[q] = -1;  // -1: no such row
    if (r < nr) {
      st_q[q] = kNone;
      if (rstep_in) {
        const int s0 = rstep_in[row0 + r];
        if (s0 < step0) st_q[q] = s0;
      }
    }
    val_q[q] = 0.0;
    mlt_q[q] = 0.0;
  }
  int info = 0;
  __syncthreads();

  constexpr int kBW = kThreads / 64 - 1;  // bulk waves
  // wave 0: the last winner's row (columns from two past its step), 16
  // bytes (two tagged words) per column, loaded after its exchange and
  // landed in LDS at the next step
  constexpr int kPF = 4;
  u32x4 brow_w[kPF];
#pragma unroll
  for (int t = 0; t < kPF; ++t) brow_w[t] = u32x4{0u, 0u, 0u, 0u};
  for (int j = 0; j < ncols; ++j) {
    const int sj = j & 1, sp = sj ^ 1;
    double* Uj = urow + sj * ncols;   // U(j, .); until overwritten it still holds U(j-2, .)
    double* Up = urow + sp * ncols;   // U(j-1, .)
    const bool upd1 = j >= 1 && sh_piv[sp] != 0.0;  // step j-1 updated the trailing part
    const bool upd2 = j >= 2 && sh_piv[sj] != 0.0;  // step j-2 did
    const unsigned tag = (unsigned)(j + 1);
    // records of step j live in buffer j mod 3 (see the header comment)
    const int bj = j % 3, bprev = (j + 2) % 3;
    const int64_t keyb = key_area_bytes(nwg), bufb = keyb + (int64_t)nwg * rec_stride;
    char* base = xch + (int64_t)bj * bufb;            // keys of step j
    char* recs = base + keyb;                         // records of step j
    const char* precs = xch + (int64_t)bprev * bufb + keyb;  // records of step j-1

    if (wave == 0) {
      // ---- (1) column j up to date, local candidate, publish -----------------
      double uj = 0.0;  // U(j-1, j)
      if (upd1) {
        uj = upd2 ? __fma_rn(-sh_lm[sp], Uj[j], sh_v1[sp]) : sh_v1[sp];
        if (lane == 0) Up[j] = uj;
      }
      // each lane's best row, with what its key carries
      double a = -1.0, bv = 0.0, blm = 0.0, bn = 0.0;
      int p = INT_MAX, r = -1;
      // (straight-line: loads for every lane, clamped to the stored rows,
      // selects instead of branches; the updated column j is stored in (4))
      const int jn = j + 1 < ncols ? j + 1 : j;
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int rr = lane + 64 * q, rq = min(rr, R - 1);
        const bool live = st_q[q] == kNone;
        const double x = Ts[(int64_t)j * R + rq];
        const double nx = Ts[(int64_t)jn * R + rq];
        const double v = upd1 ? __fma_rn(-mlt_q[q], uj, x) : x;
        val_q[q] = v;
        // NaN ranks above every number, so no step is ever left without a
        // candidate (and the NaN propagates)
        const double key = v != v ? __builtin_inf() : fabs(v);
        const bool take = live && better(key, pos_q[q], a, p);
        a = take ? key : a;
        p = take ? pos_q[q] : p;
        r = take ? rr : r;
        bv = take ? v : bv;
        blm = take ? mlt_q[q] : blm;
        bn = take ? nx : bn;
      }
      if (j + 1 >= ncols) bn = 0.0;
      {
        const int src = wave_best_lane(a, p);
        a = lane_bcast(a, src);
        p = __builtin_amdgcn_readlane(p, src);
        r = __builtin_amdgcn_readlane(r, src);
        bv = lane_bcast(bv, src);
        blm = lane_bcast(blm, src);
        bn = lane_bcast(bn, src);
      }
      // the candidate's multiplier of step j-1 and its values in columns j
      // and j+1 (the latter through step j-2: the bulk update of step j-1
      // comes after B1)
      const double lm = upd1 ? blm : 0.0;
      const double cpiv = r >= 0 ? bv : 0.0;
      const double cv1 = r >= 0 ? bn : 0.0;
      // (the candidate's row from column j+2 on is published by the bulk
      // waves after B1, before they update it)
      if (lane == 0) sh_cr = r;
      if (nwg > 1) {
        // the key: lanes 0-3 store its four word pairs in one instruction
        if (lane < 4) {
          const unsigned long long b = lane == 0 ? dbits(cpiv) : lane == 2 ? dbits(lm) : dbits(cv1);
          const unsigned p0 = lane == 1 ? (unsigned)p : (unsigned)b;
          const unsigned p1 = lane == 1 ? (unsigned)(r >= 0 ? row0 + r : -1) : (unsigned)(b >> 32);
          st_words2(rsrc_of(base, key_area_bytes(nwg)), kKeyWords * w + 2 * lane, tag, p0, p1);
        }
      } else {
        if (lane == 0) {
          sh_cp = p; sh_cpiv = cpiv; sh_clm = lm; sh_cv1 = cv1;
          if (r < 0) { st_agent_i(fail, 1); sh_stop = 1; }  // cannot happen for ncols <= nrows
        }
      }
      if (nwg > 1 && upd1) {
        // ---- (1b) the step j-1 winner's row, columns j+1 on, into LDS for
        // the bulk waves (loaded after that step's exchange; one poll per
        // column normally finds it there)
        const int bwp = __builtin_amdgcn_readfirstlane(sh_bw[sp]);
        const Rsrc pb = rsrc_of(precs + (int64_t)bwp * rec_stride, rec_stride);
        bool stop = false;
#pragma unroll
        for (int t = 0; t < kPF; ++t) {
          const int c = j + 1 + lane + 64 * t;
          if (c < ncols && !stop) {
            u32x4 v = brow_w[t];
            WaitLimit wl;
            while (!tagged2(v, (unsigned)j)) {
              if (wl.give_up(timeout_ticks, fail)) {
                stop = true;
                break;
              }
              v = ld_words2(pb, kHdrWords + 2 * c);
            }
            lbody[sp * ncols + c] = bitsd(payload2(v));
          }
        }
        // columns past the prefetched ones (panels wider than 64 kPF)
        for (int c = j + 1 + 64 * kPF + lane; c < ncols && !stop; c += 64) {
          u32x4 v = ld_words2(pb, kHdrWords + 2 * c);
          WaitLimit wl;
          while (!tagged2(v, (unsigned)j)) {
            if (wl.give_up(timeout_ticks, fail)) {
              stop = true;
              break;
            }
            v = ld_words2(pb, kHdrWords + 2 * c);
          }
          lbody[sp * ncols + c] = bitsd(payload2(v));
        }
        if (__any(stop)) {
          if (lane == 0) { st_agent_i(fail, 1); sh_stop = 1; }
        }
      }
    }
    lds_barrier();  // B1: candidate published (the bulk update may now touch its row)
    if (sh_stop) break;

    if (wave == 0) {
      // ---- (3) exchange: wait for every key, select the winner ------------------
      int win_row = -1, win_pos = INT_MAX, bw = -1;
      double piv = 0.0, wlm = 0.0, wv1 = 0.0;
      bool stop = false;
      if (nwg > 1) {
        // every lane polls the keys of workgroups lane, lane + 64, ...
        // (nwg <= 256) and folds each into its running best as it arrives
        // (candidates' positions differ, so the order of arrival does not
        // change the result)
        const int nq = __builtin_amdgcn_readfirstlane((nwg + 63) / 64);
        double ba = -1.0, bv = 0.0, blm = 0.0, bv1 = 0.0;
        int bp = INT_MAX, brow = -1;
        // done: slots read (or with nothing to read) by this lane
        unsigned done = 0xFu;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q < nq && lane + 64 * q < nwg) done &= ~(1u << q);
        WaitLimit wl;
        while (true) {
          // the loads of a poll are issued before any is examined, two
          // slots at a time (what the registers hold beside the rest): one
          // round trip per poll up to 128 workgroups
          constexpr int kCh = kThreads == 512 && RPL <= 4 ? 4 : 2;
          const Rsrc kr = rsrc_of(base, key_area_bytes(nwg));
#pragma unroll
          for (int c0 = 0; c0 < 4; c0 += kCh) {
            u32x4 x[kCh][kKeyWords / 2];
            bool poll[kCh];
#pragma unroll
            for (int i = 0; i < kCh; ++i) {
              const int q = c0 + i;
              poll[i] = q < nq && !__all((done >> q) & 1u);  // uniform
              if (poll[i]) {
                const int wq = min(lane + 64 * q, nwg - 1);
#pragma unroll
                for (int t = 0; t < kKeyWords / 2; ++t) x[i][t] = ld_words2(kr, kKeyWords * wq + 2 * t);
              }
            }
#pragma unroll
            for (int i = 0; i < kCh; ++i) {
              const int q = c0 + i;
              if (poll[i]) {
                bool ok = !((done >> q) & 1u);
#pragma unroll
                for (int t = 0; t < kKeyWords / 2; ++t) ok = ok && tagged2(x[i][t], tag);
                done |= ok ? 1u << q : 0u;
                // the magnitude the candidate was chosen by (NaN above every
                // number); a workgroup without a candidate ranks below all
                const double v = bitsd(payload2(x[i][0]));
                const int qp = (int)x[i][1].x, qrow = (int)x[i][1].z;
                const double qa = qrow < 0 ? -1.0 : (v != v ? __builtin_inf() : fabs(v));
                const bool take = ok && (bw < 0 || better(qa, qp, ba, bp));
                ba = take ? qa : ba;
                bp = take ? qp : bp;
                brow = take ? qrow : brow;
                bw = take ? lane + 64 * q : bw;
                bv = take ? v : bv;
                blm = take ? bitsd(payload2(x[i][2])) : blm;
                bv1 = take ? bitsd(payload2(x[i][3])) : bv1;
              }
            }
          }
          if (__all(done == 0xFu)) break;
          if (wl.give_up(timeout_ticks, fail)) {
            stop = true;
            break;
          }
        }
        if (!stop) {
          const int src = wave_best_lane(ba, bp);
          ba = lane_bcast(ba, src);
          bp = __builtin_amdgcn_readlane(bp, src);
          bw = __builtin_amdgcn_readlane(bw, src);
          brow = __builtin_amdgcn_readlane(brow, src);
          if (bw < 0 || ba < 0.0) {
            stop = true;  // no candidate anywhere: cannot happen for ncols <= nrows
          } else {
            win_row = brow;
            win_pos = bp;
            if (win_row < 0) stop = true;
            if (!stop) {
              piv = lane_bcast(bv, src);
              wlm = lane_bcast(blm, src);
              wv1 = lane_bcast(bv1, src);
              // start loading the winner's row (columns j+2 on): the bulk
              // waves need it at the next step
              const Rsrc wb = rsrc_of(recs + (int64_t)bw * rec_stride, rec_stride);
#pragma unroll
              for (int t = 0; t < kPF; ++t) {
                const int c = min(j + 2 + lane + 64 * t, ncols - 1);
                brow_w[t] = ld_words2(wb, kHdrWords + 2 * c);
              }
            }
          }
        }
      } else {
        win_row = row0 + sh_cr;
        win_pos = sh_cp;
        piv = sh_cpiv; wlm = sh_clm; wv1 = sh_cv1;
        bw = 0;
      }
      if (stop) {
        if (lane == 0) { st_agent_i(fail, 1); sh_stop = 1; }
      } else {
        // ---- (4) bookkeeping and multipliers of step j --------------------------
        const int wr = win_row - row0;  // local index if the winner is ours
        // multiply by the reciprocal pivot unless it would overflow.  piv is
        // the same in every lane: one uniform branch for the whole wave
        // instead of a masked branch per row
        const int how = __builtin_amdgcn_readfirstlane(
            piv == 0.0 ? 0 : (fabs(piv) >= 2.2250738585072014e-308 ? 1 : 2));  // smallest normal
        double mqs[RPL];
        if (how == 1) {
          const double rpiv = 1.0 / piv;
#pragma unroll
          for (int q = 0; q < RPL; ++q) mqs[q] = val_q[q] * rpiv;
        } else if (how == 2) {
#pragma unroll
          for (int q = 0; q < RPL; ++q) mqs[q] = val_q[q] / piv;
        } else {
#pragma unroll
          for (int q = 0; q < RPL; ++q) mqs[q] = 0.0;
        }
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
          const int r = lane + 64 * q;
          const bool live = st_q[q] == kNone, isw = r == wr;
          const double mq = live && !isw ? mqs[q] : 0.0;
          // column j: the winner keeps its pivot, the other live rows take
          // their multipliers (their values when the pivot is zero)
          if (live) Ts[(int64_t)j * R + r] = isw || piv == 0.0 ? val_q[q] : mq;
          // the winner takes position j, the row there moves to its place
          pos_q[q] = isw ? step0 + j : (pos_q[q] == step0 + j ? win_pos : pos_q[q]);
          st_q[q] = isw ? step0 + j : st_q[q];
          mlt_q[q] = mq;
        }
        if (lane == 0 && wr >= 0 && wr < R) step_s[wr] = step0 + j;
        if (lane == 0) {
          Uj[j] = piv;
          sh_piv[sj] = piv;
          sh_lm[sj] = wlm;
          sh_v1[sj] = wv1;
          sh_bw[sj] = bw;
          pivrow_s[j] = win_row;
          ipiv_s[j] = win_pos;
        }
        if (piv == 0.0 && info == 0) info = step0 + j + 1;
      }
    } else {
      // ---- (2b) bulk waves, first: publish this wave's columns c >= j+2 of
      // the workgroup's candidate row (through step j-2: before the update
      // of step j-1 below touches them)
      const int rc = sh_cr;
      if (rc >= 0) {
        constexpr int kBWp = kThreads / 64 - 1;
        const Rsrc body = rsrc_of(recs + (int64_t)w * rec_stride, rec_stride);
        for (int c = j + 1 + (wave - 1) + kBWp * lane; c < ncols; c += kBWp * 64) {
          if (c < j + 2) continue;
          const double v = Ts[(int64_t)c * R + rc];
          if (nwg > 1) {
            const unsigned long long b = dbits(v);
            st_words2(body, kHdrWords + 2 * c, tag, (unsigned)b, (unsigned)(b >> 32));
          } else {
            lbody[sj * ncols + c] = v;
          }
        }
      }
    }
    if (wave != 0 && upd1) {
      // ---- (2b) bulk waves: U(j-1, c) for this wave's columns, then the
      // rank-one update of step j-1 on them.  Wave w owns the columns
      // c = j + w + (waves - 1) t: it completes U(j-1, c) from the
      // winner's row, one update behind, with the same fused multiply-add
      // the winner's own workgroup applies, then updates those columns.
      {
        // the winner's row is in LDS (landed by wave 0 before B1, or
        // written by this workgroup itself when it is alone)
        const double lmw = sh_lm[sp];
        for (int c = j + 1 + (wave - 1) + kBW * lane; c < ncols; c += kBW * 64) {
          const double b = lbody[sp * ncols + c];
          Up[c] = upd2 ? __fma_rn(-lmw, Uj[c], b) : b;
        }
      }
      // this wave's U values are read back by all its lanes: keep the LDS
      // writes ahead of the reads
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      __builtin_amdgcn_s_waitcnt(0xC07F);
      __builtin_amdgcn_wave_barrier();
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      // Rows still active after step j-1 (step_s > j-1).  A row being chosen
      // at step j right now has step_s kNone or j: included either way, as it
      // must be (its U row is its values through step j-1).  Lanes past the
      // last stored row (lane + 64 q >= R) mirror row R-1: they load, compute
      // and store exactly what that row's own lane does, so that every load
      // and store is unconditional and inactive rows store back what they
      // read (only this wave writes its columns).
      int ro[RPL];
      double m[RPL];
      bool act[RPL];
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        ro[q] = min(lane + 64 * q, R - 1);
        act[q] = ro[q] < nr && step_s[ro[q]] > step0 + j - 1;
        m[q] = Ts[(int64_t)(j - 1) * R + ro[q]];
      }
      constexpr int kBulkWaves = kThreads / 64 - 1;
      // columns per iteration, all loads issued before any FMA (fewer for
      // eight rows per lane, which would spill)
      constexpr int kU = RPL >= 8 ? 2 : 4;
      int c = j + __builtin_amdgcn_readfirstlane(wave);  // uniform: j + 1 + (wave - 1)
      for (; c + (kU - 1) * kBulkWaves < ncols; c += kU * kBulkWaves) {
        double u[kU], x[kU][RPL];
#pragma unroll
        for (int t = 0; t < kU; ++t) {
          u[t] = Up[c + t * kBulkWaves];
#pragma unroll
          for (int q = 0; q < RPL; ++q) x[t][q] = Ts[(int64_t)(c + t * kBulkWaves) * R + ro[q]];
        }
#pragma unroll
        for (int t = 0; t < kU; ++t)
#pragma unroll
          for (int q = 0; q < RPL; ++q)
            Ts[(int64_t)(c + t * kBulkWaves) * R + ro[q]] =
                act[q] ? __fma_rn(-m[q], u[t], x[t][q]) : x[t][q];
      }
      for (; c < ncols; c += kBulkWaves) {
        const double u = Up[c];
        double x[RPL];
#pragma unroll
        for (int q = 0; q < RPL; ++q) x[q] = Ts[(int64_t)c * R + ro[q]];
#pragma unroll
        for (int q = 0; q < RPL; ++q)
          Ts[(int64_t)c * R + ro[q]] = act[q] ? __fma_rn(-m[q], u, x[q]) : x[q];
      }
    }
    lds_barrier();  // B0 of the next step
    if (sh_stop) break;
  }

  // ---- write back -------------------------------------------------------------
  if (wave == 0) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int r = lane + 64 * q;
      if (r < nr) {
        pos_s[r] = pos_q[q];
        step_s[r] = st_q[q];
      }
    }
    // the first zero pivot of the whole factorization: keep an earlier
    // block's report (the word starts at zero)
    if (lane == 0 && w == 0 && info != 0 && *info_out == 0) *info_out = info;
  }
  __syncthreads();
  if (rs == 1) {
    for (int idx = tid; idx < R * ncols; idx += kThreads) {
      const int r = idx % R, c = idx / R;
      if (r < nr) X[(int64_t)(row0 + r) + (int64_t)c * cs] = Ts[idx];
    }
  } else {
    for (int idx = tid; idx < R * ncols; idx += kThreads) {
      const int c = idx % ncols, r = idx / ncols;
      if (r < nr) X[(int64_t)(row0 + r) * rs + (int64_t)c * cs] = Ts[(int64_t)c * R + r];
    }
  }
  for (int r = tid; r < nr; r += kThreads) {
    pos_out[row0 + r] = pos_s[r];
    rstep_out[row0 + r] = step_s[r] == kNone ? total_cols : step_s[r];
  }
  if (w == 0)
    for (int c = tid; c < ncols; c += kThreads) {
      piv_row_out[c] = pivrow_s[c];
      ipiv_out[c] = ipiv_s[c];
    }
}

template <int RPL>
__global__ void __launch_bounds__(threads_for<RPL>())
panel_lu_kernel(double* __restrict__ X, int64_t rs, int64_t cs, int nrows, int ncols, int R,
                int nwg, int* __restrict__ pos_out, int* __restrict__ rstep_out,
                int* __restrict__ piv_row_out, int* __restrict__ ipiv_out,
                int* __restrict__ info_out, int* __restrict__ fail, char* __restrict__ xch,
                int64_t rec_stride, long long timeout_ticks, int step0, int total_cols,
                const int* __restrict__ pos_in, const int* __restrict__ rstep_in) {
  extern __shared__ double smem[];
  panel_body<RPL, threads_for<RPL>()>(X, rs, cs, nrows, ncols, R, nwg, pos_out, rstep_out,
                                      piv_row_out, ipiv_out,
                  info_out, fail, xch, rec_stride, timeout_ticks, (int)blockIdx.x, smem,
                  step0, total_cols, pos_in, rstep_in);
}

// Many panels in one persistent launch.  Workgroup b runs, round by round,
// the member of the panel named by sched[round * nslots + b] (task << 8 |
// member, or -1 when idle).  All members of a panel are scheduled in the
// same round, so a member waiting on its partners only waits for work of
// the same or earlier rounds, which always completes.
template <int RPL>
__global__ void __launch_bounds__(threads_for<RPL>())
panel_lu_batched_kernel(const PanelTaskDev* __restrict__ tasks, const int* __restrict__ sched,
                        int rounds, int nslots, long long timeout_ticks) {
  extern __shared__ double smem[];
  for (int r = 0; r < rounds; ++r) {
    const int e = sched[(int64_t)r * nslots + blockIdx.x];
    if (e < 0) continue;
    const PanelTaskDev t = tasks[e >> 8];
    panel_body<RPL, threads_for<RPL>()>(t.X, t.rs, t.cs, t.nrows, t.ncols, t.R, t.nwg,
                                                t.pos, t.rstep, t.piv_row, t.ipiv, t.info,
                                                t.fail, t.xch, t.rec_stride, timeout_ticks,
                                                e & 255, smem, 0, t.ncols, nullptr, nullptr);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Panels of one workgroup with at most 32 columns: the rows live in
// registers (thread t holds rows t, t + 512, ...), a row's registers holding
// its columns from the current step on (they shift by one after each step,
// so that column j is always the first register and no step selects among
// registers by a run-time index), and one barrier per step suffices.
// Step j:
//   before the barrier: each thread applies the rank-one update of step j-1
//     to its live rows (the step j-1 pivot row read from LDS) and finds its
//     best row in column j; the wave's best lane posts that candidate (rank
//     key, value, the value's reciprocal, position, row) and its row in the
//     wave's slot of the step's parity;
//   after it: every wave reads the eight slots and selects the same winner;
//     each thread stores column j of its live rows (the multipliers, or
//     the values themselves for the winner and for a zero pivot), the
//     first threads store the winner's U row from its slot, and the position
//     bookkeeping follows; every finished entry goes to memory as it is
//     produced, so nothing is left to write back at the end.
// The slots of step j are written again at step j + 2, after the barrier of
// step j + 1, which a thread reaches only after its update of step j has
// read the winner's row.  The arithmetic is the multi-workgroup kernel's:
// the same multipliers, the same fused multiply-add for each update, the
// same ranking and tie break, so the factors agree bitwise.
// ---------------------------------------------------------------------------
constexpr int kSmallThreads = 512;
constexpr int kSmallWaves = kSmallThreads / 64;

template <int CMAX, int RPT>
__global__ void __launch_bounds__(kSmallThreads)
panel_small_kernel(double* __restrict__ X, int64_t rs, int64_t cs, int nrows, int ncols,
                   int* __restrict__ pos_out, int* __restrict__ rstep_out,
                   int* __restrict__ piv_row_out, int* __restrict__ ipiv_out,
                   int* __restrict__ info_out, int* __restrict__ fail, int step0, int total_cols,
                   const int* __restrict__ pos_in, const int* __restrict__ rstep_in) {
  // a wave's slot: its candidate's rank key, value in column j, the
  // reciprocal of that value (taken here, off the path that follows the
  // barrier), position and row (packed); then the candidate's row from
  // column j+1 on, aligned with the registers of the next step
  __shared__ double s_hdr[2][kSmallWaves][4];
  __shared__ double s_row[2][kSmallWaves][CMAX];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  double x[RPT][CMAX];  // x[q][c]: column j + c of row tid + 512 q at step j
  double mlt[RPT];
  int pos[RPT], st[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = tid + kSmallThreads * q;
    const bool in = r < nrows;
    const double* xr = X + (int64_t)(in ? r : 0) * rs;
#pragma unroll
    for (int c = 0; c < CMAX; ++c) {
      x[q][c] = in && c < ncols ? *xr : 0.0;
      xr += cs;
    }
    pos[q] = in ? (pos_in ? pos_in[r] : r) : INT_MAX;
    st[q] = -1;  // no such row
    if (in) {
      st[q] = kNone;
      if (rstep_in) {
        const int s0 = rstep_in[r];
        if (s0 < step0) st[q] = s0;  // chosen by an earlier block of columns
      }
    }
    mlt[q] = 0.0;
  }

  int info = 0;
  bool upd = false;  // the previous step had a nonzero pivot
  int wprev = 0;     // slot holding the previous step's pivot row
  int j = 0;
  for (; j < ncols; ++j) {
    const int sj = j & 1, sp = sj ^ 1;
    // ---- (A) update of step j-1 on the live rows ----------------------------
    if (upd) {
      double u[CMAX];
#pragma unroll
      for (int c = 0; c < CMAX; ++c) u[c] = s_row[sp][wprev][c];
#pragma unroll
      for (int q = 0; q < RPT; ++q)
        if (st[q] == kNone) {
#pragma unroll
          for (int c = 0; c < CMAX; ++c) x[q][c] = __fma_rn(-mlt[q], u[c], x[q][c]);
        }
    }
    // ---- (B) the thread's and the wave's best live row in column j ---------
    double a = -1.0, bv = 0.0;
    int p = INT_MAX, bq = -1;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const double v = x[q][0];
      // NaN ranks above every number (see panel_body)
      const double key = v != v ? __builtin_inf() : fabs(v);
      const bool take = st[q] == kNone && better(key, pos[q], a, p);
      a = take ? key : a;
      p = take ? pos[q] : p;
      bq = take ? q : bq;
      bv = take ? v : bv;
    }
    const int src = wave_best_lane(a, p);
    if (lane == src) {
      const int r = bq < 0 ? -1 : tid + kSmallThreads * bq;
      s_hdr[sj][wave][0] = a;
      s_hdr[sj][wave][1] = bv;
      s_hdr[sj][wave][2] = 1.0 / bv;
      s_hdr[sj][wave][3] = __hiloint2double(r, p);
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        if (q != bq) continue;
#pragma unroll
        for (int c = 0; c < CMAX; ++c) s_row[sj][wave][c] = c + 1 < CMAX ? x[q][c + 1] : 0.0;
      }
    }
    lds_barrier();
    // ---- (C) the winner: lane w holds slot w; every wave selects alike ------
    double hk = -2.0, hv = 0.0, hi = 0.0;
    int hp = INT_MAX, hr = -1;
    if (lane < kSmallWaves) {
      hk = s_hdr[sj][lane][0];
      hv = s_hdr[sj][lane][1];
      hi = s_hdr[sj][lane][2];
      const double pk = s_hdr[sj][lane][3];
      hp = __double2loint(pk);
      hr = __double2hiint(pk);
    }
    const int ws = wave_best_lane(hk, hp);
    const int win_r = __builtin_amdgcn_readlane(hr, ws);
    if (win_r < 0) {  // no live row anywhere: cannot happen for ncols <= nrows
      if (tid == 0) st_agent_i(fail, 1);
      break;
    }
    const int win_pos = __builtin_amdgcn_readlane(hp, ws);
    const double piv = lane_bcast(hv, ws);
    // ---- (D) multipliers, stores and bookkeeping of step j -------------------
    const int how = __builtin_amdgcn_readfirstlane(
        piv == 0.0 ? 0 : (fabs(piv) >= 2.2250738585072014e-308 ? 1 : 2));  // smallest normal
    double mq[RPT];
    if (how == 1) {
      const double rpiv = lane_bcast(hi, ws);  // 1 / piv
#pragma unroll
      for (int q = 0; q < RPT; ++q) mq[q] = x[q][0] * rpiv;
    } else if (how == 2) {
#pragma unroll
      for (int q = 0; q < RPT; ++q) mq[q] = x[q][0] / piv;
    } else {
#pragma unroll
      for (int q = 0; q < RPT; ++q) mq[q] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + kSmallThreads * q;
      const bool live = st[q] == kNone, isw = r == win_r;
      if (live) X[(int64_t)r * rs + (int64_t)j * cs] = isw || piv == 0.0 ? x[q][0] : mq[q];
      mlt[q] = live && !isw ? mq[q] : 0.0;
      pos[q] = isw ? step0 + j : (pos[q] == step0 + j ? win_pos : pos[q]);
      st[q] = isw ? step0 + j : st[q];
    }
    // the winner's U row, columns j+1 .. ncols-1, from its slot
    if (tid < ncols - 1 - j)
      X[(int64_t)win_r * rs + (int64_t)(j + 1 + tid) * cs] = s_row[sj][ws][tid];
    // the registers move on to column j+1
#pragma unroll
    for (int q = 0; q < RPT; ++q)
#pragma unroll
      for (int c = 0; c < CMAX; ++c) x[q][c] = c + 1 < CMAX ? x[q][c + 1] : 0.0;
    if (tid == 0) {
      piv_row_out[j] = win_r;
      ipiv_out[j] = win_pos;
    }
    if (piv == 0.0 && info == 0) info = step0 + j + 1;
    upd = piv != 0.0;
    wprev = ws;
  }
  // a factorization that stopped early still hands its consumers in-range
  // rows and positions (see panel_body)
  if (tid == 0)
    for (int c = j; c < ncols; ++c) {
      piv_row_out[c] = c;
      ipiv_out[c] = step0 + c;
    }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = tid + kSmallThreads * q;
    if (r < nrows) {
      pos_out[r] = pos[q];
      rstep_out[r] = st[q] == kNone ? total_cols : st[q];
    }
  }
  if (tid == 0 && info != 0 && *info_out == 0) *info_out = info;
}

// The register-resident kernel for a panel of one workgroup, if one fits:
// CMAX the smaller of 16 and 32 that holds the columns, RPT rows per thread
// with RPT CMAX <= 64 (128 registers of panel per thread; 64 columns in one
// row per thread would leave too few registers for the rest).
int small_cmax(int ncols) { return ncols <= 16 ? 16 : ncols <= 32 ? 32 : 0; }
int small_rows_cap(int ncols) {
  const int cm = small_cmax(ncols);
  return cm ? kSmallThreads * (64 / cm) : 0;
}
bool panel_regs_enabled() {
  const char* e = std::getenv("RLU_PANEL_REGS");
  return !(e && e[0] == '0');
}
const void* small_fn(int nrows, int ncols) {
  const int cm = small_cmax(ncols);
  const int rpt = (nrows + kSmallThreads - 1) / kSmallThreads;
  if (cm == 16) {
    return rpt <= 1 ? (const void*)panel_small_kernel<16, 1>
         : rpt <= 2 ? (const void*)panel_small_kernel<16, 2>
         : rpt <= 4 ? (const void*)panel_small_kernel<16, 4> : nullptr;
  }
  if (cm == 32)
    return rpt <= 1 ? (const void*)panel_small_kernel<32, 1>
         : rpt <= 2 ? (const void*)panel_small_kernel<32, 2> : nullptr;
  return nullptr;
}

constexpr size_t kLdsLimit = 160 * 1024;

size_t lds_for(int R, int ncols) {
  return (size_t)R * ncols * 8 + (size_t)4 * ncols * 8 + (size_t)R * 8 + (size_t)ncols * 8;
}

int64_t rec_stride_for(int ncols) {
  return (8 * (int64_t)kHdrWords + 16 * (int64_t)ncols + 127) / 128 * 128;
}

}  // namespace

// Workgroups a panel aims at (rows per workgroup permitting): 128, or the
// tuning override RLU_PANEL_WG_CAP (16 .. 256) read once per process.
int panel_wg_cap() {
  static const int cap = [] {
    const char* e = std::getenv("RLU_PANEL_WG_CAP");
    const int v = e ? std::atoi(e) : 0;
    return v >= 16 && v <= 256 ? v : 128;
  }();
  return cap;
}

PanelPlan panel_plan(int nrows, int ncols, int device_cus, int /*max_wg_per_cu_hint*/) {
  PanelPlan p{};
  p.ok = false;
  if (nrows <= 0 || ncols <= 0 || ncols > nrows) return p;
  // the LDS holds R rows of the panel (leaving room for static shared data)
  const size_t budget = kLdsLimit - 1024;
  auto fits = [&](int rows) { return lds_for(rows, ncols) <= budget; };
  p.regs = false;
  int R, nwg;
  if (nrows <= small_rows_cap(ncols) && panel_regs_enabled()) {
    // one workgroup, the panel in registers (panel_small_kernel)
    p.rows_per_wg = nrows;
    p.nwg = 1;
    p.lds_bytes = 0;
    p.xch_bytes = 0;
    p.ok = true;
    p.regs = true;
    return p;
  }
  if (nrows <= 512 && fits(nrows)) {
    // one workgroup: the exchange stays in LDS
    R = nrows;
    nwg = 1;
  } else {
    // a multiple of 64 rows per workgroup (every lane holds real rows) and
    // at most 128 workgroups while 512 rows allow it: each step every
    // workgroup reads every key, so fewer workgroups make a cheaper
    // exchange, and a lane then watches at most two of them
    const int per = (nrows + panel_wg_cap() - 1) / panel_wg_cap();
    R = std::min(512, (per + 63) / 64 * 64);
    if (!fits(R)) return p;  // narrower column blocks
    nwg = (nrows + R - 1) / R;
  }
  // one workgroup per CU is what the LDS footprint guarantees; four records
  // per lane bound the exchange width
  if (nwg > device_cus || nwg > 256) return p;
  p.rows_per_wg = R;
  p.nwg = nwg;
  p.lds_bytes = lds_for(R, ncols);
  p.xch_bytes = panel_xch_bytes(nwg, ncols);
  p.ok = true;
  return p;
}

hipError_t launch_panel_lu(const PanelDesc& d, const PanelPlan& plan, hipStream_t s) {
  if (!plan.ok) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  if (plan.regs) {
    const void* fn = small_fn(d.nrows, d.ncols);
    if (!fn) return hipErrorInvalidValue;
    double* X = (double*)d.X;
    int64_t rs = d.rs, cs = d.cs;
    int nrows = d.nrows, ncols = d.ncols;
    int* pos = d.pos; int* rstep = d.rstep; int* piv_row = d.piv_row; int* ipiv = d.ipiv;
    int* info = d.info; int* fail = d.fail;
    int step0 = d.step0, total = d.total_cols > 0 ? d.total_cols : d.ncols;
    const int* pos_in = d.pos_in;
    const int* rstep_in = d.rstep_in;
    void* args[] = {&X, &rs, &cs, &nrows, &ncols, &pos, &rstep, &piv_row, &ipiv,
                    &info, &fail, &step0, &total, &pos_in, &rstep_in};
    return hipLaunchKernel(fn, dim3(1), dim3(kSmallThreads), args, 0, s);
  }
  // clear the exchange tags of both parities
  if (plan.nwg > 1) {
    e = launch_fill_u32((uint32_t*)d.xch, plan.xch_bytes / 4, 0u, s);
    if (e != hipSuccess) return e;
  }
  double* X = (double*)d.X;
  int64_t rs = d.rs, cs = d.cs;
  int nrows = d.nrows, ncols = d.ncols, R = plan.rows_per_wg, nwg = plan.nwg;
  int* pos = d.pos; int* rstep = d.rstep; int* piv_row = d.piv_row; int* ipiv = d.ipiv;
  int* info = d.info; int* fail = d.fail; char* xch = (char*)d.xch;
  long long tmo = d.timeout_ticks;
  int64_t rec_stride = rec_stride_for(d.ncols);
  int step0 = d.step0, total = d.total_cols > 0 ? d.total_cols : d.ncols;
  const int* pos_in = d.pos_in;
  const int* rstep_in = d.rstep_in;
  void* args[] = {&X, &rs, &cs, &nrows, &ncols, &R, &nwg, &pos, &rstep, &piv_row, &ipiv,
                  &info, &fail, &xch, &rec_stride, &tmo, &step0, &total, &pos_in, &rstep_in};
  const void* fn = R <= 64 ? (const void*)panel_lu_kernel<1>
                 : R <= 128 ? (const void*)panel_lu_kernel<2>
                 : R <= 256 ? (const void*)panel_lu_kernel<4>
                            : (const void*)panel_lu_kernel<8>;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)plan.lds_bytes);
  if (e != hipSuccess) return e;
  // The pivot exchange needs every workgroup resident at once.  An ordinary
  // launch gives that here: the grid is at most one workgroup per CU (the
  // plan's bound, and the LDS footprint allows no more per CU), the stream
  // runs it alone after the work before it, and every wait is bounded, so
  // a workgroup that starts late (work of other streams holding CUs) only
  // delays its partners, and one that cannot start ends the factorization
  // with the exchange-failure status rather than a hang.
  return hipLaunchKernel(fn, dim3(nwg), dim3(threads_for_rows(R)), args, (unsigned)plan.lds_bytes,
                         s);
}

int64_t panel_rec_stride(int ncols) { return rec_stride_for(ncols); }

size_t panel_xch_bytes(int nwg, int ncols) {
  return (size_t)(3 * (key_area_bytes(nwg) + (int64_t)nwg * rec_stride_for(ncols)));
}

size_t panel_lds_bytes(int R, int ncols) { return lds_for(R, ncols); }

namespace {
const void* batched_fn(int max_R) {
  return max_R <= 64 ? (const void*)panel_lu_batched_kernel<1>
       : max_R <= 128 ? (const void*)panel_lu_batched_kernel<2>
       : max_R <= 256 ? (const void*)panel_lu_batched_kernel<4>
                      : (const void*)panel_lu_batched_kernel<8>;
}
}  // namespace

int panel_batched_slots(int max_R, size_t lds_bytes, int cus) {
  const void* fn = batched_fn(max_R);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes) !=
      hipSuccess)
    return 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads_for_rows(max_R),
                                                   lds_bytes) !=
      hipSuccess)
    return 0;
  return per_cu * cus;
}

// An ordinary launch (so that it can be captured in a graph): the grid never
// exceeds what the device holds at once (panel_batched_slots), and every
// wait is bounded, so workgroups that start late only delay their partners.
hipError_t launch_panel_lu_batched(const PanelTaskDev* tasks, const int* sched, int rounds,
                                   int nslots, int max_R, size_t lds_bytes,
                                   long long timeout_ticks, hipStream_t s) {
  if (rounds <= 0 || nslots <= 0) return hipSuccess;
  const void* fn = batched_fn(max_R);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds_bytes);
  if (e != hipSuccess) return e;
  void* args[] = {&tasks, &sched, &rounds, &nslots, &timeout_ticks};
  return hipLaunchKernel(fn, dim3(nslots), dim3(threads_for_rows(max_R)), args, lds_bytes,
                         s);
}

// ---------------------------------------------------------------------------
// Between two column blocks of a blocked factorization (rows never move):
// the U rows of the block's pivots for the columns to its right,
//   L11 U12 = X(pr, c1:),   L11(j, i) = X(pr_j, c0 + i) for i < j (unit lower),
// with pr_j = piv_row[j] the row chosen at step c0 + j.  Workgroup b solves
// 16 right-hand-side columns with U12 in LDS, 16 rows at a time: the 16 rows
// of L11 the step needs are first gathered into LDS by all threads, beside
// their right-hand sides (the solve's dependency chain then only touches
// LDS and registers), then the product with the rows already solved by all
// 256 threads (four multiply-add chains per output), then the 16 x 16
// triangle by one wave, in registers.  Output U (w x nrhs, leading
// dimension w).
// ---------------------------------------------------------------------------
constexpr int kTrsmMaxW = 288;
// Right-hand-side columns per workgroup: 16 (one per thread of a row) gives
// twice the workgroups of 32 on the narrow solves between column blocks
// and halves each one's product with the rows already solved (its LDS
// reads dominate a chunk once many rows are solved).
constexpr int kTrsmCols = 16;
constexpr int kTrsmQ = kTrsmCols / 16;  // columns per thread

__global__ void __launch_bounds__(256) block_trsm_kernel(const double* __restrict__ X, int64_t ldx,
                                                         const int* __restrict__ piv_row, int c0,
                                                         int w, int64_t c1, int nrhs,
                                                         double* __restrict__ U) {
  extern __shared__ double sm[];
  double* Us = sm;                     // w x kTrsmCols, row-major
  double* Ls = sm + w * kTrsmCols;     // 16 x w: rows J0 .. J0+15 of L11, row-major
  __shared__ int prow_s[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cc0 = kTrsmCols * blockIdx.x;
  const int jj = tid >> 4, cg = tid & 15;  // a row of the block, columns cg + 16 q
  for (int J0 = 0; J0 < w; J0 += 16) {
    const int h = min(16, w - J0), len = J0 + h;
    if (tid < h) prow_s[tid] = piv_row[J0 + tid];
    __syncthreads();
    // this chunk's right-hand sides, loaded beside the L11 rows
    double acc[kTrsmQ];
#pragma unroll
    for (int q = 0; q < kTrsmQ; ++q) acc[q] = 0.0;
    if (jj < h) {
      const int64_t prow = prow_s[jj];
#pragma unroll
      for (int q = 0; q < kTrsmQ; ++q) {
        const int c = cc0 + cg + 16 * q;
        acc[q] = c < nrhs ? X[prow + (c1 + c) * ldx] : 0.0;
      }
    }
    for (int e = tid; e < h * len; e += 256) {
      const int r = e / len, i = e % len;
      Ls[r * w + i] = X[(int64_t)prow_s[r] + (int64_t)(c0 + i) * ldx];
    }
    __syncthreads();
    if (jj < h) {
      // the rows already solved (J0 is a multiple of 16): four partial sums
      // per output over i mod 4, so that four multiply-add chains run side by
      // side, added in a fixed order
      const double* lr = Ls + jj * w;
      double part[4][kTrsmQ];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < kTrsmQ; ++q) part[t][q] = 0.0;
      for (int i = 0; i < J0; i += 4) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const double l = lr[i + t];
#pragma unroll
          for (int q = 0; q < kTrsmQ; ++q)
            part[t][q] = __fma_rn(-l, Us[(i + t) * kTrsmCols + cg + 16 * q], part[t][q]);
        }
      }
#pragma unroll
      for (int q = 0; q < kTrsmQ; ++q)
        Us[(J0 + jj) * kTrsmCols + cg + 16 * q] =
            acc[q] + ((part[0][q] + part[1][q]) + (part[2][q] + part[3][q]));
    }
    __syncthreads();
    if (wave == 0 && lane < kTrsmCols) {
      // the 16 x 16 triangle in registers, a lane per column: once u_i is
      // final it updates every later row, so each u_r still takes its
      // terms in increasing i (the order of the dot-product form) while
      // the updates of one i run side by side
      // (straight-line, so that every LDS read is issued up front: rows
      // past the last, h <= r < 16, repeat row h-1 and are never stored;
      // they feed only rows after themselves)
      const int hm = h - 1;
      double u[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) u[r] = Us[(J0 + min(r, hm)) * kTrsmCols + lane];
#pragma unroll
      for (int i = 0; i < 15; ++i)
#pragma unroll
        for (int r = i + 1; r < 16; ++r)
          u[r] = __fma_rn(-Ls[min(r, hm) * w + J0 + min(i, hm)], u[i], u[r]);
#pragma unroll
      for (int r = 1; r < 16; ++r)
        if (r < h) Us[(J0 + r) * kTrsmCols + lane] = u[r];
    }
    __syncthreads();
  }
  for (int e = tid; e < w * kTrsmCols; e += 256) {
    const int j = e / kTrsmCols, c = e % kTrsmCols;
    if (cc0 + c < nrhs) U[j + (int64_t)(cc0 + c) * w] = Us[j * kTrsmCols + c];
  }
}

hipError_t launch_block_trsm(const double* X, int64_t ldx, const int* piv_row, int c0, int w,
                             int64_t c1, int nrhs, double* U, hipStream_t s) {
  if (w <= 0 || nrhs <= 0) return hipSuccess;
  if (w > kTrsmMaxW) return hipErrorInvalidValue;
  const size_t lds = (size_t)w * (kTrsmCols + 16) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)block_trsm_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(block_trsm_kernel, dim3((unsigned)((nrhs + kTrsmCols - 1) / kTrsmCols)),
                     dim3(256), lds, s, X, ldx, piv_row, c0, w, c1, nrhs, U);
  return hipGetLastError();
}

int panel_block_max_width() { return kTrsmMaxW; }

}  // namespace rlu
