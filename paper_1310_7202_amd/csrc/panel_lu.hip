// LU with partial pivoting of a tall matrix X (nrows x ncols, ncols <= nrows),
// all ncols columns factored, as used twice by Algorithm 4.1 (Shabat et al.,
// Section 4):
//   Step 3  P Y = L_y U_y                 X = Y   (m x l)
//   Step 6  B Q = L_b U_b  via  Q^T B^T = L' U'   X = B^T (n x k), whose rows
//           are the columns of B: row pivoting of B^T is column pivoting of
//           B and produces the same pivot sequence.
// The Remark after Algorithm 4.1 allows partial pivoting in Step 3.
//
// Design (one persistent cooperative launch, no host round trip):
//   * workgroup w keeps rows [w R, (w+1) R) of X resident in LDS for the whole
//     factorization; rows never move ("virtual" pivoting): each row records
//     its current position (to reproduce LAPACK's swap bookkeeping and its
//     lowest-position tie break) and the step that chose it.
//   * step j: every workgroup finds its best candidate in column j (largest
//     magnitude, lowest current position on ties) and publishes it, with the
//     candidate's current row from column j on, in an exchange record; every
//     workgroup then reads all records, selects the same winner and applies
//     the rank-one update to its own rows.  One exchange per step, no grid
//     barrier; records alternate between two buffers by step parity, which
//     is enough because a workgroup cannot publish step j+2 before every
//     workgroup has finished reading step j.
//   * every wait is bounded by a wall-clock limit; on expiry the kernel sets
//     a failure flag and all workgroups leave.
#include "rlu_device.h"
#include "rlu_kernels.h"

#include <climits>

namespace rlu {
namespace {

constexpr int kThreads = 256;
constexpr int kNone = INT_MAX;

struct RecHeader {
  unsigned long long tag;  // step + 1 once the record is complete
  double absval;           // candidate magnitude, -1 if the workgroup has none
  int pos;                 // candidate's current position
  int row;                 // candidate's original row index
  int pad[2];
};

__device__ __forceinline__ void pick(double& a, int& p, int& r, double a2, int p2, int r2) {
  if (a2 > a || (a2 == a && p2 < p)) { a = a2; p = p2; r = r2; }
}

__device__ __forceinline__ void wave_pick(double& a, int& p, int& r) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double a2 = __shfl_xor(a, off, 64);
    const int p2 = __shfl_xor(p, off, 64);
    const int r2 = __shfl_xor(r, off, 64);
    pick(a, p, r, a2, p2, r2);
  }
}

__global__ void __launch_bounds__(kThreads)
panel_lu_kernel(double* __restrict__ X, int64_t rs, int64_t cs, int nrows, int ncols, int R,
                int nwg, int* __restrict__ pos_out, int* __restrict__ rstep_out,
                int* __restrict__ piv_row_out, int* __restrict__ ipiv_out,
                int* __restrict__ info_out, int* __restrict__ fail, char* __restrict__ xch,
                int64_t rec_stride, long long timeout_ticks) {
  extern __shared__ double smem[];
  double* Ts = smem;                      // R x ncols, column-major (ld R)
  double* urow = Ts + (int64_t)R * ncols; // ncols
  double* mult = urow + ncols;            // R
  int* pos_s = (int*)(mult + R);          // R
  int* step_s = pos_s + R;                // R
  __shared__ int sh_win_wg, sh_win_row, sh_win_pos, sh_stop, sh_info;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int w = blockIdx.x;
  const int row0 = w * R;
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
  for (int r = tid; r < R; r += kThreads) {
    pos_s[r] = row0 + r;
    step_s[r] = r < nr ? kNone : -1;  // -1: padding, never active
  }
  if (tid == 0) { sh_stop = 0; sh_info = 0; }
  __syncthreads();

  const long long t_start = now_ticks();

  for (int j = 0; j < ncols; ++j) {
    // ---- (a) local candidate and (b) exchange: wave 0 ------------------------
    if (wave == 0) {
      double a = -1.0; int p = INT_MAX, r = -1;
      for (int rr = lane; rr < nr; rr += 64) {
        if (step_s[rr] == kNone) {
          // a NaN entry ranks above every number so that it is always chosen
          // (and propagates) instead of leaving a step without a candidate
          const double v = Ts[(int64_t)j * R + rr];
          pick(a, p, r, v != v ? __builtin_inf() : fabs(v), pos_s[rr], rr);
        }
      }
      wave_pick(a, p, r);   // every lane now holds the local winner
      if (nwg == 1) {
        if (r < 0) {  // cannot happen for ncols <= nrows; leave rather than index with -1
          if (lane == 0) { st_agent_i(fail, 1); sh_stop = 1; }
        } else {
        if (lane == 0) {
          sh_win_wg = 0;
          sh_win_row = row0 + r;
          sh_win_pos = p;
        }
        for (int c = j + lane; c < ncols; c += 64) urow[c] = Ts[(int64_t)c * R + r];
        }
      } else {
        char* base = xch + (int64_t)(j & 1) * nwg * rec_stride;
        {
          char* rec = base + (int64_t)w * rec_stride;
          double* rrow = (double*)(rec + sizeof(RecHeader));
          for (int c = j + lane; c < ncols; c += 64) rrow[c] = r >= 0 ? Ts[(int64_t)c * R + r] : 0.0;
          if (lane == 0) {
            RecHeader* h = (RecHeader*)rec;
            h->absval = a;
            h->pos = p;
            h->row = r >= 0 ? row0 + r : -1;
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          if (lane == 0) st_agent(&((RecHeader*)rec)->tag, (unsigned long long)(j + 1));
        }
        // wait for every record of this step
        const int nq = (nwg + 63) / 64;
        unsigned seen = 0, need = 0;
        for (int q = 0; q < nq; ++q)
          if (lane + 64 * q < nwg) need |= 1u << q;
        bool stop = false;
        while (true) {
          for (int q = 0; q < nq; ++q) {
            if ((need >> q & 1u) && !(seen >> q & 1u)) {
              const RecHeader* h = (const RecHeader*)(base + (int64_t)(lane + 64 * q) * rec_stride);
              if (ld_agent(&h->tag) == (unsigned long long)(j + 1)) seen |= 1u << q;
            }
          }
          const bool mine_done = seen == need;
          if (__all(mine_done)) break;
          if (now_ticks() - t_start > timeout_ticks || ld_agent_i(fail) != 0) {
            stop = true;
            break;
          }
        }
        if (stop) {
          if (lane == 0) { st_agent_i(fail, 1); sh_stop = 1; }
        } else {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          double ba = -1.0; int bp = INT_MAX, br = -1, bw = -1;
          for (int q = 0; q < nq; ++q) {
            const int i = lane + 64 * q;
            if (i < nwg) {
              const RecHeader* h = (const RecHeader*)(base + (int64_t)i * rec_stride);
              const double a2 = h->absval;
              const int p2 = h->pos, r2 = h->row;
              if (a2 > ba || (a2 == ba && p2 < bp)) { ba = a2; bp = p2; br = r2; bw = i; }
            }
          }
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) {
            const double a2 = __shfl_xor(ba, off, 64);
            const int p2 = __shfl_xor(bp, off, 64);
            const int r2 = __shfl_xor(br, off, 64);
            const int w2 = __shfl_xor(bw, off, 64);
            if (a2 > ba || (a2 == ba && p2 < bp)) { ba = a2; bp = p2; br = r2; bw = w2; }
          }
          if (bw < 0 || br < 0) {  // no candidate anywhere: cannot happen for ncols <= nrows
            if (lane == 0) { st_agent_i(fail, 1); sh_stop = 1; }
          } else {
            if (lane == 0) { sh_win_wg = bw; sh_win_row = br; sh_win_pos = bp; }
            const double* wrow =
                (const double*)(base + (int64_t)bw * rec_stride + sizeof(RecHeader));
            for (int c = j + lane; c < ncols; c += 64) urow[c] = wrow[c];
          }
        }
      }
    }
    __syncthreads();
    if (sh_stop) break;

    // ---- (c) positions, pivot bookkeeping, multipliers ------------------------
    const int win_row = sh_win_row, win_pos = sh_win_pos;
    const double piv = urow[j];
    const int wr = win_row - row0;  // local index if the winner is ours
    for (int r = tid; r < nr; r += kThreads) {
      const bool is_win = (r == wr);
      if (is_win) {
        pos_s[r] = j;
        step_s[r] = j;
      } else if (pos_s[r] == j) {
        pos_s[r] = win_pos;  // the row at position j moves to the winner's position
      }
      double mlt = 0.0;
      if (step_s[r] == kNone && piv != 0.0) {
        mlt = Ts[(int64_t)j * R + r] / piv;
        Ts[(int64_t)j * R + r] = mlt;
      }
      mult[r] = mlt;
    }
    if (w == 0 && tid == 0) {
      piv_row_out[j] = win_row;
      ipiv_out[j] = win_pos;
      if (piv == 0.0 && sh_info == 0) sh_info = j + 1;
    }
    __syncthreads();

    // ---- (d) rank-one update of the trailing columns ---------------------------
    const int width = ncols - j - 1;
    if (piv != 0.0 && width > 0) {
      const int total = nr * width;
      for (int idx = tid; idx < total; idx += kThreads) {
        const int r = idx % nr, c = j + 1 + idx / nr;
        if (step_s[r] == kNone) Ts[(int64_t)c * R + r] -= mult[r] * urow[c];
      }
    }
    __syncthreads();
  }

  // ---- write back -------------------------------------------------------------
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
    rstep_out[row0 + r] = step_s[r] == kNone ? ncols : step_s[r];
  }
  if (w == 0 && tid == 0) *info_out = sh_info;
}

constexpr size_t kLdsLimit = 160 * 1024;

size_t lds_for(int R, int ncols) {
  return (size_t)R * ncols * 8 + (size_t)ncols * 8 + (size_t)R * 8 + (size_t)R * 8;
}

}  // namespace

PanelPlan panel_plan(int nrows, int ncols, int device_cus, int /*max_wg_per_cu_hint*/) {
  PanelPlan p{};
  p.ok = false;
  if (nrows <= 0 || ncols <= 0 || ncols > nrows) return p;
  // largest row block that fits the LDS (leaving room for static shared data)
  const size_t budget = kLdsLimit - 1024;
  int R = (int)((budget - (size_t)ncols * 8) / ((size_t)ncols * 8 + 16));
  if (R > 4096) R = 4096;
  if (R < 1) return p;
  int nwg = (nrows + R - 1) / R;
  // spread the rows evenly over that many workgroups
  R = (nrows + nwg - 1) / nwg;
  nwg = (nrows + R - 1) / R;
  // one workgroup per CU is what the LDS footprint guarantees; 32 slots per
  // lane bound the exchange width
  if (nwg > device_cus || nwg > 64 * 32) return p;
  p.rows_per_wg = R;
  p.nwg = nwg;
  p.lds_bytes = lds_for(R, ncols);
  const int64_t stride = ((int64_t)sizeof(RecHeader) + 8 * (int64_t)ncols + 127) / 128 * 128;
  p.xch_bytes = (size_t)(2 * (int64_t)nwg * stride);
  p.ok = true;
  return p;
}

hipError_t launch_panel_lu(const PanelDesc& d, const PanelPlan& plan, hipStream_t s) {
  if (!plan.ok) return hipErrorInvalidValue;
  const int64_t stride = ((int64_t)sizeof(RecHeader) + 8 * (int64_t)d.ncols + 127) / 128 * 128;
  hipError_t e = hipFuncSetAttribute((const void*)panel_lu_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)plan.lds_bytes);
  if (e != hipSuccess) return e;
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
  int64_t rec_stride = stride;
  void* args[] = {&X, &rs, &cs, &nrows, &ncols, &R, &nwg, &pos, &rstep, &piv_row, &ipiv,
                  &info, &fail, &xch, &rec_stride, &tmo};
  return hipLaunchCooperativeKernel((const void*)panel_lu_kernel, dim3(nwg), dim3(kThreads), args,
                                    (unsigned)plan.lds_bytes, s);
}

}  // namespace rlu
