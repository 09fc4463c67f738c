// C ABI of librlu: argument validation, workspace planning and the launch
// sequence of Algorithm 4.1 (Shabat et al., Section 4) on the caller's stream.
//
// Launch sequence of rlu_factor (FP64 path):
//   Step 1  gaussian            G (n x l) from the seed, unless given
//   Step 2  gemm                Y = A G
//           q times (Section 5.2, power iterations):
//             panel_lu(Y), gemm Z^T = Lv^T A, transpose, panel_lu(Z),
//             lv_dense, gemm Y = A Lv(Z)
//   Step 3  panel_lu(Y)         packed LU of Y in place, rows never moved
//   Step 5  gemm (split-K)      S = Lv^T Lv        (Gram matrix)
//           spd_inverse         S <- S^{-1}
//           gemm                C = Lv^T A
//           gemm                B = S^{-1} C
//   Step 6  panel_lu(B^T)       packed LU of B^T in the storage of B
//   Step 8  assemble            p, q, U = U_b (k x n, positions), L_b, info
//   Step 7  gemm                L = P (Lv L_b)     (rows scattered to positions)
// Lv is the unit-lower factor of Step 3 in original row order; P enters
// only through the row positions, never through a gather of A (Step 5:
// L_y^T P A = Lv^T A).
#include "rlu_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>

static const char* const kPhaseNames[PH_COUNT] = {
    "gaussian", "sketch_gemm", "panel_lu_y", "gram_gemm", "gram_inverse", "project_gemm",
    "solve_gemm", "panel_lu_bt", "assemble_u_lb", "form_l_gemm", "sketch_splitk_sum",
    "project_splitk_sum", "power_iterations", "column_choice", "id_solve"};

namespace rlu_detail {

using namespace rlu;

// A pivoted LU of a tall panel, in one launch when its rows fit the
// workgroups the device holds at once, else in column blocks: each block is
// one launch that continues from the positions the earlier blocks left,
// followed by the block's U rows for the columns to its right (triangular
// solve) and the update of those columns (GEMM with the block's
// multipliers).  Rows never move.
struct BlockedPanel {
  int nblocks = 0, width = 0;   // every block but the last is `width` wide
  PanelPlan main{}, last{};
  size_t u12_elems = 0;
  bool ok = false;
};

BlockedPanel plan_blocked(int nrows, int ncols, int cus) {
  BlockedPanel b;
  PanelPlan p = panel_plan(nrows, ncols, cus, 1);
  if (p.ok) {
    b.nblocks = 1; b.width = ncols; b.main = p; b.last = p; b.ok = true;
    return b;
  }
  const int wmax = panel_block_max_width();
  for (int nb = 2; nb <= 64; ++nb) {
    const int w = (ncols + nb - 1) / nb;
    const int wl = ncols - (nb - 1) * w;
    if (w > wmax || wl <= 0) continue;
    PanelPlan pm = panel_plan(nrows, w, cus, 1), pl = panel_plan(nrows, wl, cus, 1);
    if (!pm.ok || !pl.ok) continue;
    b.nblocks = nb; b.width = w; b.main = pm; b.last = pl; b.ok = true;
    b.u12_elems = (size_t)w * (size_t)(ncols - w);
    return b;
  }
  return b;
}

struct Layout {
  size_t G = 0, Y = 0, part = 0, S = 0, gj = 0, C = 0, Bst = 0, Lb = 0;
  size_t pos_y = 0, rstep_y = 0, piv_y = 0, ipiv_y = 0;
  size_t pos_b = 0, rstep_b = 0, piv_b = 0, ipiv_b = 0, flags = 0, xch = 0;
  size_t total = 0;
  size_t u12 = 0, bt = 0;
  size_t zt = 0, z = 0, piv_z = 0, ipiv_z = 0;  // power iterations (Section 5.2)
  size_t sy = 0, rq = 0, qy = 0, yq = 0;        // rank-revealing Step 3
  size_t sel = 0, gk = 0, tb = 0, wb = 0, aj = 0;  // Algorithm 4.4
  size_t lpw = 0;                                   // 16-bit copies of G / Lv
  BlockedPanel py{}, pb{}, pz{};
};

bool plan_layout(const rlu_problem_t& pb, int cus, Layout& L) {
  const int64_t m = pb.m, n = pb.n, k = pb.k, l = pb.l;
  size_t off = 0;
  auto take = [&](size_t& slot, size_t bytes) {
    slot = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
  };
  const size_t d = sizeof(double);
  const size_t sa = pb.dtype == RLU_F32 ? sizeof(float) : sizeof(double);
  const bool power = pb.power_iters > 0;
  // G, or with power iterations the normalized n x l block that replaces it
  take(L.G, pb.G && !power ? 0 : (size_t)n * l * sa);
  take(L.Y, (size_t)m * l * d);
  // one partial-sum area, sized for the largest automatic split-K product
  size_t part = gemm_auto_partial_elems(m, l, n, OpA::Plain);
  part = std::max(part, gemm_auto_partial_elems(k, k, m, OpA::LvT));
  part = std::max(part, gemm_auto_partial_elems(k, n, m, OpA::LvT));
  part = std::max(part, gemm_auto_partial_elems(k, n, k, OpA::Plain));
  part = std::max(part, gemm_auto_partial_elems(m, k, k, OpA::Lv));
  if (power) part = std::max(part, gemm_auto_partial_elems(l, n, m, OpA::LvT));
  const bool rr = (pb.flags & RLU_FLAG_RRLU) != 0;
  if (rr) part = std::max(part, gemm_auto_partial_elems(l, l, m, OpA::LvT));
  const bool fast = (pb.flags & RLU_FLAG_FAST) != 0;
  if (fast) {
    part = std::max(part, gemm_auto_partial_elems(k, l, m, OpA::LvT));
    part = std::max(part, gemm_auto_partial_elems(k, n, l, OpA::Plain));
  }
  const bool lp = pb.precision == RLU_PREC_MIXED_BF16 || pb.precision == RLU_PREC_MIXED_FP16;
  size_t lpw = 0;
  if (lp) {
    part = std::max(part, gemm_lp_partial_elems(m, l, n));
    part = std::max(part, gemm_lp_partial_elems(k, n, m));
    if (power) part = std::max(part, gemm_lp_partial_elems(l, n, m));
    lpw = std::max(stream_sketch_ws_bytes(n, l), stream_project_ws_bytes(m, k));
    if (power) lpw = std::max(lpw, stream_project_ws_bytes(m, l));
  }
  take(L.part, part * d);
  take(L.lpw, lpw);
  take(L.S, (size_t)k * k * d);
  take(L.gj, spd_inverse_scratch_elems(k) * d);
  take(L.C, (size_t)k * n * d);
  take(L.Bst, (size_t)k * n * d);
  take(L.Lb, (size_t)k * k * d);
  take(L.pos_y, (size_t)m * 4);
  take(L.rstep_y, (size_t)m * 4);
  take(L.piv_y, (size_t)l * 4);
  take(L.ipiv_y, (size_t)l * 4);
  take(L.pos_b, (size_t)n * 4);
  take(L.rstep_b, (size_t)n * 4);
  take(L.piv_b, (size_t)k * 4);
  take(L.ipiv_b, (size_t)k * 4);
  take(L.flags, 64);
  take(L.zt, power ? (size_t)l * n * d : 0);
  take(L.z, power ? (size_t)n * l * d : 0);
  take(L.piv_z, power ? (size_t)l * 4 : 0);
  take(L.ipiv_z, power ? (size_t)l * 4 : 0);
  take(L.sy, rr ? (size_t)l * l * d : 0);
  take(L.rq, rr ? (size_t)l * l * d : 0);
  take(L.qy, rr ? (size_t)l * 4 : 0);
  take(L.yq, rr ? (size_t)m * l * d : 0);
  take(L.sel, fast ? (size_t)l * 4 : 0);
  take(L.gk, fast ? (size_t)k * l * d : 0);
  take(L.tb, fast ? (size_t)k * std::max<int64_t>(l - k, 1) * d : 0);
  take(L.wb, fast ? (size_t)k * l * d : 0);
  take(L.aj, fast ? (size_t)l * n * sa : 0);
  L.py = plan_blocked((int)m, (int)l, cus);
  L.pb = plan_blocked((int)n, (int)k, cus);
  if (!L.py.ok || !L.pb.ok) return false;
  size_t xch = std::max(std::max(L.py.main.xch_bytes, L.py.last.xch_bytes),
                        std::max(L.pb.main.xch_bytes, L.pb.last.xch_bytes));
  size_t u12 = std::max(L.py.u12_elems, L.pb.u12_elems);
  if (power) {
    L.pz = plan_blocked((int)n, (int)l, cus);
    if (!L.pz.ok) return false;
    xch = std::max(xch, std::max(L.pz.main.xch_bytes, L.pz.last.xch_bytes));
    u12 = std::max(u12, L.pz.u12_elems);
  }
  take(L.xch, xch);
  take(L.u12, u12 * d);
  take(L.bt, L.pb.nblocks > 1 ? (size_t)n * k * d : 0);
  L.total = off;
  return true;
}

// The integer a caller stored in an enum field.  A C caller may store any
// int there; reading it as the C++ enum type is only defined for the
// enumerators' range, so the raw bits are read and checked first.
template <typename E>
int raw_enum(const E& e) {
  static_assert(sizeof(E) == sizeof(int), "enums of the C ABI are int-sized");
  int v;
  std::memcpy(&v, &e, sizeof v);
  return v;
}

rlu_status_t validate(const rlu_problem_t* pb) {
  if (!pb) return RLU_ERR_INVALID_ARG;
  const int dt = raw_enum(pb->dtype), pr = raw_enum(pb->precision);
  if (dt != RLU_F64 && dt != RLU_F32) return RLU_ERR_INVALID_ARG;
  if (pr < RLU_PREC_FP64 || pr > RLU_PREC_MIXED_FP16) return RLU_ERR_INVALID_ARG;
  if (pb->m < 1 || pb->n < 1 || pb->k < 1 || pb->l < pb->k) return RLU_ERR_INVALID_ARG;
  if (pb->l > std::min(pb->m, pb->n)) return RLU_ERR_INVALID_ARG;
  if (pb->m >= (1LL << 31) || pb->n >= (1LL << 31)) return RLU_ERR_TOO_LARGE;
  if (pb->dtype != RLU_F64 && pb->dtype != RLU_F32) return RLU_ERR_INVALID_ARG;
  switch (pb->precision) {
    case RLU_PREC_FP64:
      if (pb->dtype != RLU_F64) return RLU_ERR_INVALID_ARG;
      break;
    case RLU_PREC_FP32:
      if (pb->dtype != RLU_F32) return RLU_ERR_INVALID_ARG;
      break;
    case RLU_PREC_MIXED_BF16:
    case RLU_PREC_MIXED_FP16:
      if (pb->dtype != RLU_F32) return RLU_ERR_INVALID_ARG;
      break;
    default:
      return RLU_ERR_INVALID_ARG;
  }
  if (pb->G && pb->ldg < pb->n) return RLU_ERR_INVALID_ARG;
  if (pb->flags & ~(uint32_t)(RLU_FLAG_CHECK_FINITE | RLU_FLAG_DIAGNOSTICS | RLU_FLAG_RRLU |
                              RLU_FLAG_FAST))
    return RLU_ERR_INVALID_ARG;
  if ((pb->flags & RLU_FLAG_RRLU) && pb->l > kSpdColPivMax) return RLU_ERR_UNSUPPORTED;
  if (pb->flags & RLU_FLAG_FAST) {
    // Algorithm 4.4 draws its own sketch matrix and has no power scheme
    if (pb->G || pb->power_iters != 0) return RLU_ERR_INVALID_ARG;
    if (pr != RLU_PREC_FP64 && pr != RLU_PREC_FP32) return RLU_ERR_UNSUPPORTED;
    if (pb->l > 1024 || id_solve_rows((int)pb->l) < 1) return RLU_ERR_UNSUPPORTED;
  }
  if (pb->power_iters < 0 || pb->power_iters > RLU_MAX_POWER_ITERS) return RLU_ERR_INVALID_ARG;
  if (!spd_inverse_supported(pb->k)) return RLU_ERR_UNSUPPORTED;
  return RLU_OK;
}

rlu_status_t validate_io(const rlu_problem_t* pb, const rlu_buffers_t* io) {
  if (!io) return RLU_ERR_INVALID_ARG;
  if (!io->A || !io->L || !io->U || !io->p || !io->q || !io->info) return RLU_ERR_INVALID_ARG;
  if (io->lda < pb->m || io->ldl < pb->m || io->ldu < pb->k) return RLU_ERR_INVALID_ARG;
  if (pb->flags & RLU_FLAG_DIAGNOSTICS) {
    if (io->Y && io->ldy < pb->m) return RLU_ERR_INVALID_ARG;
    if (io->B && io->ldb < pb->k) return RLU_ERR_INVALID_ARG;
  }
  return RLU_OK;
}

rlu_status_t ensure_ws(rlu_handle_s* h, size_t bytes) {
  if (bytes <= h->ws_bytes) return RLU_OK;
  if (h->ws) {
    if (hipFree(h->ws) != hipSuccess) return RLU_ERR_DEVICE;
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  if (hipMalloc(&h->ws, bytes) != hipSuccess) {
    h->ws = nullptr;
    return RLU_ERR_OUT_OF_MEMORY;
  }
  h->ws_bytes = bytes;
  return RLU_OK;
}

rlu_status_t begin_timing(rlu_handle_s* h) {
  h->cur = nullptr;
  if (!h->timing) return RLU_OK;
  TimingSlot& t = h->ring[h->ring_next];
  // timing-only events: no system-scope fence (cache write-back and
  // invalidation) when they are recorded, which would idle the device for
  // several microseconds at every event; they are only read for their
  // timestamps after the call
  auto mk = [](hipEvent_t* e) {
    return hipEventCreateWithFlags(e, hipEventDisableSystemFence) == hipSuccess;
  };
  for (int p = 0; p < PH_COUNT; ++p) {
    for (int e = 0; e < 2; ++e)
      if (!t.ev[p][e] && !mk(&t.ev[p][e])) return RLU_ERR_DEVICE;
    t.used[p] = false;
  }
  t.nk = 0;
  if (h->timing_mode == 3)
    for (int k = 0; k < kMaxKernelTimes; ++k)
      for (int e = 0; e < 2; ++e)
        if (!t.kev[k][e] && !mk(&t.kev[k][e])) return RLU_ERR_DEVICE;
  t.valid = true;
  h->cur = &t;
  h->ring_next = (h->ring_next + 1) % RLU_TIMING_RING;
  if (h->ring_filled < RLU_TIMING_RING) ++h->ring_filled;
  return RLU_OK;
}

}  // namespace rlu_detail

namespace {

using namespace rlu;
using namespace rlu_detail;

// Pivoted LU of the column-major panel X (nrows x ncols, leading dimension
// ld), in one launch or in column blocks (BlockedPanel).
rlu_status_t run_panel(rlu_handle_s* h, double* X, int64_t ld, int nrows, int ncols,
                       const BlockedPanel& bp, int* pos, int* rstep, int* piv, int* ipiv,
                       int* info, int* fail, void* xch, double* u12, long long tmo,
                       hipStream_t s) {
  for (int b = 0; b < bp.nblocks; ++b) {
    const int c0 = b * bp.width;
    const int wb = b == bp.nblocks - 1 ? ncols - c0 : bp.width;
    PanelDesc d{};
    d.X = X + (int64_t)c0 * ld; d.rs = 1; d.cs = ld; d.nrows = nrows; d.ncols = wb;
    d.pos = pos; d.rstep = rstep; d.piv_row = piv + c0; d.ipiv = ipiv + c0;
    d.info = info; d.fail = fail; d.xch = xch; d.timeout_ticks = tmo;
    d.step0 = c0; d.total_cols = ncols;
    d.pos_in = b ? pos : nullptr;
    d.rstep_in = b ? rstep : nullptr;
    {
      KernelScope ks(h, s);
      HIP_TRY(launch_panel_lu(d, b == bp.nblocks - 1 ? bp.last : bp.main, s));
    }
    const int c1 = c0 + wb;
    if (c1 < ncols) {
      // U rows of this block's pivots for the columns to its right ...
      HIP_TRY(launch_block_trsm(X, ld, piv + c0, c0, wb, c1, ncols - c1, u12, s));
      // ... and the update of those columns by the block's multipliers
      GemmDesc g{};
      g.M = nrows; g.N = ncols - c1; g.K = wb;
      g.A = X + (int64_t)c0 * ld; g.lda = ld; g.opa = OpA::LvStrict; g.astep = rstep;
      g.acol0 = c0;
      g.B = u12; g.ldb = wb; g.opb = OpB::Plain;
      g.C = X + (int64_t)c1 * ld; g.ldc = ld;
      g.ksplit = 1; g.csub = true;
      HIP_TRY(launch_gemm<double>(g, s));
    }
  }
  return RLU_OK;
}

// The FP64 path (T = double) and the FP32 path (T = float: FP32 storage of
// A, G, L, U and FP32 MFMA for the two products with A).  The pivoted LUs,
// the Gram matrix, its inverse and B are FP64 in both.
//
// The mixed forms (T = float) replace the FP32 MFMA of the two products with
// BF16 or FP16 MFMA accumulating in FP32 (gemm_lp.hip).
template <typename T>
rlu_status_t factor_path(rlu_handle_s* h, const rlu_problem_t& pb, const rlu_buffers_t& io,
                         hipStream_t s, const Layout& Ly) {
  const bool lp = pb.precision == RLU_PREC_MIXED_BF16 || pb.precision == RLU_PREC_MIXED_FP16;
  const bool fp16 = pb.precision == RLU_PREC_MIXED_FP16;
  const bool kF32 = pb.precision == RLU_PREC_FP32;   // diagnostics stored in FP32
  const int64_t m = pb.m, n = pb.n, k = pb.k, l = pb.l;
  void* ws = h->ws;
  double* Y = at<double>(ws, Ly.Y);   // the sketch; Y Q_y from Step 3 on with RLU_FLAG_RRLU
  double* S = at<double>(ws, Ly.S);
  double* C = at<double>(ws, Ly.C);
  double* Bst = at<double>(ws, Ly.Bst);
  double* Lb = at<double>(ws, Ly.Lb);
  int* pos_y = at<int>(ws, Ly.pos_y);
  int* rstep_y = at<int>(ws, Ly.rstep_y);
  int* piv_y = at<int>(ws, Ly.piv_y);
  int* ipiv_y = at<int>(ws, Ly.ipiv_y);
  int* pos_b = at<int>(ws, Ly.pos_b);
  int* rstep_b = at<int>(ws, Ly.rstep_b);
  int* piv_b = at<int>(ws, Ly.piv_b);
  int* ipiv_b = at<int>(ws, Ly.ipiv_b);
  int* flags = at<int>(ws, Ly.flags);  // [0] info_y, [1] info_b, [2] exchange failure; [8] max|A| (FP16)
  void* xch = at<void>(ws, Ly.xch);
  const bool diag = (pb.flags & RLU_FLAG_DIAGNOSTICS) != 0;

  // the flags start at zero: cleared by Step 1's Gaussian launch when this
  // call draws G (one launch less on small problems), else by a fill here
  const bool clear_in_step1 = !(pb.flags & RLU_FLAG_FAST) && !pb.G && !(lp && fp16) &&
                              !h->xch_preset_fail;
  if (!clear_in_step1) HIP_TRY(launch_fill_u32((uint32_t*)flags, 16, 0u, s));
  // a test of the failure path: the exchange starts as if a partner had
  // already given up
  if (h->xch_preset_fail) HIP_TRY(launch_fill_u32((uint32_t*)flags + 2, 1, 1u, s));
  const long long tmo = h->xch_timeout;
  // FP16 products: the range of A (max|A|, flags[8]), from which they scale A
  // by a power of two before rounding it (lp_scale); BF16 keeps FP32's range
  const unsigned* amax = nullptr;
  if (lp && fp16) {
    HIP_TRY(launch_absmax((const float*)io.A, io.lda, m, n, (unsigned*)(flags + 8), s));
    amax = (const unsigned*)(flags + 8);
  }

  // Step 1 (Algorithm 4.4: the SRFT R = D F S in the place of G)
  const bool fast = (pb.flags & RLU_FLAG_FAST) != 0;
  const T* G = (const T*)pb.G;
  int64_t ldg = pb.ldg;
  if (fast) {
    T* R = at<T>(ws, Ly.G);
    PhaseScope ph(h, PH_GAUSSIAN, s);
    HIP_TRY(launch_srft<T>(R, n, n, (int)l, pb.seed, at<int>(ws, Ly.sel), s));
    G = R;
    ldg = n;
  } else if (!G) {
    T* Gw = at<T>(ws, Ly.G);
    PhaseScope ph(h, PH_GAUSSIAN, s);
    HIP_TRY(launch_gaussian<T>(Gw, n, n, l, pb.seed, s,
                               clear_in_step1 ? (uint32_t*)flags : nullptr));
    G = Gw;
    ldg = n;
  }
  // Y (m x l) = A X for an n x l block X of the storage type (Step 2's
  // product); phase ids < 0 leave it untimed
  auto times_a = [&](const T* X, int64_t ldx, int ph_gemm, int ph_sum) -> rlu_status_t {
    GemmDesc d{};
    d.M = m; d.N = l; d.K = n;
    d.A = io.A; d.lda = io.lda; d.opa = OpA::Plain;
    d.B = X; d.ldb = ldx; d.opb = OpB::Plain;
    d.C = Y; d.ldc = m;
    d.ksplit = 0; d.partial = at<void>(ws, Ly.part);
    if (lp) d.lp_ws = at<void>(ws, Ly.lpw);
    d.amax = amax;
    int ks = 1;
    d.no_sum = true; d.ksplit_out = &ks;
    {
      PhaseScope ph(h, ph_gemm, s);
      if (lp) HIP_TRY(launch_gemm_lp(d, fp16, s));
      else HIP_TRY((launch_gemm_t<T, T, T, double>(d, s)));
    }
    if (ks > 1) {
      PhaseScope ph(h, ph_sum, s);
      HIP_TRY(launch_splitk_sum_f64(m, l, ks, (const double*)d.partial, Y, m, nullptr, s));
    }
    return RLU_OK;
  };
  // Out (rows x n, FP64) = Lv^T A with Lv (m x rows) the unit-lower factor
  // of the pivoted LU of Y (the product of Step 5 and of the power scheme)
  auto lvt_times_a = [&](double* Out, int64_t rows, int ph_gemm, int ph_sum) -> rlu_status_t {
    GemmDesc d{};
    d.M = rows; d.N = n; d.K = m;
    d.A = Y; d.lda = m; d.opa = OpA::LvT; d.astep = rstep_y;
    d.B = io.A; d.ldb = io.lda; d.opb = OpB::Plain;
    d.C = Out; d.ldc = rows;
    d.ksplit = 0; d.partial = at<void>(ws, Ly.part);
    if (lp) d.lp_ws = at<void>(ws, Ly.lpw);
    d.amax = amax;
    int ks = 1;
    d.no_sum = true; d.ksplit_out = &ks;
    {
      PhaseScope ph(h, ph_gemm, s);
      if (lp) HIP_TRY(launch_gemm_lp(d, fp16, s));
      else HIP_TRY((launch_gemm_t<double, T, T, double>(d, s)));
    }
    if (ks > 1) {
      PhaseScope ph(h, ph_sum, s);
      HIP_TRY(launch_splitk_sum_f64(rows, n, ks, (const double*)d.partial, Out, rows, nullptr, s));
    }
    return RLU_OK;
  };

  // Step 2: Y = A G
  {
    rlu_status_t st = times_a(G, ldg, PH_SKETCH, PH_SKETCH_SUM);
    if (st != RLU_OK) return st;
  }
  // the non-finite check the caller asked for: a NaN or infinity in A or G
  // makes its row of Y non-finite
  if (pb.flags & RLU_FLAG_CHECK_FINITE)
    HIP_TRY(launch_check_finite(FiniteTaskDev{Y, m * l, flags + 4}, s));
  // Section 5.2: q power iterations, Y <- A (A^T Y).  Before each product
  // the block is replaced by the unit-lower factor of its pivoted LU in its
  // own row order (bounded entries, same column space).  The normalizations
  // use the positions and row steps of Steps 3 and 6 as scratch and their
  // zero-pivot words go to flags[3].
  if (pb.power_iters > 0) {
    PhaseScope ph(h, PH_POWER, s);
    double* Zt = at<double>(ws, Ly.zt);
    double* Z = at<double>(ws, Ly.z);
    T* Gz = at<T>(ws, Ly.G);
    double* u12 = at<double>(ws, Ly.u12);
    for (int it = 0; it < pb.power_iters; ++it) {
      rlu_status_t st = run_panel(h, Y, m, (int)m, (int)l, Ly.py, pos_y, rstep_y, piv_y, ipiv_y,
                                  flags + 3, flags + 2, xch, u12, tmo, s);
      if (st != RLU_OK) return st;
      st = lvt_times_a(Zt, l, -1, -1);  // Z^T = Lv(Y)^T A  (l x n)
      if (st != RLU_OK) return st;
      HIP_TRY(launch_transpose(Zt, l, Z, n, l, n, s));
      st = run_panel(h, Z, n, (int)n, (int)l, Ly.pz, pos_b, rstep_b, at<int>(ws, Ly.piv_z),
                     at<int>(ws, Ly.ipiv_z), flags + 3, flags + 2, xch, u12, tmo, s);
      if (st != RLU_OK) return st;
      HIP_TRY(launch_lv_dense<T>(Z, n, rstep_b, Gz, n, n, l, s));
      st = times_a(Gz, n, -1, -1);      // Y = A Lv(Z)
      if (st != RLU_OK) return st;
    }
  }
  if (diag && io.Y) {
    if (kF32) HIP_TRY((launch_convert2d<double, float>(Y, m, (float*)io.Y, io.ldy, m, l, s)));
    else HIP_TRY(launch_copy2d<double>(Y, m, (double*)io.Y, io.ldy, m, l, s));
  }
  // Step 3 as listed (RRLU): the column order Q_y of a column-pivoted QR of
  // Y from its Gram matrix (pivoted Cholesky), then Y Q_y replaces Y
  if (pb.flags & RLU_FLAG_RRLU) {
    PhaseScope ph(h, PH_COLPIV, s);
    double* Sy = at<double>(ws, Ly.sy);
    int* qy = at<int>(ws, Ly.qy);
    // S_y = Y^T Y through the Lv operand forms with every row step l (all
    // entries stored); the row steps are rewritten by Step 3's panel
    HIP_TRY(launch_fill_u32((uint32_t*)rstep_y, (size_t)m, (uint32_t)l, s));
    GemmDesc d{};
    d.M = l; d.N = l; d.K = m;
    d.A = Y; d.lda = m; d.opa = OpA::LvT; d.astep = rstep_y;
    d.B = Y; d.ldb = m; d.opb = OpB::Lv; d.bstep = rstep_y;
    d.C = Sy; d.ldc = l;
    d.ksplit = 0; d.partial = at<void>(ws, Ly.part);
    HIP_TRY(launch_gemm<double>(d, s));
    HIP_TRY(launch_colpiv_gram(Sy, l, (int)l, at<double>(ws, Ly.rq), qy, s));
    double* Yq = at<double>(ws, Ly.yq);
    HIP_TRY(launch_gather_cols(Y, m, qy, Yq, m, m, (int)l, s));
    if (diag && io.qy) HIP_TRY(launch_copy_i32(qy, io.qy, l, s));
    Y = Yq;
  }
  // Step 3 (+ Step 4: only the first k columns of the unit-lower factor are used)
  {
    PhaseScope ph(h, PH_PANEL_Y, s);
    rlu_status_t st = run_panel(h, Y, m, (int)m, (int)l, Ly.py, pos_y, rstep_y, piv_y, ipiv_y,
                                flags + 0, flags + 2, xch, at<double>(ws, Ly.u12), tmo, s);
    if (st != RLU_OK) return st;
  }
  if (diag && io.ipiv) HIP_TRY(launch_copy_i32(ipiv_y, io.ipiv, l, s));
  if (fast) {
    // Algorithm 4.4, Steps 5-6: the ID Y = X Y(J, :) from Step 3's LU (J =
    // the rows its steps chose, X = Lv L11^{-1}) and B = L_y^+ P X A(J, :)
    // = W A(J, :) with W = [I_k, T] L11^{-1}, T = S^{-1} Lv_k^T Lv(:, k:l)
    double* Gk = at<double>(ws, Ly.gk);
    {
      GemmDesc d{};  // [S, C2] = Lv_k^T Lv  (k x l)
      d.M = k; d.N = l; d.K = m;
      d.A = Y; d.lda = m; d.opa = OpA::LvT; d.astep = rstep_y;
      d.B = Y; d.ldb = m; d.opb = OpB::Lv; d.bstep = rstep_y;
      d.C = Gk; d.ldc = k;
      d.ksplit = 0; d.partial = at<void>(ws, Ly.part);
      PhaseScope ph(h, PH_GRAM, s);
      HIP_TRY(launch_gemm<double>(d, s));
    }
    {
      PhaseScope ph(h, PH_GRAM_INV, s);
      HIP_TRY(launch_spd_inverse_scratch(Gk, k, at<double>(ws, Ly.gj), s));
    }
    double* Tb = at<double>(ws, Ly.tb);
    if (l > k) {
      GemmDesc d{};  // T = S^{-1} C2
      d.M = k; d.N = l - k; d.K = k;
      d.A = Gk; d.lda = k; d.opa = OpA::Plain;
      d.B = Gk + k * k; d.ldb = k; d.opb = OpB::Plain;
      d.C = Tb; d.ldc = k;
      d.ksplit = 1;
      PhaseScope ph(h, PH_SOLVE, s);
      HIP_TRY(launch_gemm<double>(d, s));
    }
    double* Wb = at<double>(ws, Ly.wb);
    {
      PhaseScope ph(h, PH_ID_SOLVE, s);
      HIP_TRY(launch_id_solve(Tb, k, Y, m, piv_y, (int)k, (int)l, Wb, k, s));
    }
    {
      T* AJ = at<T>(ws, Ly.aj);
      PhaseScope ph(h, PH_PROJECT, s);
      HIP_TRY(launch_gather_rows<T>((const T*)io.A, io.lda, piv_y, (int)l, n, AJ, l, s));
      GemmDesc d{};  // B = W A(J, :)
      d.M = k; d.N = n; d.K = l;
      d.A = Wb; d.lda = k; d.opa = OpA::Plain;
      d.B = AJ; d.ldb = l; d.opb = OpB::Plain;
      d.C = Bst; d.ldc = k;
      d.ksplit = 0; d.partial = at<void>(ws, Ly.part);
      HIP_TRY((launch_gemm_t<double, T, T, double>(d, s)));
    }
  } else {
  // Step 5: S = Lv^T Lv, S <- S^{-1}, C = Lv^T A
  {
    GemmDesc d{};
    d.M = k; d.N = k; d.K = m;
    d.A = Y; d.lda = m; d.opa = OpA::LvT; d.astep = rstep_y;
    d.B = Y; d.ldb = m; d.opb = OpB::Lv; d.bstep = rstep_y;
    d.C = S; d.ldc = k;
    d.sym = true;  // S = Lv^T Lv
    d.ksplit = 0; d.partial = at<void>(ws, Ly.part);
    PhaseScope ph(h, PH_GRAM, s);
    HIP_TRY(launch_gemm<double>(d, s));
  }
  // The inverse runs on the caller's stream before the projection: forking
  // it to a second stream to overlap the projection saved at most the ~10 us
  // of a one-workgroup inverse and, once a process had created more streams
  // than hardware queues, cost up to ~300 us per call in the fork and join.
  {
    PhaseScope ph(h, PH_GRAM_INV, s);
    HIP_TRY(launch_spd_inverse_scratch(S, k, at<double>(ws, Ly.gj), s));
  }
  {
    rlu_status_t st = lvt_times_a(C, k, PH_PROJECT, PH_PROJECT_SUM);
    if (st != RLU_OK) return st;
  }
  {
    GemmDesc d{};
    d.M = k; d.N = n; d.K = k;
    d.A = S; d.lda = k; d.opa = OpA::Plain;
    d.B = C; d.ldb = k; d.opb = OpB::Plain;
    d.C = Bst; d.ldc = k;
    d.ksplit = 1;
    PhaseScope ph(h, PH_SOLVE, s);
    HIP_TRY(launch_gemm<double>(d, s));
  }
  }  // Step 5 of Algorithm 4.1
  if (diag && io.B) {
    if (kF32) HIP_TRY((launch_convert2d<double, float>(Bst, k, (float*)io.B, io.ldb, k, n, s)));
    else HIP_TRY(launch_copy2d<double>(Bst, k, (double*)io.B, io.ldb, k, n, s));
  }
  // Step 6 through the LU of B^T
  {
    PhaseScope ph(h, PH_PANEL_B, s);
    if (Ly.pb.nblocks == 1) {
      PanelDesc d{};
      d.X = Bst; d.rs = k; d.cs = 1; d.nrows = (int)n; d.ncols = (int)k;
      d.pos = pos_b; d.rstep = rstep_b; d.piv_row = piv_b; d.ipiv = ipiv_b;
      d.info = flags + 1; d.fail = flags + 2; d.xch = xch; d.timeout_ticks = tmo;
      KernelScope ks(h, s);
      HIP_TRY(launch_panel_lu(d, Ly.pb.main, s));
    } else {
      // blocked: on a column-major copy of B^T, then back into B's storage
      double* Bt = at<double>(ws, Ly.bt);
      HIP_TRY(launch_transpose(Bst, k, Bt, n, k, n, s));
      rlu_status_t st = run_panel(h, Bt, n, (int)n, (int)k, Ly.pb, pos_b, rstep_b, piv_b, ipiv_b,
                                  flags + 1, flags + 2, xch, at<double>(ws, Ly.u12), tmo, s);
      if (st != RLU_OK) return st;
      HIP_TRY(launch_transpose(Bt, n, Bst, k, n, k, s));
    }
  }
  if (diag && io.qpiv) HIP_TRY(launch_copy_i32(ipiv_b, io.qpiv, k, s));
  {
    // p and q, Step 8 (U = U_b), the L_b that Step 7 needs and the info
    // words, in one launch
    PhaseScope ph(h, PH_ASSEMBLE, s);
    AsmTaskDev a{};
    a.pos_y = pos_y; a.pos_b = pos_b; a.Bst = Bst; a.piv_b = piv_b; a.rstep_b = rstep_b;
    a.m = m; a.n = n; a.k = k;
    a.p = io.p; a.q = io.q; a.U = io.U; a.ldu = io.ldu; a.Lb = Lb;
    a.flags = flags; a.info = io.info;
    HIP_TRY(launch_assemble_one<T>(a, s));
  }
  {
    GemmDesc d{};
    d.M = m; d.N = k; d.K = k;
    d.A = Y; d.lda = m; d.opa = OpA::Lv; d.astep = rstep_y;
    d.B = Lb; d.ldb = k; d.opb = OpB::Plain;
    d.b_lower = true;  // L_b is unit lower triangular
    d.C = io.L; d.ldc = io.ldl;
    d.rowmap = pos_y;
    d.ksplit = 1;
    PhaseScope ph(h, PH_FORM_L, s);
    HIP_TRY((launch_gemm_t<double, double, double, T>(d, s)));
  }
  return RLU_OK;
}

// ----- Rank-deficient least squares (Section 4.4, Algorithm 4.3) ------------

rlu_status_t lstsq_validate(const rlu_lstsq_t* ls) {
  if (!ls) return RLU_ERR_INVALID_ARG;
  if (ls->m < 1 || ls->n < 1 || ls->k < 1 || ls->k > std::min(ls->m, ls->n) || ls->nrhs < 0)
    return RLU_ERR_INVALID_ARG;
  if (ls->m >= (1LL << 31) || ls->n >= (1LL << 31) || ls->nrhs >= (1LL << 31))
    return RLU_ERR_TOO_LARGE;
  const int dt = raw_enum(ls->dtype);
  if (dt != RLU_F64 && dt != RLU_F32) return RLU_ERR_INVALID_ARG;
  if (ls->ldl < ls->m || ls->ldu < ls->k || ls->ldb < ls->m || ls->ldx < ls->n)
    return RLU_ERR_INVALID_ARG;
  if (ls->nrhs > 0 && (!ls->L || !ls->U || !ls->p || !ls->q || !ls->b || !ls->x))
    return RLU_ERR_INVALID_ARG;
  if (ls->k > kLsMaxK || !spd_inverse_supported(ls->k)) return RLU_ERR_UNSUPPORTED;
  return RLU_OK;
}

struct LsLayout {
  size_t Ld = 0, bd = 0, S = 0, gj = 0, C = 0, Yk = 0, steps = 0, part = 0, total = 0;
};

LsLayout lstsq_layout(const rlu_lstsq_t& ls) {
  LsLayout L;
  size_t off = 0;
  auto take = [&](size_t& slot, size_t bytes) {
    slot = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
  };
  const size_t d = sizeof(double);
  const int64_t m = ls.m, k = ls.k, r = std::max<int64_t>(ls.nrhs, 1);
  take(L.Ld, (size_t)m * k * d);
  take(L.bd, ls.dtype == RLU_F32 ? (size_t)m * r * d : 0);
  take(L.S, (size_t)k * k * d);
  take(L.gj, spd_inverse_scratch_elems(k) * d);
  take(L.C, (size_t)k * r * d);
  take(L.Yk, (size_t)k * r * d);
  take(L.steps, (size_t)m * 4);
  take(L.part, std::max(gemm_auto_partial_elems(k, k, m, OpA::LvT),
                        gemm_auto_partial_elems(k, r, m, OpA::LvT)) * d);
  L.total = off;
  return L;
}

// Step 2 as in Step 5 of Algorithm 4.1: with Ld = P^T L (rows scattered),
// L^T P b = Ld^T b and L^T L = Ld^T Ld; Ld enters the products through the
// in-place Lv operand forms with every row step set to k (all entries
// stored), so no transposed copy is made.
template <typename T>
rlu_status_t lstsq_path(rlu_handle_s* h, const rlu_lstsq_t& ls, hipStream_t s,
                        const LsLayout& Ly) {
  const int64_t m = ls.m, n = ls.n, k = ls.k, r = ls.nrhs;
  void* ws = h->ws;
  double* Ld = at<double>(ws, Ly.Ld);
  double* S = at<double>(ws, Ly.S);
  double* C = at<double>(ws, Ly.C);
  double* Yk = at<double>(ws, Ly.Yk);
  int* steps = at<int>(ws, Ly.steps);
  HIP_TRY(launch_fill_u32((uint32_t*)steps, (size_t)m, (uint32_t)k, s));
  HIP_TRY(launch_lstsq_scatter_rows<T>((const T*)ls.L, ls.ldl, ls.p, m, k, Ld, s));
  const double* bd = (const double*)ls.b;
  int64_t ldb = ls.ldb;
  if (std::is_same<T, float>::value) {
    double* bw = at<double>(ws, Ly.bd);
    HIP_TRY((launch_convert2d<float, double>((const float*)ls.b, ls.ldb, bw, m, m, r, s)));
    bd = bw;
    ldb = m;
  }
  {  // S = Ld^T Ld
    GemmDesc g{};
    g.M = k; g.N = k; g.K = m;
    g.A = Ld; g.lda = m; g.opa = OpA::LvT; g.astep = steps;
    g.B = Ld; g.ldb = m; g.opb = OpB::Lv; g.bstep = steps;
    g.C = S; g.ldc = k;
    g.ksplit = 0; g.partial = at<void>(ws, Ly.part);
    HIP_TRY(launch_gemm<double>(g, s));
  }
  HIP_TRY(launch_spd_inverse_scratch(S, k, at<double>(ws, Ly.gj), s));
  {  // C = Ld^T b
    GemmDesc g{};
    g.M = k; g.N = r; g.K = m;
    g.A = Ld; g.lda = m; g.opa = OpA::LvT; g.astep = steps;
    g.B = bd; g.ldb = ldb; g.opb = OpB::Plain;
    g.C = C; g.ldc = k;
    g.ksplit = 0; g.partial = at<void>(ws, Ly.part);
    HIP_TRY(launch_gemm<double>(g, s));
  }
  {  // y = S^{-1} C
    GemmDesc g{};
    g.M = k; g.N = r; g.K = k;
    g.A = S; g.lda = k; g.opa = OpA::Plain;
    g.B = C; g.ldb = k; g.opb = OpB::Plain;
    g.C = Yk; g.ldc = k;
    g.ksplit = 1;
    HIP_TRY(launch_gemm<double>(g, s));
  }
  // Steps 3-5
  HIP_TRY(launch_lstsq_back<T>((const T*)ls.U, ls.ldu, Yk, k, ls.q, n, r, (T*)ls.x, ls.ldx, s));
  return RLU_OK;
}

}  // namespace

// ----- Device scratch of rlu_factor_noalloc ----------------------------------
// A file-scope device array that the loader places on every device the
// library runs on, held until the process ends.  Host code never uses its
// name as an address: rlu_create looks up each device's copy once, with
// that device current, and rlu_factor_noalloc passes that address on.
constexpr size_t kStaticScratchBytes = RLU_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Once per device, with `device` current: the address of its scratch copy.
void lookup_scratch(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p) g_scratch_ptr[device] = p;
}

void* scratch_of(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}
}  // namespace

using namespace rlu_detail;

extern "C" {

rlu_status_t rlu_create(rlu_handle_t* out, int device) {
  if (!out) return RLU_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return RLU_ERR_INVALID_ARG;
  rlu_handle_s* h = new (std::nothrow) rlu_handle_s();
  if (!h) return RLU_ERR_OUT_OF_MEMORY;
  h->device = device;
  int prev = 0;
  hipGetDevice(&prev);
  if (hipSetDevice(device) != hipSuccess) { delete h; return RLU_ERR_DEVICE; }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) h->cus = prop.multiProcessorCount;
  // (the capture stream of rlu_factor_batched is created on its first use)
  if (hipEventCreateWithFlags(&h->ev_stage, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_panel, hipEventDisableTiming) != hipSuccess) {
    hipSetDevice(prev);
    delete h;
    return RLU_ERR_DEVICE;
  }
  lookup_scratch(device);  // set-up of rlu_factor_noalloc on this device
  hipSetDevice(prev);
  *out = h;
  return RLU_OK;
}

rlu_status_t rlu_destroy(rlu_handle_t h) {
  if (!h) return RLU_ERR_INVALID_ARG;
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(h->device);
  hipDeviceSynchronize();
  if (h->ws) hipFree(h->ws);
  for (auto& t : h->ring) {
    for (int p = 0; p < PH_COUNT; ++p)
      for (int e = 0; e < 2; ++e)
        if (t.ev[p][e]) hipEventDestroy(t.ev[p][e]);
    for (int k = 0; k < kMaxKernelTimes; ++k)
      for (int e = 0; e < 2; ++e)
        if (t.kev[k][e]) hipEventDestroy(t.kev[k][e]);
  }
  if (h->bgraph.exec) hipGraphExecDestroy(h->bgraph.exec);
  if (h->bgraph.graph) hipGraphDestroy(h->bgraph.graph);
  if (h->bws) hipFree(h->bws);
  if (h->stage) hipHostFree(h->stage);
  if (h->ev_stage) hipEventDestroy(h->ev_stage);
  if (h->ev_panel) hipEventDestroy(h->ev_panel);
  if (h->cap) hipStreamDestroy(h->cap);
  hipSetDevice(prev);
  delete h;
  return RLU_OK;
}

rlu_status_t rlu_workspace_size(const rlu_problem_t* pb, size_t* bytes) {
  if (!bytes) return RLU_ERR_INVALID_ARG;
  const rlu_status_t st = validate(pb);
  if (st != RLU_OK) return st;
  Layout L;
  if (!plan_layout(*pb, 256, L)) return RLU_ERR_UNSUPPORTED;
  *bytes = L.total;
  return RLU_OK;
}

rlu_status_t rlu_factor(rlu_handle_t h, const rlu_problem_t* pb, const rlu_buffers_t* io,
                        rlu_stream_t stream) {
  if (!h) return RLU_ERR_INVALID_ARG;
  rlu_status_t st = validate(pb);
  if (st != RLU_OK) return st;
  st = validate_io(pb, io);
  if (st != RLU_OK) return st;
  Layout L;
  if (!plan_layout(*pb, h->cus, L)) return RLU_ERR_UNSUPPORTED;
  int prev = 0;
  hipGetDevice(&prev);
  if (prev != h->device && hipSetDevice(h->device) != hipSuccess) return RLU_ERR_DEVICE;
  st = ensure_ws(h, L.total);
  if (st == RLU_OK) st = begin_timing(h);
  if (st == RLU_OK) {
    if (pb->precision == RLU_PREC_FP64)
      st = factor_path<double>(h, *pb, *io, (hipStream_t)stream, L);
    else
      st = factor_path<float>(h, *pb, *io, (hipStream_t)stream, L);
  }
  if (prev != h->device) hipSetDevice(prev);
  return st;
}

rlu_status_t rlu_factor_noalloc(rlu_handle_t h, const rlu_problem_t* pb,
                                const rlu_buffers_t* io, rlu_stream_t stream) {
  if (!h) return RLU_ERR_INVALID_ARG;
  rlu_status_t st = validate(pb);
  if (st != RLU_OK) return st;
  st = validate_io(pb, io);
  if (st != RLU_OK) return st;
  Layout L;
  if (!plan_layout(*pb, h->cus, L)) return RLU_ERR_UNSUPPORTED;
  if (L.total > kStaticScratchBytes) return RLU_ERR_TOO_LARGE;
  void* ws = scratch_of(h->device);
  if (!ws) return RLU_ERR_DEVICE;
  int prev = 0;
  hipGetDevice(&prev);
  if (prev != h->device && hipSetDevice(h->device) != hipSuccess) return RLU_ERR_DEVICE;
  // the handle's own workspace and timing are left alone: a view of the
  // handle whose workspace is the device scratch, with timing off
  void* const ws_own = h->ws;
  const size_t ws_own_bytes = h->ws_bytes;
  const bool timing = h->timing;
  h->ws = ws;
  h->ws_bytes = kStaticScratchBytes;
  h->timing = false;
  h->cur = nullptr;
  if (pb->precision == RLU_PREC_FP64)
    st = factor_path<double>(h, *pb, *io, (hipStream_t)stream, L);
  else
    st = factor_path<float>(h, *pb, *io, (hipStream_t)stream, L);
  h->ws = ws_own;
  h->ws_bytes = ws_own_bytes;
  h->timing = timing;
  if (prev != h->device) hipSetDevice(prev);
  return st;
}

rlu_status_t rlu_lstsq_workspace_size(const rlu_lstsq_t* ls, size_t* bytes) {
  if (!bytes) return RLU_ERR_INVALID_ARG;
  const rlu_status_t st = lstsq_validate(ls);
  if (st != RLU_OK) return st;
  *bytes = lstsq_layout(*ls).total;
  return RLU_OK;
}

rlu_status_t rlu_lstsq(rlu_handle_t h, const rlu_lstsq_t* ls, rlu_stream_t stream) {
  if (!h) return RLU_ERR_INVALID_ARG;
  rlu_status_t st = lstsq_validate(ls);
  if (st != RLU_OK) return st;
  if (ls->nrhs == 0) return RLU_OK;
  const LsLayout L = lstsq_layout(*ls);
  int prev = 0;
  hipGetDevice(&prev);
  if (prev != h->device && hipSetDevice(h->device) != hipSuccess) return RLU_ERR_DEVICE;
  st = ensure_ws(h, L.total);
  if (st == RLU_OK) {
    if (ls->dtype == RLU_F64) st = lstsq_path<double>(h, *ls, (hipStream_t)stream, L);
    else st = lstsq_path<float>(h, *ls, (hipStream_t)stream, L);
  }
  if (prev != h->device) hipSetDevice(prev);
  return st;
}

rlu_status_t rlu_set_timing(rlu_handle_t h, int enable) {
  if (!h || enable < 0 || enable > 3) return RLU_ERR_INVALID_ARG;
  h->timing = enable != 0;
  h->timing_mode = enable;
  if (!h->timing) { h->ring_filled = 0; h->ring_next = 0; }
  return RLU_OK;
}

rlu_status_t rlu_phase_times(rlu_handle_t h, int back, float* ms, const char** names, int cap,
                             int* count) {
  if (!h || back < 0 || back >= h->ring_filled || cap < 0) return RLU_ERR_INVALID_ARG;
  const int slot = ((h->ring_next - 1 - back) % RLU_TIMING_RING + RLU_TIMING_RING) % RLU_TIMING_RING;
  TimingSlot& t = h->ring[slot];
  if (!t.valid) return RLU_ERR_INVALID_ARG;
  for (int p = 0; p < PH_COUNT && p < cap; ++p) {
    float v = 0.f;
    if (t.used[p]) {
      if (hipEventSynchronize(t.ev[p][1]) != hipSuccess ||
          hipEventElapsedTime(&v, t.ev[p][0], t.ev[p][1]) != hipSuccess)
        return RLU_ERR_DEVICE;
    }
    if (ms) ms[p] = v;
    if (names) names[p] = kPhaseNames[p];
  }
  for (int k = 0; k < t.nk && PH_COUNT + k < cap; ++k) {
    float v = 0.f;
    if (hipEventSynchronize(t.kev[k][1]) != hipSuccess ||
        hipEventElapsedTime(&v, t.kev[k][0], t.kev[k][1]) != hipSuccess)
      return RLU_ERR_DEVICE;
    if (ms) ms[PH_COUNT + k] = v;
    if (names) names[PH_COUNT + k] = "panel_lu_kernel";
  }
  if (count) *count = PH_COUNT + t.nk;
  return RLU_OK;
}

rlu_status_t rlu_check_info(const int32_t info_host[3]) {
  if (!info_host) return RLU_ERR_INVALID_ARG;
  if (info_host[2] & 1) return RLU_ERR_DEVICE;
  if (info_host[2] & 2) return RLU_ERR_NONFINITE;
  if (info_host[2] != 0) return RLU_ERR_DEVICE;
  if (info_host[0] != 0 || info_host[1] != 0) return RLU_WARN_ZERO_PIVOT;
  return RLU_OK;
}

rlu_status_t rlu_set_exchange_limit(rlu_handle_t h, int64_t timeout_ticks, int preset_failure) {
  if (!h || preset_failure < 0 || preset_failure > 1) return RLU_ERR_INVALID_ARG;
  h->xch_timeout = timeout_ticks < 0 ? kTimeoutTicks : (long long)timeout_ticks;
  h->xch_preset_fail = preset_failure != 0;
  return RLU_OK;
}

const char* rlu_status_string(rlu_status_t st) {
  switch (st) {
    case RLU_OK: return "ok";
    case RLU_PENDING: return "pending";
    case RLU_WARN_ZERO_PIVOT: return "zero pivot (rank below k)";
    case RLU_ERR_INVALID_ARG: return "invalid argument";
    case RLU_ERR_OUT_OF_MEMORY: return "out of device memory";
    case RLU_ERR_DEVICE: return "device error";
    case RLU_ERR_TOO_LARGE: return "problem too large";
    case RLU_ERR_QUEUE_FULL: return "queue full";
    case RLU_ERR_NONFINITE: return "non-finite input";
    case RLU_ERR_UNKNOWN_TICKET: return "unknown ticket";
    case RLU_ERR_UNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

const char* rlu_version(void) { return "rlu-mi355x 0.1 (gfx950)"; }

}  // extern "C"
