// Host-side launchers of the librlu HIP kernels (internal interface between
// the kernel translation units and the C ABI in rlu_api.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rlu {

// ----- Step 1: Gaussian test matrix (rng.hip) ------------------------------
// clear (optional): 16 words the launch also sets to zero (a call's flags,
// saving it a launch of its own).
template <typename T>
hipError_t launch_gaussian(T* G, int64_t ldg, int64_t n, int64_t l, uint64_t seed,
                           hipStream_t s, uint32_t* clear = nullptr);
struct GaussTaskDev { void* G; int64_t ldg, n, l; uint64_t seed; };
// One launch for a batch of test matrices (max_elems = largest n l).
template <typename T>
hipError_t launch_gaussian_batched(const GaussTaskDev* tasks, int count, int64_t max_elems,
                                   hipStream_t s);

// Step 1 of Algorithm 4.4: the SRFT R = D F S (n x l, storage T, ld ldr)
// drawn from `seed`; sel (length l, device) receives S's column indices.
// l <= 1024, l <= n < 2^31.
template <typename T>
hipError_t launch_srft(T* R, int64_t ldr, int64_t n, int l, uint64_t seed, int* sel,
                       hipStream_t s);

// ----- MFMA GEMM (gemm.hip) -----------------------------------------------
// C(M x N) = op(A)(M x K) * op(B)(K x N), all column-major with leading
// dimensions.  Operand forms:
enum class OpA {
  Plain,      // A(i, kk) = A[i + kk*lda]                      (M contiguous)
  LvT,        // A(i, kk) = Lv(kk, i), Lv stored as Y[kk + i*lda]
  Lv,         // A(i, kk) = Lv(i, kk), Lv stored as Y[i + kk*lda]
  LvStrict    // A(i, kk) = Y[i + kk*lda] if acol0 + kk < astep[i], else 0 (the
              // multipliers of a block of columns starting at acol0)
};
enum class OpB {
  Plain,      // B(kk, j) = B[kk + j*ldb]                      (K contiguous)
  Lv          // B(kk, j) = Lv(kk, j), Lv stored as Y[kk + j*ldb]
};
struct GemmDesc {
  int64_t M, N, K;
  const void* A; int64_t lda; OpA opa; const int* astep;  // Lv row steps
  const void* B; int64_t ldb; OpB opb; const int* bstep;
  void* C; int64_t ldc;
  const int* rowmap;   // optional: output row i goes to C row rowmap[i]
  int ksplit;          // 0: automatic split-K (uses `partial` if given), 1: none,
                       // >1: that many partial sums, added in a fixed order
  void* partial;       // partial-sum workspace (gemm_auto_partial_elems elements)
  bool no_sum;         // with a split: leave the partial sums (launch_splitk_sum_f64 adds them)
  int* ksplit_out;     // optional: receives the split used (1 = none)
  int acol0;           // LvStrict: global index of the first column of A
  bool csub;           // C -= op(A) op(B) instead of C = ... (requires ksplit 1)
  bool b_lower;        // op(B) is lower triangular (B(t, j) = 0 for t < j): a tile
                       // skips the K slices above its first column
  bool sym;            // C is symmetric (M == N, op(A) = op(B)^T): only the tiles on
                       // and below the diagonal are computed, each also written to
                       // its mirror image (square tiles, no rowmap or csub)
  void* lp_ws;         // low-precision products: room for the pre-converted small
                       // operand (stream_sketch_ws_bytes / stream_project_ws_bytes)
  const unsigned* amax;  // FP16 products: max|A| (FP32 bits) for the range scale of A
                         // (lp_scale); null: unscaled
};
template <typename T>
hipError_t launch_gemm(const GemmDesc& d, hipStream_t s);
// Operand storage types TA, TB, MFMA type TC, output type TO (instantiated for
// the combinations the library uses).
template <typename TA, typename TB, typename TC, typename TO>
hipError_t launch_gemm_t(const GemmDesc& d, hipStream_t s);
size_t gemm_partial_elems(int64_t M, int64_t N, int ksplit);
size_t gemm_auto_partial_elems(int64_t M, int64_t N, int64_t K, OpA opa);
// C = sum of ksplit partial products (M x N each, stored contiguously), added
// in a fixed order; optional output row map.
hipError_t launch_splitk_sum_f64(int64_t M, int64_t N, int ksplit, const double* partial,
                                 double* C, int64_t ldc, const int* rowmap, hipStream_t s);
// Low-precision products of the mixed form (gemm_lp.hip): BF16 (or FP16) MFMA
// with FP32 accumulation and an FP64 result.  Y = A G (opa Plain: FP32 A and
// G) or C = Lv^T A (opa LvT: FP64 Lv carried as a 16-bit hi + lo pair, FP32
// A).  ksplit is chosen internally when `partial` is given.
hipError_t launch_gemm_lp(const GemmDesc& d, bool fp16, hipStream_t s);
size_t gemm_lp_partial_elems(int64_t M, int64_t N, int64_t K);
// Streaming forms of the two low-precision passes over A (gemm_lp_stream.hip),
// taken by launch_gemm_lp when d.lp_ws is given and the shape fits: a
// workgroup owns 64 rows (Y = A G) or 64 columns (C = Lv^T A) of A over the
// whole of the small dimension, so A is read once; the small operand is
// rounded once into lp_ws.  npad / rpad: the padded small dimension (-1 when
// it exceeds the compiled widths).
int64_t stream_sketch_npad(int64_t N);
size_t stream_sketch_ws_bytes(int64_t K, int64_t N);
size_t stream_sketch_partial_elems(int64_t M, int64_t N, int64_t K);
bool stream_sketch_applies(const GemmDesc& d);
hipError_t launch_sketch_stream_lp(const GemmDesc& d, bool fp16, hipStream_t s);
int64_t stream_project_rpad(int64_t R);
size_t stream_project_ws_bytes(int64_t K, int64_t R);
size_t stream_project_partial_elems(int64_t R, int64_t N, int64_t K);
bool stream_project_applies(const GemmDesc& d);
hipError_t launch_project_stream_lp(const GemmDesc& d, bool fp16, hipStream_t s);
// Tuning override of the tile shape (index into the compiled shapes; -1 = automatic).
void gemm_force_config(int id);
// Grouped form: many independent products in one launch.  Each workgroup
// reads its (task, tile) from `map` (one int2 per workgroup).  Split-K
// tasks (ksplit > 1) write `partial` (ksplit x M x N, FP64 output only) and
// need launch_splitk_sum_grouped afterwards.
struct GemmTaskDev {
  int64_t M, N, K;
  const void* A; int64_t lda; const int* astep;
  const void* B; int64_t ldb; const int* bstep;
  void* C; int64_t ldc; const int* rowmap;
  void* partial; int ksplit; int tiles_m, tiles_n;
  const unsigned* amax;  // as GemmDesc::amax (low-precision products)
};
// Compiled tile shapes (index = cfg; gemm_cfg_name gives "BMxBNxBK").
enum { GEMM_CFG_64x64 = 0, GEMM_CFG_64x112 = 1, GEMM_CFG_112x64 = 2, GEMM_CFG_64x112x32 = 3,
       GEMM_CFG_112x64x32 = 4, GEMM_CFG_64x64x32 = 6, GEMM_CFG_128x64 = 7,
       GEMM_CFG_64x128 = 8, GEMM_CFG_COUNT = 11 };
void gemm_group_tile(int cfg, int* bm, int* bn);
bool gemm_group_cfg_valid(int cfg);
const char* gemm_cfg_name(int cfg);
// The five products of the method as grouped launches.
enum class GemmRole { Sketch = 0, Gram = 1, Project = 2, Solve = 3, FormL = 4 };
hipError_t launch_gemm_grouped_role(GemmRole role, bool f32, int cfg, const GemmTaskDev* tasks,
                                    const int2* map, int nwg, hipStream_t s);
hipError_t launch_splitk_sum_grouped(const GemmTaskDev* tasks, int count, int64_t max_elems,
                                     hipStream_t s);
// Grouped low-precision products (64 x 64 tiles, no split-K): opa Plain
// (FP32 A and G) or LvT (FP64 Lv as a hi + lo pair, FP32 A), FP64 output.
hipError_t launch_gemm_lp_grouped(OpA opa, bool fp16, const GemmTaskDev* tasks, const int2* map,
                                  int nwg, hipStream_t s);
// max|A| of an FP32 matrix (m x n, column-major) into *word as FP32 bits, by
// atomic maximum (the word must start at zero): the FP16 products' range.
hipError_t launch_absmax(const float* A, int64_t lda, int64_t m, int64_t n, unsigned* word,
                         hipStream_t s);
struct AbsmaxTaskDev { const float* A; int64_t lda, m, n; unsigned* word; };
hipError_t launch_absmax_batched(const AbsmaxTaskDev* tasks, int count, hipStream_t s);

// ----- Pivoted LU of a tall matrix, rows spread over workgroups (panel_lu.hip)
struct PanelDesc {
  void* X; int64_t rs, cs;   // element (row r, col c) at X[r*rs + c*cs]
  int nrows, ncols;          // factors all ncols columns, ncols <= nrows
  int* pos;                  // out [nrows]: final position of each row
  int* rstep;                // out [nrows]: step that chose the row (ncols if none)
  int* piv_row;              // out [ncols]: row chosen at each step
  int* ipiv;                 // out [ncols]: LAPACK-style swap target (position)
  int* info;                 // out: first zero-pivot step (1-based), 0 if none
  int* fail;                 // out: set to 1 if the exchange timed out
  void* xch;                 // exchange area, panel_xch_bytes()
  long long timeout_ticks;   // bound on every wait (100 MHz ticks)
  // Continuing a factorization whose first step0 columns were factored by
  // earlier launches (X, piv_row and ipiv then point at column step0):
  int step0;                 // global index of the first column (0: fresh)
  int total_cols;            // columns of the whole factorization (0: ncols)
  const int* pos_in;         // positions after the earlier columns (nullable)
  const int* rstep_in;       // choosing steps so far (nullable: none chosen)
};
// regs: one workgroup holding the panel in registers (at most 32 columns and
// 1024 or 2048 rows for up to 32 or 16 columns); RLU_PANEL_REGS=0
// in the environment, read at each plan, turns it off (the LDS-resident
// kernels then take these panels, as they take all others).
struct PanelPlan { int rows_per_wg; int nwg; size_t lds_bytes; size_t xch_bytes; bool ok; bool regs; };
PanelPlan panel_plan(int nrows, int ncols, int device_cus, int max_wg_per_cu_hint);
hipError_t launch_panel_lu(const PanelDesc& d, const PanelPlan& plan, hipStream_t s);
// Between column blocks of a blocked factorization of a column-major X:
// U (w x nrhs, ld w) = L11^{-1} X(pr, c1 : c1 + nrhs), L11 the unit-lower
// multipliers of the block's pivot rows pr = piv_row[0..w) (columns c0..).
hipError_t launch_block_trsm(const double* X, int64_t ldx, const int* piv_row, int c0, int w,
                             int64_t c1, int nrhs, double* U, hipStream_t s);
int panel_block_max_width();
// One panel of a batched launch, as the device reads it.
struct PanelTaskDev {
  double* X; int64_t rs, cs;
  int nrows, ncols, R, nwg;
  int* pos; int* rstep; int* piv_row; int* ipiv; int* info; int* fail;
  char* xch; int64_t rec_stride;
};
int64_t panel_rec_stride(int ncols);
// exchange area of a panel launch with nwg workgroups (three step buffers)
size_t panel_xch_bytes(int nwg, int ncols);
size_t panel_lds_bytes(int R, int ncols);
// Workgroups of the batched panel kernel the device holds at once (0 on error).
int panel_batched_slots(int max_R, size_t lds_bytes, int cus);
// Persistent launch over many panels (tasks and the round schedule in device
// memory; nslots workgroups, each round one panel member per workgroup).
// Exchange areas must be zeroed beforehand.
hipError_t launch_panel_lu_batched(const PanelTaskDev* tasks, const int* sched, int rounds,
                                   int nslots, int max_R, size_t lds_bytes,
                                   long long timeout_ticks, hipStream_t s);

// ----- Inverse of the k x k Gram matrix (spd_inverse.hip) ------------------
// The blocked symmetric sweep: one launch per 64 pivots (plus a copy when
// the block count is odd, k > 64); the scratch of a matrix holds
// spd_inverse_scratch_elems(k) doubles (unused for k <= 64).
constexpr int64_t kSpdMaxK = 1024;
bool spd_inverse_supported(int64_t k);
struct SpdTaskDev { double* S; int k; double* scratch; };
size_t spd_inverse_scratch_elems(int64_t k);
// Batch: one entry per matrix, tasks in device memory.
hipError_t launch_spd_inverse_batched(const SpdTaskDev* tasks, int count, int64_t kmax,
                                     hipStream_t s);
// One matrix.
hipError_t launch_spd_inverse_scratch(double* S, int64_t k, double* scratch, hipStream_t s);

// ----- Steps 5-6 of Algorithm 4.4 (fast_lu.hip) ------------------------------
// W (k x l) with W L11 = [I_k, T], L11(c', c) = Y[J[c'] + c ldy] (c < c') the
// unit-lower factor of Step 3 on the rows J it chose; T is k x (l - k).
int id_solve_rows(int l);   // rows of W per workgroup (0: l too large)
hipError_t launch_id_solve(const double* T, int64_t ldt, const double* Y, int64_t ldy,
                           const int* J, int k, int l, double* W, int64_t ldw, hipStream_t s);
// AJ (l x n, ld ldaj) = A(J, :)
template <typename T>
hipError_t launch_gather_rows(const T* A, int64_t lda, const int* J, int l, int64_t n, T* AJ,
                              int64_t ldaj, hipStream_t s);

// ----- Rank-revealing Step 3 (rrlu.hip) --------------------------------------
// Column order of a column-pivoted QR of Y from its Gram matrix S = Y^T Y
// (l x l, FP64, ld lds): pivoted Cholesky in one workgroup, l <= kSpdColPivMax;
// R is l x l FP64 scratch, qy (length l) receives the order.
constexpr int kSpdColPivMax = 1024;
hipError_t launch_colpiv_gram(const double* S, int64_t lds, int l, double* R, int* qy,
                              hipStream_t s);
// Yq(:, j) = Y(:, qy[j]) for j < l (m rows).
hipError_t launch_gather_cols(const double* Y, int64_t ldy, const int* qy, double* Yq,
                              int64_t ldq, int64_t m, int l, hipStream_t s);

// ----- Rank-deficient least squares, Algorithm 4.3 (lstsq.hip) -------------
constexpr int kLsMaxK = 1024;   // largest k of the back substitution (= kSpdMaxK)
// Ld (m x k, FP64, ld m) with row p[i] = row i of L (entries of p outside
// [0, m) are skipped).
template <typename T>
hipError_t launch_lstsq_scatter_rows(const T* L, int64_t ldl, const int64_t* p, int64_t m,
                                     int64_t k, double* Ld, hipStream_t s);
// X(:, r) = Q (U_1^{-1} Y(:, r); 0) for r < nrhs; U_1 = U(0:k, 0:k); Y is
// k x nrhs FP64 (ld k); a zero diagonal entry of U_1 gives a zero unknown.
template <typename T>
hipError_t launch_lstsq_back(const T* U, int64_t ldu, const double* Y, int64_t k,
                             const int64_t* q, int64_t n, int64_t nrhs, T* X, int64_t ldx,
                             hipStream_t s);

// ----- Permutations and factor assembly (finish.hip) ------------------------
// dst (rows x cols, TO) = src (TI), element-wise conversion
template <typename TI, typename TO>
hipError_t launch_convert2d(const TI* src, int64_t lds, TO* dst, int64_t ldd, int64_t rows,
                            int64_t cols, hipStream_t s);
template <typename T>
hipError_t launch_copy2d(const T* src, int64_t lds, T* dst, int64_t ldd, int64_t rows,
                         int64_t cols, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, size_t count, uint32_t v, hipStream_t s);
// out (rows x cols, TO) = the unit-lower factor Lv held in place in X by a
// pivoted LU with row steps rstep (see lv_value); the normalization of the
// power iterations (Section 5.2)
template <typename TO>
hipError_t launch_lv_dense(const double* X, int64_t ldx, const int* rstep, TO* out, int64_t ldo,
                           int64_t rows, int64_t cols, hipStream_t s);
// Batched: task t gives out (rows x cols, TO, ld ldo) = Lv of the panel whose
// entry (i, c) is X[i rs + c cs] (max_elems = largest rows cols).
struct LvDenseTaskDev {
  const double* X; int64_t rs, cs; const int* rstep;
  void* out; int64_t ldo, rows, cols;
};
template <typename TO>
hipError_t launch_lv_dense_batched(const LvDenseTaskDev* tasks, int count, int64_t max_elems,
                                   hipStream_t s);
hipError_t launch_copy_i32(const int* src, int32_t* dst, int64_t n, hipStream_t s);
// dst (cols x rows, ld ldd) = src (rows x cols, ld lds)^T
hipError_t launch_transpose(const double* src, int64_t lds, double* dst, int64_t ldd,
                            int64_t rows, int64_t cols, hipStream_t s);
// Batched assembly of p, q, U (TO), L_b and info (max_elems = largest
// m + n + k n + k k of the batch).
struct AsmTaskDev {
  const int* pos_y; const int* pos_b; const double* Bst; const int* piv_b; const int* rstep_b;
  int64_t m, n, k;
  int64_t* p; int64_t* q; void* U; int64_t ldu; double* Lb;
  const int* flags; int32_t* info;
};
template <typename TO>
hipError_t launch_assemble_batched(const AsmTaskDev* tasks, int count, int64_t max_elems,
                                   hipStream_t s);
// The same for one problem, its task passed by value.
template <typename TO>
hipError_t launch_assemble_one(const AsmTaskDev& t, hipStream_t s);
// flag = 1 if Y (count contiguous FP64 values) holds a NaN or an infinity;
// the flag is left alone otherwise.
struct FiniteTaskDev { const double* Y; int64_t count; int* flag; };
hipError_t launch_check_finite(const FiniteTaskDev& t, hipStream_t s);
hipError_t launch_check_finite_batched(const FiniteTaskDev* tasks, int count, int64_t max_elems,
                                       hipStream_t s);

}  // namespace rlu
