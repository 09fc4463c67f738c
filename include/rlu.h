/*
 * rlu.h -- C ABI of the MI355X randomized LU library (librlu.so).
 *
 * Computes the randomized LU decomposition of Shabat, Shmueli, Aizenbud and
 * Averbuch (arXiv 1310.7202), Section 4, Algorithm 4.1: for an m x n matrix A,
 * a target rank k and a sketch width l (k <= l <= min(m, n)),
 *
 *   Step 1  G      <- n x l i.i.d. N(0, 1)
 *   Step 2  Y      <- A G
 *   Step 3  P Y    =  L_y U_y        (LU with partial pivoting; the Remark
 *                                     after Algorithm 4.1 allows it in place
 *                                     of a rank-revealing LU)
 *   Step 4  L_y    <- L_y(:, 1:k)
 *   Step 5  B      <- L_y^+ P A      (pseudo-inverse through the Gram matrix
 *                                     L_y^T L_y, as in the Remark after
 *                                     Algorithm 4.1)
 *   Step 6  B Q    =  L_b U_b        (LU with column pivoting)
 *   Step 7  L      <- L_y L_b
 *   Step 8  U      <- U_b
 *
 * with ||P A Q - L U||_2 controlled by sigma_{k+1}(A) (Theorem 4.1).
 *
 * Conventions
 *   - Matrices are column-major with an explicit leading dimension; indices
 *     are 0-based.
 *   - Every matrix, permutation and info pointer in rlu_buffers_t is a DEVICE
 *     pointer on the handle's device.  The caller owns all of them.
 *   - Permutations are index vectors: (P A)(i, :) = A(p[i], :) and
 *     (A Q)(:, j) = A(:, q[j]).
 *   - L (m x k) is unit lower trapezoidal with the unit diagonal stored;
 *     U (k x n) is upper trapezoidal with zeros stored below the diagonal.
 *   - All work is enqueued on the caller's stream; rlu_factor returns once the
 *     work is enqueued.  No value is read back to the host on the way.
 *
 * Errors
 *   - Argument errors return a negative status synchronously, before any
 *     device work is enqueued.
 *   - Data-dependent conditions never stop the path: a zero pivot (rank of
 *     the sketch or of B below k) is reported in the device word info[0] (for
 *     Step 3) or info[1] (for Step 6) as the 1-based step where it occurred,
 *     0 meaning none.  The factors stay defined (see the zero-pivot rules in
 *     the documentation of rlu_factor).
 *   - info[2] is a bit set.  Bit 0 (value 1): a device-side failure of the
 *     cross-workgroup pivot exchange (one of its waits did not complete
 *     within its time limit); the outputs are then undefined.  Bit 1 (value
 *     2): with RLU_FLAG_CHECK_FINITE, a NaN or an infinity was found in the
 *     sketch Y = A G, i.e. in A or G (a non-finite entry of either reaches
 *     every entry of its row of Y) or in an overflowed product; the outputs
 *     are then unspecified.  rlu_check_info maps the three words to a status.
 *   - No exception crosses this interface.
 *
 * Threading: a handle may be used by one host thread at a time and serves
 * one stream at a time: its workspace (Y, the Gram matrix, the pivot
 * exchange area, the split-K partials) is reused by every call, and nothing
 * orders calls on different streams, so a caller that switches streams
 * must order the calls itself (or use one handle per stream).  A pivoted
 * LU spread over workgroups needs all of them resident at once (at most one
 * per CU, 128 by default); calls on several streams at once share the CUs,
 * and if their pivoted LUs together leave one without its workgroups, its
 * waits reach their time limit and the call reports the exchange failure
 * (info[2] bit 0) instead of hanging.
 *
 * Environment (tuning and tests; results are the same bits either way):
 *   RLU_PANEL_WG_CAP  16..256, read once per process: the most workgroups
 *                     a pivoted LU spread over workgroups aims at (128).
 *   RLU_PANEL_REGS=0  read at each call: pivoted LUs that fit one
 *                     workgroup's registers use the LDS-resident kernels.
 */
#ifndef RLU_H
#define RLU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RLU_OK = 0,
  RLU_PENDING = 1,
  RLU_WARN_ZERO_PIVOT = 2,
  RLU_ERR_INVALID_ARG = -1,
  RLU_ERR_OUT_OF_MEMORY = -2,
  RLU_ERR_DEVICE = -3,
  RLU_ERR_TOO_LARGE = -4,
  RLU_ERR_QUEUE_FULL = -5,
  RLU_ERR_NONFINITE = -6,
  RLU_ERR_UNKNOWN_TICKET = -7,
  RLU_ERR_UNSUPPORTED = -8
} rlu_status_t;

/* Storage type of A, G, L and U. */
typedef enum { RLU_F64 = 0, RLU_F32 = 1 } rlu_dtype_t;

/* Arithmetic of the two large products (Steps 2 and 5).  The pivoted LUs
 * (Steps 3 and 6), the Gram matrix and its inverse are FP64 in every mode. */
typedef enum {
  RLU_PREC_FP64 = 0,       /* requires RLU_F64 storage                      */
  RLU_PREC_FP32 = 1,       /* requires RLU_F32 storage                      */
  RLU_PREC_MIXED_BF16 = 2, /* RLU_F32 storage; bf16 MFMA, fp32 accumulation */
  RLU_PREC_MIXED_FP16 = 3  /* RLU_F32 storage; fp16 MFMA, fp32 accumulation */
} rlu_precision_t;

enum {
  RLU_FLAG_CHECK_FINITE = 1u, /* scan the sketch for NaN / infinity: info[2]
                                 bit 1, status RLU_ERR_NONFINITE (one pass
                                 over the m x l sketch, no pass over A)   */
  RLU_FLAG_DIAGNOSTICS = 2u,  /* fill the optional diagnostic outputs      */
  RLU_FLAG_RRLU = 4u,         /* Step 3 as Algorithm 4.1 lists it: a
                                 rank-revealing LU P Y Q_y = L_y U_y, Q_y
                                 the column order of a column-pivoted QR of
                                 Y (see rlu_factor); rlu_factor only,
                                 l <= 1024                                  */
  RLU_FLAG_FAST = 8u          /* Algorithm 4.4, fast randomized LU: SRFT
                                 sketch and interpolative decomposition (see
                                 rlu_factor); rlu_factor only, FP64 / FP32,
                                 G = NULL, no power iterations, l <= 1024  */
};

/* Problem description (Algorithm 4.1, Input): A is m x n, k the target rank,
 * l the number of sketch columns.  Requires 1 <= k <= l <= min(m, n). */
typedef struct {
  int64_t m, n, k, l;
  rlu_dtype_t dtype;
  rlu_precision_t precision;
  uint64_t seed;      /* Step 1: G from Philox4x32-10 + Box-Muller, see below */
  const void* G;      /* optional caller G (n x l, storage dtype, device);    */
  int64_t ldg;        /*   NULL => generated from seed                        */
  uint32_t flags;
  int32_t power_iters; /* q of Section 5.2, 0..RLU_MAX_POWER_ITERS: Step 2
                          becomes Y = (A A^T)^q A G, each product but the last
                          replaced by the unit-lower factor of its pivoted LU
                          (same column space; see rlu_factor).  0 = plain
                          Step 2.  In rlu_factor_batched every problem of a
                          call must have the same q (else RLU_ERR_INVALID_ARG);
                          the server runs a request with q != 0 alone. */
} rlu_problem_t;

#define RLU_MAX_POWER_ITERS 16

/* Step 1 generator: key = (seed mod 2^32, seed div 2^32); element (i, j) of G
 * has column-major index e = i + j*n and uses counter (e/2 mod 2^32,
 * e/2 div 2^32, 0, 0); the four output words give u1 = ((x1:x0 >> 11) + 1)
 * 2^-53 and u2 = (x3:x2 >> 11) 2^-53, and the Box-Muller pair
 * sqrt(-2 ln u1) (cos, sin)(2 pi u2) goes to the even and odd e. */

/* Inputs and outputs (Algorithm 4.1, Output), all device pointers. */
typedef struct {
  const void* A; int64_t lda;  /* in  m x n, lda >= m; never modified           */
  void* L; int64_t ldl;        /* out m x k, ldl >= m: unit lower trapezoidal   */
  void* U; int64_t ldu;        /* out k x n, ldu >= k: upper trapezoidal        */
  int64_t* p;                  /* out length m: row permutation P               */
  int64_t* q;                  /* out length n: column permutation Q            */
  int32_t* info;               /* out 3 words: zero-pivot step of Step 3, of
                                  Step 6 (1-based, 0 = none), failure bits
                                  (1: exchange, 2: non-finite input)         */
  /* Optional diagnostics, filled only with RLU_FLAG_DIAGNOSTICS (each may be
   * NULL).  Y and B use the storage dtype of the FP64/FP32 path (FP64 for the
   * FP64 and mixed modes, FP32 for the FP32 mode). */
  void* Y; int64_t ldy;        /* out m x l: the sketch A G (before Step 3)     */
  void* B; int64_t ldb;        /* out k x n: B = L_y^+ P A (before Step 6)      */
  int32_t* ipiv;               /* out length l: Step 3 swap sequence (LAPACK)   */
  int32_t* qpiv;               /* out length k: Step 6 swap sequence            */
  int32_t* qy;                 /* out length l: Step 3 column order Q_y, with
                                  RLU_FLAG_RRLU ((Y Q_y)(:, j) = Y(:, qy[j]))  */
} rlu_buffers_t;

typedef struct rlu_handle_s* rlu_handle_t;
typedef void* rlu_stream_t; /* a hipStream_t; NULL = the null stream */

/* Create a handle bound to HIP device `device` (the handle caches device
 * workspace, and for rlu_factor_batched a capture stream and the recorded
 * launch graph). */
rlu_status_t rlu_create(rlu_handle_t* h, int device);
rlu_status_t rlu_destroy(rlu_handle_t h);

/* Device workspace rlu_factor needs for this problem, in bytes (the handle
 * allocates and caches it; the figure is what it will hold). */
rlu_status_t rlu_workspace_size(const rlu_problem_t* pb, size_t* bytes);

/* Algorithm 4.1, Steps 1-8, enqueued on `stream`.
 *
 * Power iterations (Section 5.2, pb->power_iters = q > 0): Step 2 computes
 * A G and then q times one product with A^T and one with A.  Before each
 * product after the first, the current block (m x l or n x l) is replaced
 * by the unit-lower factor of its partial-pivot LU in its own row order
 * (P^T L = X U^{-1}), so the entries stay bounded by 1; in exact arithmetic
 * this changes neither the pivots nor the factors of Steps 3-8 relative to
 * the plain (A A^T)^q A G.  A zero pivot inside such a normalization is not
 * reported (Step 3 reports the rank of the final sketch).  The optional
 * diagnostic Y is the final sketch.
 *
 * Rank-revealing Step 3 (pb->flags & RLU_FLAG_RRLU, Algorithm 4.1 as listed
 * with the RRLU of Section 3.1): the sketch's columns are first put in the
 * order Q_y of a column-pivoted QR of Y (Businger-Golub: at each step the
 * remaining column with the largest norm orthogonal to those chosen, lowest
 * current position on ties), computed as a pivoted Cholesky of the Gram
 * matrix Y^T Y (the same order in exact arithmetic); then P (Y Q_y) =
 * L_y U_y by partial pivoting, and Steps 4-8 as usual.  With partial
 * pivoting alone only the first k sketch columns reach the result; here
 * the k columns of the l that the column-pivoted QR ranks first do.
 * Requires l <= 1024; rlu_factor_batched and the server reject the flag
 * (RLU_ERR_UNSUPPORTED).
 *
 * Fast randomized LU (pb->flags & RLU_FLAG_FAST, Section 4.5, Algorithm
 * 4.4): Step 1 draws the SRFT R = D F S (Section 3.3) from pb->seed instead
 * of G -- F the orthonormal discrete Hartley transform (real, so a real A
 * keeps real factors), D = diag(+1 / -1), S l distinct columns in a random
 * order; the draws use the Philox4x32-10 key of Step 1 with counters
 * (i div 128, 0, 1, 0) for the sign of row i (bit i mod 128 of the four
 * words, bit 0 = +1) and (j, 0, 2, 0) for step j of a partial Fisher-Yates
 * shuffle of 0..n-1 that exchanges positions j and j + ((x1:x0) mod (n-j)).
 * Y = A R; Step 3 as above (partial pivoting, or RRLU with RLU_FLAG_RRLU);
 * the full-rank ID Y = X Y(J, :) comes from Step 3's LU (J = the l rows its
 * steps chose, X = Y Y(J, :)^{-1}); B = L_y^+ P X A(J, :), which reads only
 * the l rows J of A; Steps 7-9 as in Algorithm 4.1.  With diagnostics, Y is
 * A R and B this B.
 *
 * Zero pivots: in Step 3 the LAPACK getf2 convention holds (no scaling, no
 * update, info[0] = first such step); in Step 6, column j of L_b below the
 * diagonal is zero and row j of U_b is zero (info[1] = first such step).
 * Ties in a pivot search go to the lowest current position. */
rlu_status_t rlu_factor(rlu_handle_t h, const rlu_problem_t* pb,
                        const rlu_buffers_t* io, rlu_stream_t stream);

/* rlu_factor for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same launch sequence and results as rlu_factor, with its workspace in a
 * fixed device scratch array of RLU_NOALLOC_SCRATCH_BYTES that the library
 * holds on every device it runs on until the process ends (located once per
 * device by rlu_create).  The call allocates nothing and leaves the handle's
 * own workspace alone; phase timing does not apply.  Problems whose
 * workspace (rlu_workspace_size) exceeds the scratch return
 * RLU_ERR_TOO_LARGE before any device work (8192 x 8192 with k = 200, l =
 * 210 fits; 16384 x 16384 with k = 500 does not).  Every call on a device
 * shares that device's scratch, which keeps the last call's contents (each
 * call clears what must start at zero): calls that overlap on one device,
 * from any handle, thread or stream, race and give undefined results, so
 * order them (one stream, or events).  RLU_ERR_DEVICE if the scratch could
 * not be located on the handle's device. */
#define RLU_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
rlu_status_t rlu_factor_noalloc(rlu_handle_t h, const rlu_problem_t* pb,
                                const rlu_buffers_t* io, rlu_stream_t stream);

/* Many independent problems (Algorithm 4.1 for each), enqueued on `stream`
 * as one launch per kernel of the method for the whole batch.
 *
 * pbs[i] and ios[i] describe problem i exactly as for rlu_factor; shapes may
 * all differ, but every problem must use the same dtype and precision, and
 * RLU_FLAG_DIAGNOSTICS is not available here (RLU_ERR_INVALID_ARG).  Each
 * problem's results are those rlu_factor defines for it (same pivot rules;
 * products may round differently because tile shapes and K splits differ).
 * The handle owns a separate batch workspace.  The launch sequence is
 * recorded once as a HIP graph and replayed for later calls with identical
 * arrays (same problems, same buffers); phase timing, when enabled, runs it
 * without the graph.  RLU_ERR_UNSUPPORTED if a panel (l or k columns) is too
 * wide for the batched pivoted LU or a problem needs more workgroups than
 * the device holds at once.  count = 0 is a no-op. */
rlu_status_t rlu_factor_batched(rlu_handle_t h, int32_t count, const rlu_problem_t* pbs,
                                const rlu_buffers_t* ios, rlu_stream_t stream);

/* Rank-deficient least squares on the factors (Section 4.4, Algorithm 4.3):
 * for P A Q ~ L U from rlu_factor (same m, n, k, dtype), minimize
 * ||A x - b|| for each column of b by
 *   Step 2  y   <- L^+ P b        (Gram route, as Step 5: (L^T L)^{-1} L^T,
 *                                  with P folded into the rows of L)
 *   Step 3  z_1 <- U_1^{-1} y     (U_1 = the leading k x k block of U)
 *   Step 4  z   <- (z_1; 0)       (z_2 = 0: x has at most k nonzeros)
 *   Step 5  x   <- Q z            (x[q[j]] = z[j])
 * Arithmetic is FP64 for both storage types.  A zero diagonal entry of U_1
 * (a zero pivot of Step 6, whose row of U is zero) leaves its unknown 0.
 * All pointers are device pointers on the handle's device; L, U, p, q and b
 * are read only, x is written (n x nrhs).  p and q must be the permutations
 * rlu_factor returned: entries outside [0, m) or [0, n) are skipped (no
 * out-of-range access) and the result is then undefined.  Requires
 * 1 <= k <= min(m, n), k <= 1024, nrhs >= 0 (0: no-op), ldl >= m,
 * ldu >= k, ldb >= m, ldx >= n; otherwise RLU_ERR_INVALID_ARG (k > 1024:
 * RLU_ERR_UNSUPPORTED) before any device work.  Uses the handle's workspace,
 * so calls on one handle are ordered like rlu_factor calls. */
typedef struct {
  int64_t m, n, k;
  rlu_dtype_t dtype;           /* storage of L, U, b and x                   */
  const void* L; int64_t ldl;  /* m x k, unit lower trapezoidal (rlu_factor) */
  const void* U; int64_t ldu;  /* k x n, upper trapezoidal                   */
  const int64_t* p;            /* length m: (P A)(i, :) = A(p[i], :)        */
  const int64_t* q;            /* length n: (A Q)(:, j) = A(:, q[j])        */
  int64_t nrhs;
  const void* b; int64_t ldb;  /* m x nrhs                                   */
  void* x; int64_t ldx;        /* out n x nrhs                               */
} rlu_lstsq_t;

/* Device workspace rlu_lstsq needs for this problem, in bytes. */
rlu_status_t rlu_lstsq_workspace_size(const rlu_lstsq_t* ls, size_t* bytes);
rlu_status_t rlu_lstsq(rlu_handle_t h, const rlu_lstsq_t* ls, rlu_stream_t stream);

/* Tile shapes of the grouped products of rlu_factor_batched, for tuning
 * tools.  product: 0 sketch (Step 2), 1 Gram matrix, 2 projection (Step 5),
 * 3 S^{-1} C, 4 L = Lv L_b (Step 7).  cfg: an index for which rlu_tile_name
 * returns a name ("BMxBNxBK"), or -1 for the library's tuned table.  The
 * setting applies to later calls on this handle. */
rlu_status_t rlu_set_tile(rlu_handle_t h, int32_t product, int32_t cfg);
const char* rlu_tile_name(int32_t cfg);  /* NULL if cfg is not a grouped tile */

/* ------------------------------------------------------------------------
 * Serving: a request loop with continuous batching.
 *
 * A server owns one scheduler thread, two streams and a handle on `device`.
 * Submitted requests wait in a FIFO queue; the scheduler admits them in
 * order while the HBM footprint of every admitted, unreleased request stays
 * within hbm_budget_bytes (a request that alone exceeds the budget is
 * rejected at submit with RLU_ERR_TOO_LARGE), and launches all admitted
 * requests of the head's dtype and precision as one batch (the kernels of
 * rlu_factor_batched) on a free stream.  Requests that arrive while batches
 * run are admitted as memory frees up and overlap with them on the device.
 * Each request's factors are those rlu_factor_batched gives for it alone.
 * Footprint = the request's share of a batch workspace (freed when its batch
 * completes) + its outputs L, U, p, q, info (held until rlu_serve_release).
 * ---------------------------------------------------------------------- */
typedef struct rlu_server_s* rlu_server_t;

typedef struct {
  int device;
  size_t hbm_budget_bytes; /* 0: 90% of the device memory free at creation   */
  int32_t max_inflight;    /* admitted, unfinished requests; 0 = no limit     */
  int32_t max_queue;       /* queued requests; 0 = no limit                   */
} rlu_server_config_t;

typedef struct {
  rlu_status_t status;     /* RLU_PENDING, RLU_OK, RLU_WARN_ZERO_PIVOT, or an
                              error (RLU_ERR_DEVICE: exchange failure;
                              RLU_ERR_NONFINITE: the requested check found a
                              NaN or infinity)                                 */
  const void* L; int64_t ldl;  /* server-owned device outputs, valid until    */
  const void* U; int64_t ldu;  /*   rlu_serve_release (NULL unless finished)  */
  const int64_t* p;
  const int64_t* q;
  int32_t info[3];             /* the rlu_factor info words                   */
  double t_submit_us, t_start_us, t_done_us;  /* server clock: submitted,
                              launched in a batch, completion observed        */
} rlu_result_t;

rlu_status_t rlu_serve_create(const rlu_server_config_t* cfg, rlu_server_t* srv);

/* Queue Algorithm 4.1 for the device matrix A (m x n, lda >= m; it must stay
 * valid and unmodified until the request finishes).  pb->G must be NULL or a
 * device matrix that stays valid likewise; RLU_FLAG_DIAGNOSTICS is not
 * available.  Errors: argument errors, RLU_ERR_UNSUPPORTED (a shape the
 * batched kernels cannot run), RLU_ERR_TOO_LARGE (footprint above the
 * budget), RLU_ERR_QUEUE_FULL.  Thread-safe. */
rlu_status_t rlu_serve_submit(rlu_server_t srv, const rlu_problem_t* pb, const void* A,
                              int64_t lda, uint64_t* ticket);

/* Non-blocking.  Returns the request's status (RLU_PENDING while queued or
 * running) and, if out is not NULL, fills it.  RLU_ERR_UNKNOWN_TICKET for a
 * ticket never issued or already released.  Thread-safe. */
rlu_status_t rlu_serve_poll(rlu_server_t srv, uint64_t ticket, rlu_result_t* out);

/* Copy a finished request's L, U, p, q (and info if dst->info is not NULL)
 * into the caller's device buffers on `stream` (leading dimensions from
 * dst).  RLU_PENDING if not finished.  Synchronize the stream before
 * releasing the ticket. */
rlu_status_t rlu_serve_copy(rlu_server_t srv, uint64_t ticket, const rlu_buffers_t* dst,
                            rlu_stream_t stream);

/* Free a finished request's outputs and forget the ticket (RLU_PENDING if
 * it has not finished; nothing is released then). */
rlu_status_t rlu_serve_release(rlu_server_t srv, uint64_t ticket);

/* HBM footprint the server charges for this request, in bytes (no device
 * needed). */
rlu_status_t rlu_serve_footprint(const rlu_problem_t* pb, size_t* bytes);

/* Bytes admitted and unreleased, queued and admitted-unfinished requests. */
rlu_status_t rlu_serve_stats(rlu_server_t srv, size_t* used_bytes, int32_t* queued,
                             int32_t* inflight);

/* Finish every queued and running request, then free everything (tickets
 * not released are freed too). */
rlu_status_t rlu_serve_destroy(rlu_server_t srv);

/* Phase timing for measurement tools.  enable = 1: rlu_factor records a HIP
 * event pair around each phase on the stream that runs the phase (the
 * caller's stream);
 * enable = 2: around the sketch product (Step 2) only, so that timing the
 * dominant product adds one event pair per call;
 * enable = 3: around the sketch product and around every launch of the
 * pivoted-LU kernel (Steps 3 and 6, their column blocks and the power
 * iterations' normalizations; the first RLU_MAX_KERNEL_TIMES launches of a
 * call); 0: off.  The handle keeps the events of the last RLU_TIMING_RING
 * calls.  Other values: RLU_ERR_INVALID_ARG. */
#define RLU_TIMING_RING 64
#define RLU_MAX_PHASES 16
#define RLU_MAX_KERNEL_TIMES 16
rlu_status_t rlu_set_timing(rlu_handle_t h, int enable);

/* Durations (milliseconds) of the phases of the call `back` calls before the
 * most recent one (back = 0: the most recent), waiting for its events.
 * Fills up to `cap` entries of ms[] and names[] (static strings; either may
 * be NULL) and stores the entry count in *count: the phases (fewer than
 * RLU_MAX_PHASES; untimed phases read 0), then, in timing mode 3, one entry
 * named "panel_lu_kernel" per timed pivoted-LU kernel launch, in launch
 * order (so cap = RLU_MAX_PHASES + RLU_MAX_KERNEL_TIMES always suffices).
 * RLU_ERR_INVALID_ARG if no timed call is that far back. */
rlu_status_t rlu_phase_times(rlu_handle_t h, int back, float* ms, const char** names, int cap,
                             int* count);

/* Map the three info words (already copied to the host) to a status:
 * RLU_ERR_DEVICE if the exchange failed (info[2] bit 0, or any bit this
 * version does not define), RLU_ERR_NONFINITE if the requested non-finite
 * check found a NaN or infinity (bit 1), RLU_WARN_ZERO_PIVOT if a zero pivot
 * occurred, RLU_OK otherwise. */
rlu_status_t rlu_check_info(const int32_t info_host[3]);

/* For tests of the failure path of the pivot exchange (callers that want to
 * see RLU_ERR_DEVICE produced without a faulty device).  timeout_ticks bounds
 * each wait of the exchange, in ticks of the 100 MHz device clock, counted
 * from the wait's first unsuccessful poll (< 0: the library default, 2 s;
 * 0: a wait gives up at its second unsuccessful poll).  preset_failure = 1
 * makes later rlu_factor calls start as if a partner workgroup had already
 * given up: every wait that does not succeed at once ends, every kernel
 * exits normally and info[2] bit 0 is set.  Applies to later calls on this
 * handle (the timeout also to rlu_factor_batched; preset_failure only to
 * rlu_factor).  RLU_ERR_INVALID_ARG for preset_failure outside {0, 1}. */
rlu_status_t rlu_set_exchange_limit(rlu_handle_t h, int64_t timeout_ticks, int preset_failure);

const char* rlu_status_string(rlu_status_t st);

/* Library version string. */
const char* rlu_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RLU_H */
