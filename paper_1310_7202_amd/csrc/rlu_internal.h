// Host-side state shared by the translation units of the C ABI (rlu_api.cpp,
// rlu_batch.cpp): the handle, argument validation, workspace and timing
// helpers.
#pragma once

#include "../../include/rlu.h"
#include "rlu_kernels.h"

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

// Phases of rlu_factor / rlu_factor_batched that the timing facility reports.
enum Phase {
  PH_GAUSSIAN = 0, PH_SKETCH, PH_PANEL_Y, PH_GRAM, PH_GRAM_INV, PH_PROJECT, PH_SOLVE,
  PH_PANEL_B, PH_ASSEMBLE, PH_FORM_L, PH_SKETCH_SUM, PH_PROJECT_SUM, PH_POWER, PH_COLPIV,
  PH_ID_SOLVE, PH_COUNT
};

// Timing mode 3 also times every launch of the pivoted-LU kernel of a call
// (up to kMaxKernelTimes of them; later launches are not timed).
constexpr int kMaxKernelTimes = 16;

struct TimingSlot {
  hipEvent_t ev[PH_COUNT][2] = {};
  bool used[PH_COUNT] = {};
  hipEvent_t kev[kMaxKernelTimes][2] = {};
  int nk = 0;
  bool valid = false;
};

// The launch sequence of one batch, captured once and replayed while the
// same problems and buffers come back.
struct BatchGraph {
  std::vector<char> sig;       // problems, buffers and workspace base it was built for
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct rlu_handle_s {
  int device = 0;
  bool timing = false;
  int timing_mode = 0;      // 1: every phase, 2: the sketch product only, 3: the
                            // sketch product and every pivoted-LU kernel launch
  int ring_next = 0;        // next slot to fill
  int ring_filled = 0;      // number of valid slots
  TimingSlot ring[RLU_TIMING_RING];
  TimingSlot* cur = nullptr;
  int cus = 256;
  void* ws = nullptr;            // workspace of rlu_factor
  size_t ws_bytes = 0;
  // rlu_factor_batched
  void* bws = nullptr;           // batch workspace (data, exchange areas, task tables)
  size_t bws_bytes = 0;
  void* stage = nullptr;         // pinned staging of the task tables
  size_t stage_bytes = 0;
  hipEvent_t ev_stage = nullptr; // last upload from `stage` done
  hipStream_t cap = nullptr;     // capture stream
  hipEvent_t ev_panel = nullptr; // last batched panel launch (eager calls)
  BatchGraph bgraph;
  int tile_override[5] = {-1, -1, -1, -1, -1};  // rlu_set_tile
  long long xch_timeout = 200LL * 1000 * 1000;  // bound on each exchange wait (ticks)
  bool xch_preset_fail = false;                 // rlu_set_exchange_limit
};

namespace rlu_detail {

constexpr long long kTimeoutTicks = 200LL * 1000 * 1000;  // 2 s of the 100 MHz clock

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

template <typename P>
P* at(void* base, size_t off) { return (P*)((char*)base + off); }

#define HIP_TRY(expr)                                                                \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      if (getenv("RLU_LOG"))                                                         \
        fprintf(stderr, "librlu: %s failed: %s\n", #expr, hipGetErrorString(e_));    \
      return RLU_ERR_DEVICE;                                                         \
    }                                                                                \
  } while (0)

rlu_status_t validate(const rlu_problem_t* pb);
rlu_status_t validate_io(const rlu_problem_t* pb, const rlu_buffers_t* io);
rlu_status_t begin_timing(rlu_handle_s* h);

// Batched path (rlu_batch.cpp), also used by the server.
rlu_status_t batched_validate(int count, const rlu_problem_t* pbs, const rlu_buffers_t* ios);
rlu_status_t batched_item_bytes(const rlu_problem_t& pb, int cus, size_t* bytes);
rlu_status_t batched_ws_bytes(int count, const rlu_problem_t* pbs, const rlu_buffers_t* ios,
                              int cus, size_t* bytes);
rlu_status_t batched_enqueue_ws(rlu_handle_s* h, int count, const rlu_problem_t* pbs,
                                const rlu_buffers_t* ios, hipStream_t s, void* ws,
                                size_t ws_bytes, hipEvent_t gate);

// Event pair around a phase when timing is on (recorded on the phase's
// stream); id < 0 records nothing.
struct PhaseScope {
  rlu_handle_s* h; int id; hipStream_t s; bool on;
  PhaseScope(rlu_handle_s* h_, int id_, hipStream_t s_)
      : h(h_), id(id_), s(s_),
        on(id_ >= 0 && h_->timing && h_->cur && (h_->timing_mode == 1 || id_ == PH_SKETCH)) {
    if (on) {
      h->cur->used[id] = true;
      hipEventRecord(h->cur->ev[id][0], s);
    }
  }
  ~PhaseScope() {
    if (on) hipEventRecord(h->cur->ev[id][1], s);
  }
};

// Event pair around one launch of the pivoted-LU kernel (timing mode 3).
struct KernelScope {
  rlu_handle_s* h; hipStream_t s; int idx;
  KernelScope(rlu_handle_s* h_, hipStream_t s_) : h(h_), s(s_), idx(-1) {
    if (h && h->timing && h->timing_mode == 3 && h->cur && h->cur->nk < kMaxKernelTimes) {
      idx = h->cur->nk++;
      hipEventRecord(h->cur->kev[idx][0], s);
    }
  }
  ~KernelScope() {
    if (idx >= 0) hipEventRecord(h->cur->kev[idx][1], s);
  }
};

// Scoped switch to the handle's device.
struct DeviceScope {
  int prev = 0; int dev; bool ok = true;
  explicit DeviceScope(int d) : dev(d) {
    hipGetDevice(&prev);
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceScope() {
    if (prev != dev) hipSetDevice(prev);
  }
};

}  // namespace rlu_detail
