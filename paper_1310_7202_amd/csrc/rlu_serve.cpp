// Serving form of Algorithm 4.1 (Shabat et al., Section 4): a request loop
// with continuous batching.
//
//   * rlu_serve_submit validates a request, computes its HBM footprint (its
//     share of a batch workspace plus the outputs the server keeps for it)
//     and queues it; a request larger than the whole budget is rejected.
//   * One scheduler thread admits queued requests strictly in FIFO order
//     while the footprint of everything admitted and not yet released stays
//     within the budget, and launches every admitted request of the head's
//     precision as one batch (rlu_batch.cpp kernels) on whichever of the
//     server's streams is free.  Batches on different streams overlap on
//     the device; their pivoted-LU launches are ordered by one gate event,
//     since each of those keeps every workgroup of the device busy.
//   * When a batch's completion event fires, its requests become done (info
//     words were copied to pinned host memory by the same stream) and its
//     workspace is returned to the stream-ordered allocator; outputs stay
//     until rlu_serve_release.
// Each problem's results depend only on that problem: tile shapes and splits
// are chosen per problem and the pivoted LU gives the same bits for any
// number of rows per workgroup, so a request's factors are the same alone
// and in any mix.
#include "rlu_internal.h"
#include "serve_policy.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace rlu_detail;

namespace {

enum ReqState { Q_QUEUED = 0, Q_RUNNING = 1, Q_DONE = 2, Q_FAILED = 3 };

struct Req {
  uint64_t ticket = 0;
  rlu_problem_t pb{};
  const void* A = nullptr;
  int64_t lda = 0;
  size_t ws_bytes = 0, out_bytes = 0;
  void* out = nullptr;  // L | U | p | q | info (device)
  size_t offU = 0, offp = 0, offq = 0, offinfo = 0;
  int state = Q_QUEUED;
  rlu_status_t status = RLU_PENDING;
  int32_t info[3] = {0, 0, 0};
  double t_submit = 0, t_start = 0, t_done = 0;
  bool solo = false;    // too large for the batched kernels: runs alone (rlu_factor)
};

struct Flight {
  std::vector<Req*> reqs;
  int stream = -1;
  void* ws = nullptr;
  bool recorded = false;           // completion event recorded
  rlu_status_t launch_status = RLU_OK;
};

size_t elem_size(const rlu_problem_t& pb) { return pb.dtype == RLU_F32 ? 4 : 8; }

// Outputs the server holds for a request: L (m x k), U (k x n), p, q, info.
size_t output_layout(const rlu_problem_t& pb, size_t* offU, size_t* offp, size_t* offq,
                     size_t* offinfo) {
  const size_t s = elem_size(pb);
  size_t off = align_up((size_t)pb.m * pb.k * s);
  *offU = off;
  off = align_up(off + (size_t)pb.k * pb.n * s);
  *offp = off;
  off = align_up(off + (size_t)pb.m * 8);
  *offq = off;
  off = align_up(off + (size_t)pb.n * 8);
  *offinfo = off;
  return align_up(off + 16);
}

// Workspace a request needs: its share of a batch, or, for a shape the
// batched kernels cannot run or a request with power iterations, the
// single-problem workspace (it then runs alone through rlu_factor).

// Argument checks of a request: those of the batched form for the request
// on its own (a request with power iterations runs alone).
rlu_status_t request_validate(const rlu_problem_t* pb) {
  if (!pb) return RLU_ERR_INVALID_ARG;
  rlu_status_t st = validate(pb);
  if (st != RLU_OK) return st;
  rlu_problem_t v = *pb;
  v.power_iters = 0;
  return batched_validate(1, &v, nullptr);
}

rlu_status_t request_ws_bytes(const rlu_problem_t& pb, int cus, size_t* bytes, bool* solo) {
  *solo = false;
  // a request with power iterations (Section 5.2) runs alone, so that the
  // batches the server forms keep one q
  rlu_status_t st = pb.power_iters != 0 ? RLU_ERR_UNSUPPORTED : batched_item_bytes(pb, cus, bytes);
  if (st != RLU_ERR_UNSUPPORTED) return st;
  st = rlu_workspace_size(&pb, bytes);
  if (st == RLU_OK) *solo = true;
  return st;
}

double now_us(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct rlu_server_s {
  rlu_server_config_t cfg{};
  rlu_handle_s* h = nullptr;                 // batched launches (task-table staging)
  std::vector<rlu_handle_s*> solo_h;          // per stream: requests that run alone
  std::vector<hipStream_t> streams;
  std::vector<bool> busy;
  std::vector<hipEvent_t> done;      // per stream: completion of its batch
  std::vector<int32_t*> info_host;   // per stream: pinned info words of its batch
  hipEvent_t gate = nullptr;
  std::chrono::steady_clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv;
  rlu_serve::Policy policy{0, 0, 0};  // queue, budget and in-flight accounting
  std::unordered_map<uint64_t, Req*> reqs;
  std::vector<Flight> flights;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread thr;

  void loop();
  bool launch_one(std::unique_lock<std::mutex>& lk);
  bool reap(std::unique_lock<std::mutex>& lk);
};

namespace {

constexpr int kStreams = 2;
constexpr int kMaxBatch = 256;

}  // namespace

// Complete finished batches.  Called with the lock held.
bool rlu_server_s::reap(std::unique_lock<std::mutex>&) {
  bool any = false;
  for (size_t i = 0; i < flights.size();) {
    Flight& f = flights[i];
    const hipError_t q = f.recorded ? hipEventQuery(done[f.stream]) : hipSuccess;
    if (q == hipErrorNotReady) { ++i; continue; }
    const double t = now_us(t0);
    for (size_t r = 0; r < f.reqs.size(); ++r) {
      Req* rq = f.reqs[r];
      rq->t_done = t;
      if (f.launch_status != RLU_OK || q != hipSuccess) {
        rq->state = Q_FAILED;
        rq->status = f.launch_status != RLU_OK ? f.launch_status : RLU_ERR_DEVICE;
      } else {
        std::memcpy(rq->info, info_host[f.stream] + 3 * r, sizeof(rq->info));
        rq->state = Q_DONE;
        rq->status = rlu_check_info(rq->info);
      }
      policy.complete(rq->ws_bytes);
      rq->ws_bytes = 0;
    }
    if (f.ws) hipFreeAsync(f.ws, streams[f.stream]);
    busy[f.stream] = false;
    flights.erase(flights.begin() + i);
    any = true;
  }
  if (any) cv.notify_all();
  return any;
}

// Admit from the head of the queue and launch one batch on a free stream.
// Called with the lock held; drops it around the device calls.
bool rlu_server_s::launch_one(std::unique_lock<std::mutex>& lk) {
  int sidx = -1;
  for (int i = 0; i < (int)streams.size(); ++i)
    if (!busy[i]) { sidx = i; break; }
  if (sidx < 0 || policy.queued() == 0) return false;
  // strict FIFO from the head (serve_policy.h)
  std::vector<Req*> batch;
  for (const rlu_serve::Entry& e : policy.admit(kMaxBatch)) {
    auto it = reqs.find(e.ticket);  // a queued request cannot be released
    if (it == reqs.end()) continue;
    it->second->state = Q_RUNNING;
    batch.push_back(it->second);
  }
  if (batch.empty()) return false;
  const bool solo = batch.front()->solo;
  busy[sidx] = true;
  const double t = now_us(t0);
  for (Req* r : batch) r->t_start = t;
  lk.unlock();

  Flight f;
  f.reqs = batch;
  f.stream = sidx;
  hipStream_t s = streams[sidx];
  const int n = (int)batch.size();
  std::vector<rlu_problem_t> pbs(n);
  std::vector<rlu_buffers_t> ios(n);
  rlu_status_t st = RLU_OK;
  for (int i = 0; i < n && st == RLU_OK; ++i) {
    Req* r = batch[i];
    if (!r->out && hipMallocAsync(&r->out, r->out_bytes, s) != hipSuccess) {
      r->out = nullptr;
      st = RLU_ERR_OUT_OF_MEMORY;
      break;
    }
    pbs[i] = r->pb;
    rlu_buffers_t& io = ios[i];
    io = rlu_buffers_t{};
    io.A = r->A; io.lda = r->lda;
    io.L = r->out; io.ldl = r->pb.m;
    io.U = (char*)r->out + r->offU; io.ldu = r->pb.k;
    io.p = (int64_t*)((char*)r->out + r->offp);
    io.q = (int64_t*)((char*)r->out + r->offq);
    io.info = (int32_t*)((char*)r->out + r->offinfo);
  }
  if (solo) {
    // the single-problem path keeps every workgroup busy in its pivoted LUs
    // (persistent launches that need all their workgroups resident): order
    // it after the last panel launch and make the next one wait for all of it
    if (st == RLU_OK && hipStreamWaitEvent(s, gate, 0) != hipSuccess) st = RLU_ERR_DEVICE;
    if (st == RLU_OK) st = rlu_factor(solo_h[sidx], &pbs[0], &ios[0], s);
    if (st == RLU_OK && hipEventRecord(gate, s) != hipSuccess) st = RLU_ERR_DEVICE;
  } else {
    size_t wsb = 0;
    if (st == RLU_OK) st = batched_ws_bytes(n, pbs.data(), ios.data(), h->cus, &wsb);
    if (st == RLU_OK && hipMallocAsync(&f.ws, wsb, s) != hipSuccess) {
      f.ws = nullptr;
      st = RLU_ERR_OUT_OF_MEMORY;
    }
    if (st == RLU_OK) st = batched_enqueue_ws(h, n, pbs.data(), ios.data(), s, f.ws, wsb, gate);
  }
  for (int i = 0; i < n && st == RLU_OK; ++i)
    if (hipMemcpyAsync(info_host[sidx] + 3 * i, ios[i].info, 12, hipMemcpyDeviceToHost, s) !=
        hipSuccess)
      st = RLU_ERR_DEVICE;
  if (hipEventRecord(done[sidx], s) == hipSuccess) f.recorded = true;
  else hipStreamSynchronize(s);  // nothing to wait on: drain before reaping it as failed
  f.launch_status = st;
  lk.lock();
  flights.push_back(f);
  return true;
}

void rlu_server_s::loop() {
  hipSetDevice(cfg.device);
  std::unique_lock<std::mutex> lk(mu);
  while (true) {
    bool progress = reap(lk);
    while (launch_one(lk)) progress = true;
    if (stop && policy.queued() == 0 && flights.empty()) break;
    if (!progress) {
      if (flights.empty())
        cv.wait_for(lk, std::chrono::milliseconds(5));
      else
        cv.wait_for(lk, std::chrono::microseconds(20));  // poll completion events
    }
  }
}

extern "C" {

rlu_status_t rlu_serve_footprint(const rlu_problem_t* pb, size_t* bytes) {
  if (!pb || !bytes) return RLU_ERR_INVALID_ARG;
  rlu_status_t st = request_validate(pb);
  if (st != RLU_OK) return st;
  size_t ws = 0, oU, op, oq, oi;
  bool solo = false;
  st = request_ws_bytes(*pb, 256, &ws, &solo);
  if (st != RLU_OK) return st;
  *bytes = ws + output_layout(*pb, &oU, &op, &oq, &oi);
  return RLU_OK;
}

rlu_status_t rlu_serve_create(const rlu_server_config_t* cfg, rlu_server_t* out) {
  if (!cfg || !out) return RLU_ERR_INVALID_ARG;
  *out = nullptr;
  if (cfg->max_inflight < 0 || cfg->max_queue < 0) return RLU_ERR_INVALID_ARG;
  rlu_server_s* srv = new (std::nothrow) rlu_server_s();
  if (!srv) return RLU_ERR_OUT_OF_MEMORY;
  srv->cfg = *cfg;
  auto fail = [srv](rlu_status_t st) {
    for (hipEvent_t x : srv->done) hipEventDestroy(x);
    for (int32_t* x : srv->info_host) hipHostFree(x);
    for (hipStream_t x : srv->streams) hipStreamDestroy(x);
    for (rlu_handle_s* x : srv->solo_h) rlu_destroy(x);
    if (srv->gate) hipEventDestroy(srv->gate);
    if (srv->h) rlu_destroy(srv->h);
    delete srv;
    return st;
  };
  rlu_status_t st = rlu_create(&srv->h, cfg->device);
  if (st != RLU_OK) { srv->h = nullptr; return fail(st); }
  DeviceScope dev(cfg->device);
  if (srv->cfg.hbm_budget_bytes == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return fail(RLU_ERR_DEVICE);
    srv->cfg.hbm_budget_bytes = fr / 10 * 9;
  }
  srv->policy = rlu_serve::Policy(srv->cfg.hbm_budget_bytes, srv->cfg.max_inflight,
                                  srv->cfg.max_queue);
  for (int i = 0; i < kStreams; ++i) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return fail(RLU_ERR_DEVICE);
    srv->streams.push_back(s);
    srv->busy.push_back(false);
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return fail(RLU_ERR_DEVICE);
    srv->done.push_back(e);
    int32_t* ih = nullptr;
    if (hipHostMalloc((void**)&ih, 12 * (size_t)kMaxBatch, hipHostMallocDefault) != hipSuccess)
      return fail(RLU_ERR_OUT_OF_MEMORY);
    srv->info_host.push_back(ih);
    rlu_handle_s* hs = nullptr;
    st = rlu_create(&hs, cfg->device);
    if (st != RLU_OK) return fail(st);
    srv->solo_h.push_back(hs);
  }
  if (hipEventCreateWithFlags(&srv->gate, hipEventDisableTiming) != hipSuccess)
    return fail(RLU_ERR_DEVICE);
  srv->t0 = std::chrono::steady_clock::now();
  srv->thr = std::thread([srv]() { srv->loop(); });
  *out = srv;
  return RLU_OK;
}

rlu_status_t rlu_serve_submit(rlu_server_t srv, const rlu_problem_t* pb, const void* A,
                              int64_t lda, uint64_t* ticket) {
  if (!srv || !pb || !A || !ticket) return RLU_ERR_INVALID_ARG;
  if (lda < pb->m) return RLU_ERR_INVALID_ARG;
  rlu_status_t st = request_validate(pb);
  if (st != RLU_OK) return st;
  Req* r = new (std::nothrow) Req();
  if (!r) return RLU_ERR_OUT_OF_MEMORY;
  r->pb = *pb;
  r->A = A;
  r->lda = lda;
  st = request_ws_bytes(*pb, srv->h->cus, &r->ws_bytes, &r->solo);
  if (st != RLU_OK) { delete r; return st; }
  r->out_bytes = output_layout(*pb, &r->offU, &r->offp, &r->offq, &r->offinfo);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) { delete r; return RLU_ERR_INVALID_ARG; }
    const rlu_serve::Verdict v = srv->policy.offer(r->ws_bytes, r->out_bytes);
    if (v != rlu_serve::Verdict::Accept) {
      delete r;
      return v == rlu_serve::Verdict::TooLarge ? RLU_ERR_TOO_LARGE : RLU_ERR_QUEUE_FULL;
    }
    r->ticket = srv->next_ticket++;
    r->t_submit = now_us(srv->t0);
    rlu_serve::Entry e;
    e.ticket = r->ticket;
    e.ws = r->ws_bytes;
    e.out = r->out_bytes;
    e.key = (int)r->pb.dtype * 16 + (int)r->pb.precision;
    e.solo = r->solo;
    srv->policy.push(e);
    srv->reqs[r->ticket] = r;
    *ticket = r->ticket;
  }
  srv->cv.notify_all();
  return RLU_OK;
}

rlu_status_t rlu_serve_poll(rlu_server_t srv, uint64_t ticket, rlu_result_t* out) {
  if (!srv) return RLU_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return RLU_ERR_UNKNOWN_TICKET;
  Req* r = it->second;
  if (r->state == Q_QUEUED || r->state == Q_RUNNING) {
    if (out) {
      std::memset(out, 0, sizeof(*out));
      out->status = RLU_PENDING;
      out->t_submit_us = r->t_submit;
      out->t_start_us = r->t_start;
    }
    return RLU_PENDING;
  }
  if (out) {
    out->status = r->status;
    const bool ok = r->state == Q_DONE;
    out->L = ok ? r->out : nullptr;
    out->U = ok ? (const char*)r->out + r->offU : nullptr;
    out->p = ok ? (const int64_t*)((const char*)r->out + r->offp) : nullptr;
    out->q = ok ? (const int64_t*)((const char*)r->out + r->offq) : nullptr;
    out->ldl = r->pb.m;
    out->ldu = r->pb.k;
    std::memcpy(out->info, r->info, sizeof(out->info));
    out->t_submit_us = r->t_submit;
    out->t_start_us = r->t_start;
    out->t_done_us = r->t_done;
  }
  return r->status;
}

rlu_status_t rlu_serve_copy(rlu_server_t srv, uint64_t ticket, const rlu_buffers_t* dst,
                            rlu_stream_t stream) {
  if (!srv || !dst) return RLU_ERR_INVALID_ARG;
  Req* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return RLU_ERR_UNKNOWN_TICKET;
    r = it->second;
    if (r->state == Q_QUEUED || r->state == Q_RUNNING) return RLU_PENDING;
    if (r->state != Q_DONE) return r->status;
  }
  const rlu_problem_t& pb = r->pb;
  if (!dst->L || !dst->U || !dst->p || !dst->q || dst->ldl < pb.m || dst->ldu < pb.k)
    return RLU_ERR_INVALID_ARG;
  DeviceScope dev(srv->cfg.device);
  hipStream_t s = (hipStream_t)stream;
  const size_t es = elem_size(pb);
  HIP_TRY(hipMemcpy2DAsync(dst->L, dst->ldl * es, r->out, pb.m * es, pb.m * es, pb.k,
                           hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpy2DAsync(dst->U, dst->ldu * es, (char*)r->out + r->offU, pb.k * es, pb.k * es,
                           pb.n, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(dst->p, (char*)r->out + r->offp, pb.m * 8, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(dst->q, (char*)r->out + r->offq, pb.n * 8, hipMemcpyDeviceToDevice, s));
  if (dst->info)
    HIP_TRY(hipMemcpyAsync(dst->info, (char*)r->out + r->offinfo, 12, hipMemcpyDeviceToDevice, s));
  return RLU_OK;
}

rlu_status_t rlu_serve_release(rlu_server_t srv, uint64_t ticket) {
  if (!srv) return RLU_ERR_INVALID_ARG;
  Req* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return RLU_ERR_UNKNOWN_TICKET;
    r = it->second;
    if (r->state == Q_QUEUED || r->state == Q_RUNNING) return RLU_PENDING;
    srv->reqs.erase(it);
    srv->policy.release(r->out_bytes);
  }
  if (r->out) {
    DeviceScope dev(srv->cfg.device);
    hipFreeAsync(r->out, srv->streams[0]);
  }
  delete r;
  srv->cv.notify_all();
  return RLU_OK;
}

rlu_status_t rlu_serve_stats(rlu_server_t srv, size_t* used_bytes, int32_t* queued,
                             int32_t* inflight) {
  if (!srv) return RLU_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (used_bytes) *used_bytes = srv->policy.used();
  if (queued) *queued = (int32_t)srv->policy.queued();
  if (inflight) *inflight = srv->policy.inflight();
  return RLU_OK;
}

rlu_status_t rlu_serve_destroy(rlu_server_t srv) {
  if (!srv) return RLU_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv.notify_all();
  if (srv->thr.joinable()) srv->thr.join();
  DeviceScope dev(srv->cfg.device);
  for (auto& kv : srv->reqs) {
    if (kv.second->out) hipFreeAsync(kv.second->out, srv->streams[0]);
    delete kv.second;
  }
  srv->reqs.clear();
  for (hipStream_t s : srv->streams) hipStreamSynchronize(s);
  if (srv->gate) hipEventDestroy(srv->gate);
  for (hipEvent_t x : srv->done) hipEventDestroy(x);
  for (int32_t* x : srv->info_host) hipHostFree(x);
  for (hipStream_t s : srv->streams) hipStreamDestroy(s);
  for (rlu_handle_s* x : srv->solo_h) rlu_destroy(x);
  rlu_destroy(srv->h);
  delete srv;
  return RLU_OK;
}

}  // extern "C"
