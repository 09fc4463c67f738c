// Admission policy of the serving form (rlu_serve.cpp), as a pure host state
// machine: no device, no threads, no clock.  The server drives it under its
// lock; tests drive it directly with a simulated clock.
//
//   * offer: a request whose footprint (its share of a batch workspace plus
//     the outputs the server keeps for it) exceeds the whole budget is
//     refused (it could never run); so is any request while the queue holds
//     max_queue entries (max_queue 0: unbounded).
//   * admit: strictly FIFO from the head of the queue.  A batch takes the
//     head and the requests behind it while they have the head's key (one
//     storage type and precision per batch) and the head's solo flag (a
//     request the batched kernels cannot run goes alone), while the charged
//     total stays within the budget and the admitted-and-not-done count
//     stays under max_inflight (0: no limit).  The first request that does
//     not fit ends the batch and keeps its place: nothing overtakes it.
//   * complete: a request of a batch finished; its workspace share returns.
//   * release: its outputs were released; their share returns.
#ifndef RLU_SERVE_POLICY_H
#define RLU_SERVE_POLICY_H

#include <cstddef>
#include <cstdint>
#include <deque>
#include <vector>

namespace rlu_serve {

struct Entry {
  uint64_t ticket = 0;
  size_t ws = 0, out = 0;  // workspace share and output bytes
  int key = 0;             // storage type and precision
  bool solo = false;       // runs alone
};

enum class Verdict { Accept, TooLarge, QueueFull };

class Policy {
 public:
  Policy(size_t budget, int max_inflight, int max_queue)
      : budget_(budget), max_inflight_(max_inflight), max_queue_(max_queue) {}

  Verdict offer(size_t ws, size_t out) const {
    if (ws + out > budget_) return Verdict::TooLarge;
    if (max_queue_ > 0 && (int)queue_.size() >= max_queue_) return Verdict::QueueFull;
    return Verdict::Accept;
  }
  void push(const Entry& e) { queue_.push_back(e); }

  // The next batch (at most max_batch requests; one when the head is solo).
  std::vector<Entry> admit(int max_batch) {
    std::vector<Entry> batch;
    if (queue_.empty()) return batch;
    const Entry head = queue_.front();
    const int cap = head.solo ? 1 : max_batch;
    while (!queue_.empty() && (int)batch.size() < cap) {
      const Entry& r = queue_.front();
      if (r.solo != head.solo || r.key != head.key) break;
      if (max_inflight_ > 0 && inflight_ >= max_inflight_) break;
      const size_t fp = r.ws + r.out;
      if (used_ + fp > budget_) break;
      used_ += fp;
      ++inflight_;
      batch.push_back(r);
      queue_.pop_front();
    }
    return batch;
  }
  void complete(size_t ws) {
    used_ -= ws;
    --inflight_;
  }
  void release(size_t out) { used_ -= out; }

  size_t used() const { return used_; }
  int inflight() const { return inflight_; }
  size_t queued() const { return queue_.size(); }
  size_t budget() const { return budget_; }

 private:
  size_t budget_;
  int max_inflight_, max_queue_;
  std::deque<Entry> queue_;
  size_t used_ = 0;
  int inflight_ = 0;
};

}  // namespace rlu_serve

#endif  // RLU_SERVE_POLICY_H
