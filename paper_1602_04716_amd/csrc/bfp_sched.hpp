// bfp_sched.hpp -- host-side core of the serving loop: device-memory arena
// (the HBM ledger), request admission and tick building.  Plain C++ with no
// HIP calls: the executor that turns a tick into device work is a template
// parameter, so the same core runs with the HIP executor in libbfp and with a
// fake executor in the CPU tests.
//
// Continuous batching: each tick takes every request admitted since the last
// launch; up to `Executor::kStreams` ticks are in flight at once (one per
// stream), so requests that arrive while a tick runs are admitted and launched
// on the other stream before it finishes.  A request is admitted only when a
// slot is free and the arena can hold its result; otherwise it waits in FIFO
// order.
#pragma once
#include <stdint.h>

#include <chrono>
#include <deque>
#include <map>
#include <mutex>
#include <vector>

namespace bfp {

inline int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// First-fit allocator over [0, capacity) with coalescing free list; all
// offsets and sizes are multiples of kAlign.
class Arena {
 public:
  static constexpr uint64_t kAlign = 256;
  explicit Arena(uint64_t capacity) : cap_(capacity / kAlign * kAlign) {
    if (cap_) free_[0] = cap_;
  }
  // Returns true and the offset, or false if no free range is large enough.
  bool alloc(uint64_t bytes, uint64_t* off) {
    const uint64_t sz = round(bytes);
    if (sz == 0 || sz > cap_) return false;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= sz) {
        *off = it->first;
        const uint64_t rest = it->second - sz, start = it->first + sz;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += sz;
        if (used_ > high_) high_ = used_;
        live_[*off] = sz;
        return true;
      }
    }
    return false;
  }
  // Returns the bytes released (0 if `off` is not a live allocation).
  uint64_t release(uint64_t off) {
    auto lv = live_.find(off);
    if (lv == live_.end()) return 0;
    const uint64_t freed = lv->second;
    uint64_t sz = freed;
    live_.erase(lv);
    used_ -= sz;
    uint64_t start = off;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first == off + sz) {
      sz += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == start) {
        start = pv->first;
        sz += pv->second;
        free_.erase(pv);
      }
    }
    free_[start] = sz;
    return freed;
  }
  uint64_t used() const { return used_; }
  uint64_t high_water() const { return high_; }
  uint64_t capacity() const { return cap_; }
  size_t live_count() const { return live_.size(); }
  size_t free_ranges() const { return free_.size(); }
  static uint64_t round(uint64_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

 private:
  uint64_t cap_;
  uint64_t used_ = 0, high_ = 0;
  std::map<uint64_t, uint64_t> free_;  // offset -> size
  std::map<uint64_t, uint64_t> live_;  // offset -> size
};

struct SchedRequest {
  uint64_t id = 0;
  int op = 0;
  uint8_t e = 0, m = 0, round = 0;
  uint64_t n = 0;                 // elements computed: a prefix of both operands
  uint64_t na = 0, nb = 0;        // operand lengths (their plane strides follow from them)
  uint64_t a_off = 0, b_off = 0;  // arena offsets of resident operands
  uint64_t c_off = 0;             // arena offset of the result (set at admission)
  uint64_t c_bytes = 0;
  uint32_t c_handle = 0;          // result handle (set at admission)
  int64_t t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
  int status = 0;
};

struct SchedStats {
  uint64_t submitted = 0, admitted = 0, completed = 0, ticks = 0, max_tick_requests = 0;
  uint64_t max_inflight_ticks = 0, deferred_budget = 0;
};

// Resident vectors by handle (operands put by the caller, and results).
struct Resident {
  uint64_t off = 0, bytes = 0, n = 0;
  uint8_t e = 0, m = 0;
  bool live = false;
};

template <class Executor>
class Scheduler {
 public:
  Scheduler(Executor& ex, uint64_t budget, int slots) : ex_(ex), arena_(budget), slots_(slots) {}

  std::mutex& mutex() { return mu_; }

  // Free each result as soon as its request completes (the completion is
  // still reported, with result handle 0).
  void set_autofree(bool on) { autofree_ = on; }

  // ---- resident vectors (caller holds mutex) ----
  bool alloc_resident(uint64_t bytes, uint8_t e, uint8_t m, uint64_t n, uint32_t* handle, uint64_t* off) {
    if (!arena_.alloc(bytes, off)) return false;
    Resident r;
    r.off = *off;
    r.bytes = Arena::round(bytes);
    r.n = n;
    r.e = e;
    r.m = m;
    r.live = true;
    res_.push_back(r);
    *handle = (uint32_t)res_.size();  // handles start at 1
    return true;
  }
  const Resident* resident(uint32_t h) const {
    if (h == 0 || h > res_.size() || !res_[h - 1].live) return nullptr;
    return &res_[h - 1];
  }
  bool free_resident(uint32_t h) {
    if (h == 0 || h > res_.size() || !res_[h - 1].live) return false;
    arena_.release(res_[h - 1].off);
    res_[h - 1].live = false;
    return true;
  }

  // ---- requests (caller holds mutex) ----
  void submit(const SchedRequest& r) {
    pending_.push_back(r);
    pending_.back().t_submit = now_ns();
    stats_.submitted++;
  }

  // One scheduling pass (caller holds mutex): collect finished ticks, admit,
  // launch.  Returns true if anything changed.
  // One scheduling pass: completions, FIFO admission, and a launch of the
  // admitted requests on a free stream.  Equivalent to collect(), launching
  // the returned batch, and commit().
  bool step() {
    std::vector<SchedRequest> batch;
    bool changed = collect(&batch);
    if (!batch.empty()) {
      commit(&batch, ex_.launch(batch));
      changed = true;
    }
    return changed;
  }

  // Completions and admission; if a stream is free and requests were
  // admitted, moves them into *batch (stamped with their launch time) and
  // reserves the stream.  The caller launches the batch on the executor --
  // without the scheduler's lock if it holds one, since only the scheduling
  // thread touches the executor -- and then calls commit().
  bool collect(std::vector<SchedRequest>* batch) {
    bool changed = false;
    // completions
    std::vector<SchedRequest> done;
    while (ex_.poll_done(&done)) {
      changed = true;
      const int64_t t = now_ns();
      for (auto& r : done) {
        r.t_done = t;
        inflight_reqs_--;
        if (autofree_ && r.status == 0) {
          free_resident(r.c_handle);
          r.c_handle = 0;
        }
        completed_.push_back(r);
        stats_.completed++;
      }
      done.clear();
      inflight_ticks_--;
    }
    // admission: FIFO, needs a slot and room for the result
    while (!pending_.empty() && inflight_reqs_ + (int)next_.size() < slots_) {
      SchedRequest& r = pending_.front();
      uint64_t off;
      uint32_t h;
      if (!alloc_resident(r.c_bytes, r.e, r.m, r.n, &h, &off)) {
        stats_.deferred_budget++;
        break;
      }
      r.c_off = off;
      r.c_handle = h;
      r.t_admit = now_ns();
      next_.push_back(r);
      pending_.pop_front();
      stats_.admitted++;
      changed = true;
    }
    // hand a tick to the caller if a stream is free
    if (!next_.empty() && inflight_ticks_ < Executor::kStreams) {
      const int64_t t = now_ns();
      for (auto& r : next_) r.t_launch = t;
      batch->swap(next_);
      next_.clear();
      inflight_ticks_++;          // the stream is taken until commit() or the tick's completion
      inflight_reqs_ += (int)batch->size();
      changed = true;
    }
    return changed;
  }

  // Record the outcome of launching a batch from collect(): st == 0 keeps it
  // in flight until the executor reports it done; otherwise its results are
  // released and it completes with status st.
  void commit(std::vector<SchedRequest>* batch, int st) {
    if (st != 0) {
      inflight_ticks_--;
      inflight_reqs_ -= (int)batch->size();
      for (auto& r : *batch) {  // failed launch: release the results, report the error
        free_resident(r.c_handle);
        r.c_handle = 0;
        r.status = st;
        r.t_done = now_ns();
        completed_.push_back(r);
        stats_.completed++;
      }
    } else {
      stats_.ticks++;
      if (batch->size() > stats_.max_tick_requests) stats_.max_tick_requests = batch->size();
      if ((uint64_t)inflight_ticks_ > stats_.max_inflight_ticks) stats_.max_inflight_ticks = inflight_ticks_;
    }
    batch->clear();
  }

  size_t take_completed(SchedRequest* out, size_t max) {
    size_t k = 0;
    while (k < max && !completed_.empty()) {
      out[k++] = completed_.front();
      completed_.pop_front();
    }
    return k;
  }

  bool idle() const { return pending_.empty() && next_.empty() && inflight_ticks_ == 0; }
  uint64_t used() const { return arena_.used(); }
  uint64_t high_water() const { return arena_.high_water(); }
  uint64_t capacity() const { return arena_.capacity(); }
  size_t pending() const { return pending_.size(); }
  int inflight_requests() const { return inflight_reqs_; }
  const SchedStats& stats() const { return stats_; }

 private:
  Executor& ex_;
  Arena arena_;
  int slots_;
  std::mutex mu_;
  std::vector<Resident> res_;
  std::deque<SchedRequest> pending_;
  std::vector<SchedRequest> next_;
  std::deque<SchedRequest> completed_;
  int inflight_reqs_ = 0;
  int inflight_ticks_ = 0;
  bool autofree_ = false;
  SchedStats stats_;
};

}  // namespace bfp
