// bfp_sched.hpp -- host-side core of the serving loop: device-memory arena
// (the HBM ledger), resident-vector table, request admission and tick
// building.  Plain C++ with no HIP calls: the executor that turns a tick into
// device work is a template parameter, so the same core runs with the HIP
// executor in libbfp and with a fake executor in the CPU tests.
//
// Continuous batching: each tick takes every request admitted since the last
// launch; up to `Executor::kStreams` ticks are in flight at once (one per
// stream), so requests that arrive while a tick runs are admitted and launched
// on the other stream before it finishes.  A request is admitted only when a
// slot is free and the arena can hold its result; otherwise it waits in FIFO
// order.
//
// Lifetimes: every resident vector counts the requests that read or write it
// (queued, admitted or running).  Freeing a vector that requests still hold
// retires its handle at once but returns its arena range only when the last
// of those requests completes, so a later put can never land on memory a
// running tick still reads.  Handles carry the generation of their table
// slot, so a handle of a freed vector is rejected even after its slot holds
// another vector.
#pragma once
#include <stdint.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_set>
#include <vector>

#include "bfp.h"

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

constexpr uint32_t kNoSlot = 0xFFFFFFFFu;

struct SchedRequest {
  uint64_t id = 0;
  int op = 0;
  uint8_t e = 0, m = 0, round = 0;
  uint64_t n = 0;                 // elements computed: a prefix of both operands
  uint64_t na = 0, nb = 0;        // operand lengths (their plane strides follow from them)
  uint64_t a_off = 0, b_off = 0;  // arena offsets of resident operands
  uint64_t c_off = 0;             // arena offset of the result (set at admission)
  uint64_t c_bytes = 0;
  uint64_t c_handle = 0;          // result handle (set at admission)
  uint32_t a_slot = kNoSlot, b_slot = kNoSlot, c_slot = kNoSlot;  // table slots held by the request
  int64_t t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
  int status = 0;
};

struct SchedStats {
  uint64_t submitted = 0, admitted = 0, completed = 0, ticks = 0, max_tick_requests = 0;
  uint64_t max_inflight_ticks = 0, deferred_budget = 0;
  uint64_t deferred_frees = 0, cancelled = 0, timed_out = 0;
};

// A resident vector: an operand put by the caller or a request's result.
struct Resident {
  uint64_t off = 0, bytes = 0, n = 0;
  uint8_t e = 0, m = 0;
  bool live = false;    // the slot holds a vector whose arena range is allocated
  bool retired = false; // freed by the caller while requests still hold it
  uint32_t gen = 1;     // generation of the slot (high half of its handles)
  uint32_t refs = 0;    // requests (queued, admitted, running) that read or write it
};

inline uint64_t make_handle(uint32_t slot, uint32_t gen) { return ((uint64_t)gen << 32) | ((uint64_t)slot + 1u); }

template <class Executor>
class Scheduler {
 public:
  Scheduler(Executor& ex, uint64_t budget, int slots) : ex_(ex), arena_(budget), slots_(slots) {}

  std::mutex& mutex() { return mu_; }

  // Free each result as soon as its request completes (the completion is
  // still reported, with result handle 0).
  void set_autofree(bool on) { autofree_ = on; }
  // Requests not launched within `ns` of their submission complete with
  // BFP_E_TIMEOUT (0: no limit).
  void set_queue_timeout(int64_t ns) { queue_timeout_ns_ = ns > 0 ? ns : 0; }
  // Largest tick, in bytes of operand and result planes (a, b and c of every
  // request; at least one request per tick; 0: no limit; 4 GiB by default).
  // Bounded ticks complete their requests progressively instead of all at
  // the end of one long launch, and a backlog alternates between the two
  // streams (measured at saturation with 4096 slots: 1.77e6 requests/s with
  // 4 GiB ticks against 1.08e6 with no limit).
  void set_tick_limit(uint64_t bytes) { tick_limit_ = bytes; }

  // ---- resident vectors (caller holds mutex) ----
  bool alloc_resident(uint64_t bytes, uint8_t e, uint8_t m, uint64_t n, uint64_t* handle, uint64_t* off) {
    if (!arena_.alloc(bytes, off)) return false;
    uint32_t slot;
    if (!free_slots_.empty()) {
      slot = free_slots_.front();
      free_slots_.pop_front();
    } else {
      slot = (uint32_t)res_.size();
      res_.emplace_back();
    }
    Resident& r = res_[slot];
    r.off = *off;
    r.bytes = Arena::round(bytes);
    r.n = n;
    r.e = e;
    r.m = m;
    r.live = true;
    r.retired = false;
    r.refs = 0;
    *handle = make_handle(slot, r.gen);
    return true;
  }
  // Slot of a live, not retired vector, or kNoSlot.
  uint32_t slot_of(uint64_t h) const {
    const uint64_t s1 = h & 0xFFFFFFFFull;
    if (s1 == 0 || s1 > res_.size()) return kNoSlot;
    const uint32_t slot = (uint32_t)(s1 - 1);
    const Resident& r = res_[slot];
    if (!r.live || r.retired || r.gen != (uint32_t)(h >> 32)) return kNoSlot;
    return slot;
  }
  const Resident* resident(uint64_t h) const {
    const uint32_t s = slot_of(h);
    return s == kNoSlot ? nullptr : &res_[s];
  }
  // Retire handle h.  Its range goes back to the arena now if no request
  // holds it, else when the last holder completes.  False if h is not a
  // live handle.
  bool free_resident(uint64_t h) {
    const uint32_t s = slot_of(h);
    if (s == kNoSlot) return false;
    Resident& r = res_[s];
    r.retired = true;
    if (r.refs == 0) reclaim(s);
    else stats_.deferred_frees++;
    return true;
  }
  // Hold vector h for the caller's own use of its memory (for example an
  // unpack); returns its slot (kNoSlot if h is not live).  Pair with unpin.
  uint32_t pin(uint64_t h) {
    const uint32_t s = slot_of(h);
    if (s != kNoSlot) res_[s].refs++;
    return s;
  }
  void unpin(uint32_t slot) { unref(slot); }
  size_t resident_slots() const { return res_.size(); }
  size_t live_residents() const { return arena_.live_count(); }

  // ---- requests (caller holds mutex) ----
  // Queue r (id, op, e, m, round, n and c_bytes set by the caller) on
  // operands ha and hb.  Checks that both handles are live, of r's format
  // and at least n long, and that the result could ever fit in the arena;
  // returns BFP_OK or the error, and on success holds both operands until
  // the request completes.
  int submit(SchedRequest r, uint64_t ha, uint64_t hb) {
    const uint32_t sa = slot_of(ha), sb = slot_of(hb);
    if (sa == kNoSlot || sb == kNoSlot) return BFP_E_ARG;
    const Resident& ra = res_[sa];
    const Resident& rb = res_[sb];
    if (ra.e != r.e || ra.m != r.m || rb.e != r.e || rb.m != r.m) return BFP_E_FORMAT;
    if (r.n == 0 || r.n > ra.n || r.n > rb.n) return BFP_E_ARG;  // a prefix of each operand
    if (Arena::round(r.c_bytes) > arena_.capacity()) return BFP_E_BUDGET;
    r.a_off = ra.off;
    r.b_off = rb.off;
    r.na = ra.n;
    r.nb = rb.n;
    r.a_slot = sa;
    r.b_slot = sb;
    r.c_slot = kNoSlot;
    r.c_handle = 0;
    r.status = 0;
    res_[sa].refs++;
    res_[sb].refs++;
    r.t_submit = now_ns();
    pending_.push_back(r);
    stats_.submitted++;
    return BFP_OK;
  }

  // Withdraw a request that has not been launched: it completes with
  // BFP_E_CANCELLED and releases what it held.  BFP_E_BUSY if it is on the
  // device (it then completes normally), BFP_E_ARG if no request with this
  // id is queued or running.
  int cancel(uint64_t id) {
    for (auto it = pending_.begin(); it != pending_.end(); ++it)
      if (it->id == id) {
        SchedRequest r = *it;
        pending_.erase(it);
        drop(r, BFP_E_CANCELLED);
        stats_.cancelled++;
        return BFP_OK;
      }
    for (auto it = next_.begin(); it != next_.end(); ++it)
      if (it->id == id) {
        SchedRequest r = *it;
        next_.erase(it);
        drop(r, BFP_E_CANCELLED);
        stats_.cancelled++;
        return BFP_OK;
      }
    return launched_.count(id) ? BFP_E_BUSY : BFP_E_ARG;
  }

  // One scheduling pass: completions, FIFO admission, and a launch of the
  // admitted requests on a free stream.  Equivalent to collect(), launching
  // the returned batch, and commit().  Returns true if anything changed.
  bool step() {
    std::vector<SchedRequest> batch;
    bool changed = collect(&batch);
    if (!batch.empty()) {
      commit(&batch, ex_.launch(batch));
      changed = true;
    }
    return changed;
  }

  // Completions, expiry and admission; if a stream is free and requests
  // were admitted, moves them into *batch (stamped with their launch time)
  // and reserves the stream.  The caller launches the batch on the executor
  // -- without the scheduler's lock if it holds one, since only the
  // scheduling thread touches the executor -- and then calls commit().
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
        launched_.erase(r.id);
        finish(r);
      }
      done.clear();
      inflight_ticks_--;
    }
    // expiry: submission times grow along both queues
    if (queue_timeout_ns_ > 0) {
      const int64_t limit = now_ns() - queue_timeout_ns_;
      while (!next_.empty() && next_.front().t_submit < limit) {
        SchedRequest r = next_.front();
        next_.erase(next_.begin());
        drop(r, BFP_E_TIMEOUT);
        stats_.timed_out++;
        changed = true;
      }
      while (!pending_.empty() && pending_.front().t_submit < limit) {
        SchedRequest r = pending_.front();
        pending_.pop_front();
        drop(r, BFP_E_TIMEOUT);
        stats_.timed_out++;
        changed = true;
      }
    }
    // admission: FIFO, needs a slot and room for the result
    while (!pending_.empty() && inflight_reqs_ + (int)next_.size() < slots_) {
      SchedRequest& r = pending_.front();
      uint64_t off, h;
      if (!alloc_resident(r.c_bytes, r.e, r.m, r.n, &h, &off)) {
        stats_.deferred_budget++;
        break;
      }
      r.c_off = off;
      r.c_handle = h;
      r.c_slot = (uint32_t)((h & 0xFFFFFFFFull) - 1);
      res_[r.c_slot].refs++;  // the result is held until its request completes
      r.t_admit = now_ns();
      next_.push_back(r);
      pending_.pop_front();
      stats_.admitted++;
      changed = true;
    }
    // hand a tick to the caller if a stream is free: the admitted requests
    // in FIFO order, up to the tick limit
    if (!next_.empty() && inflight_ticks_ < Executor::kStreams) {
      const int64_t t = now_ns();
      size_t take = next_.size();
      if (tick_limit_) {
        uint64_t bytes = 0;
        for (take = 0; take < next_.size(); ++take) {
          bytes += 3 * next_[take].c_bytes;
          if (take > 0 && bytes > tick_limit_) break;
        }
      }
      batch->assign(next_.begin(), next_.begin() + take);
      next_.erase(next_.begin(), next_.begin() + take);
      for (auto& r : *batch) {
        r.t_launch = t;
        launched_.insert(r.id);
      }
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
      const int64_t t = now_ns();
      for (auto& r : *batch) {  // failed launch: release the results, report the error
        launched_.erase(r.id);
        r.t_done = t;
        drop(r, st);
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
  void reclaim(uint32_t s) {
    Resident& r = res_[s];
    arena_.release(r.off);
    r.live = false;
    r.retired = false;
    r.refs = 0;
    r.gen = r.gen + 1u ? r.gen + 1u : 1u;  // generation 0 is never issued
    free_slots_.push_back(s);
  }
  void unref(uint32_t s) {
    if (s == kNoSlot || s >= res_.size()) return;
    Resident& r = res_[s];
    if (!r.live || r.refs == 0) return;
    if (--r.refs == 0 && r.retired) reclaim(s);
  }
  // A request that ran: drop its holds on the operands and the result (the
  // result stays live for the caller unless autofree is on).
  void finish(SchedRequest& r) {
    unref(r.a_slot);
    unref(r.b_slot);
    if (r.c_slot != kNoSlot) {
      unref(r.c_slot);
      if (r.status != 0 || autofree_) {
        free_resident(r.c_handle);
        r.c_handle = 0;
      }
    }
    completed_.push_back(r);
    stats_.completed++;
  }
  // A request that did not run (cancelled, expired or a failed launch):
  // complete it with `status`; its result, if admitted, is freed.
  void drop(SchedRequest& r, int status) {
    r.status = status;
    if (!r.t_done) r.t_done = now_ns();
    finish(r);
  }

  Executor& ex_;
  Arena arena_;
  int slots_;
  std::mutex mu_;
  std::vector<Resident> res_;
  std::deque<uint32_t> free_slots_;  // reused oldest first, so a slot's generations advance slowly
  std::deque<SchedRequest> pending_;
  std::vector<SchedRequest> next_;
  std::deque<SchedRequest> completed_;
  std::unordered_set<uint64_t> launched_;  // ids handed to the executor and not yet completed
  int inflight_reqs_ = 0;
  int inflight_ticks_ = 0;
  int64_t queue_timeout_ns_ = 0;
  uint64_t tick_limit_ = 4ull << 30;
  bool autofree_ = false;
  SchedStats stats_;
};

// The serving worker: one scheduling pass after another until `stop` --
// completions, expiry and admission under the scheduler's lock, the launch
// of a collected tick without it (only this thread touches the executor, so
// submitters and pollers proceed meanwhile), then the commit under the lock.
// Sleeps on `cv` (about 2 ms at most) when nothing is queued or running.
template <class Executor>
void serve_loop(Scheduler<Executor>& sched, Executor& ex, const std::atomic<bool>& stop,
                std::condition_variable& cv) {
  std::unique_lock<std::mutex> lk(sched.mutex());
  std::vector<SchedRequest> batch;
  while (!stop.load()) {
    bool changed = sched.collect(&batch);
    if (!batch.empty()) {
      lk.unlock();
      const int st = ex.launch(batch);
      lk.lock();
      sched.commit(&batch, st);
      changed = true;
    }
    if (sched.idle()) {
      // a system-clock deadline: the wait is a bounded nap (submissions and
      // stop notify `cv`), and libstdc++ waits on it with
      // pthread_cond_timedwait, which ThreadSanitizer follows (a steady-clock
      // wait_for goes through pthread_cond_clockwait, which the sanitizer of
      // this toolchain does not intercept)
      cv.wait_until(lk, std::chrono::system_clock::now() + std::chrono::milliseconds(2));
    } else if (!changed) {
      // ticks in flight: release the lock briefly so callers can submit/poll
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    }
  }
}

}  // namespace bfp
