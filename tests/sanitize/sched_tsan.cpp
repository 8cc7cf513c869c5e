// sched_tsan.cpp -- test driver built with ThreadSanitizer: the serving
// scheduler with its real worker loop (serve_loop) and a fake executor whose
// ticks finish after a random delay, raced by submitter threads (put, submit,
// free, cancel, each under the scheduler's lock as the C ABI takes it) and
// poller threads (completions).  Checks that every accepted request completes
// exactly once and that every byte returns to the arena.
#include <stdint.h>
#include <stdio.h>

#include <atomic>
#include <deque>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "bfp_sched.hpp"

namespace {
struct DelayExecutor {
  static constexpr int kStreams = 2;
  std::deque<std::pair<int64_t, std::vector<bfp::SchedRequest>>> running;  // worker thread only
  std::mt19937 rng{7};
  int launch(const std::vector<bfp::SchedRequest>& reqs) {
    if (rng() % 50 == 0) return -5;  // a failed launch now and then
    running.emplace_back(bfp::now_ns() + (int64_t)(rng() % 200) * 1000, reqs);
    return 0;
  }
  bool poll_done(std::vector<bfp::SchedRequest>* out) {
    if (running.empty() || running.front().first > bfp::now_ns()) return false;
    *out = running.front().second;
    running.pop_front();
    return true;
  }
};
}  // namespace

int main() {
  DelayExecutor ex;
  bfp::Scheduler<DelayExecutor> sched(ex, 64ull << 20, 64);
  sched.set_tick_limit(1 << 20);
  std::atomic<bool> stop{false};
  std::condition_variable cv;
  std::thread worker([&] { bfp::serve_loop(sched, ex, stop, cv); });
  std::mutex book_mu;
  std::set<uint64_t> accepted, completed;
  std::atomic<uint64_t> next_id{1};
  std::atomic<int> dup{0};
  std::atomic<bool> submitting{true};
  std::vector<std::thread> threads;
  for (int t = 0; t < 4; ++t)
    threads.emplace_back([&, t] {
      std::mt19937_64 rng(100 + t);
      std::vector<uint64_t> mine;
      for (int it = 0; it < 20000; ++it) {
        const unsigned x = (unsigned)(rng() % 100);
        std::lock_guard<std::mutex> lk(sched.mutex());
        if (x < 20 || mine.empty()) {
          uint64_t h, off;
          if (sched.alloc_resident(4096 * (1 + rng() % 16), 5, 10, 1 + rng() % 50000, &h, &off)) mine.push_back(h);
        } else if (x < 35) {
          const size_t i = rng() % mine.size();
          sched.free_resident(mine[i]);
          mine.erase(mine.begin() + i);
        } else if (x < 90) {
          bfp::SchedRequest r;
          r.id = next_id.fetch_add(1);
          r.e = 5;
          r.m = 10;
          r.n = 1 + rng() % 1000;
          r.c_bytes = 256 * (1 + rng() % 64);
          if (sched.submit(r, mine[rng() % mine.size()], mine[rng() % mine.size()]) == 0) {
            std::lock_guard<std::mutex> bk(book_mu);
            accepted.insert(r.id);
          }
        } else {
          (void)sched.cancel(1 + rng() % next_id.load());
        }
        cv.notify_one();
      }
      std::lock_guard<std::mutex> lk(sched.mutex());
      for (uint64_t h : mine) sched.free_resident(h);
    });
  for (int t = 0; t < 2; ++t)
    threads.emplace_back([&] {
      bfp::SchedRequest buf[64];
      for (;;) {
        size_t k;
        bool idle;
        {
          std::lock_guard<std::mutex> lk(sched.mutex());
          k = sched.take_completed(buf, 64);
          for (size_t i = 0; i < k; ++i)
            if (buf[i].status == 0) sched.free_resident(buf[i].c_handle);
          idle = sched.idle();
        }
        {
          std::lock_guard<std::mutex> bk(book_mu);
          for (size_t i = 0; i < k; ++i)
            if (!completed.insert(buf[i].id).second) dup++;
        }
        if (k == 0 && idle && !submitting.load()) break;
        if (k == 0) std::this_thread::yield();
      }
    });
  for (int t = 0; t < 4; ++t) threads[t].join();
  submitting.store(false);
  cv.notify_one();
  for (size_t t = 4; t < threads.size(); ++t) threads[t].join();
  stop.store(true);
  cv.notify_one();
  worker.join();
  int bad = 0;
  if (dup.load()) {
    fprintf(stderr, "%d requests completed twice\n", dup.load());
    bad++;
  }
  if (accepted != completed) {
    fprintf(stderr, "%zu accepted, %zu completed\n", accepted.size(), completed.size());
    bad++;
  }
  if (sched.used() != 0) {
    fprintf(stderr, "%llu bytes still in use\n", (unsigned long long)sched.used());
    bad++;
  }
  if (bad) return 1;
  printf("sched_tsan ok: %zu requests\n", accepted.size());
  return 0;
}
