// bfp_server.hip -- serving loop: device-resident bitslice vectors, requests
// admitted under an HBM budget, continuous batching on two streams.
//
// The scheduler core (admission, ledger, ticks) is bfp_sched.hpp; this file
// supplies the HIP executor and the C ABI.  All resident vectors live in one
// device arena allocated at creation (the budget); the arena's first-fit
// allocator is the ledger, so admission can never exceed the budget.  A
// worker thread runs the scheduler: it collects finished ticks (event
// queries), admits queued requests while slots and arena space allow, and
// launches each tick's requests as one batched persistent kernel
// (bfp_batch.hpp) on whichever of the two streams is free, so a tick can start
// while the previous one is still running.
#include <hip/hip_runtime.h>

#include <cstring>

#include <atomic>
#include <condition_variable>
#include <new>
#include <thread>

#include "bfp.h"
#include "bfp_batch.hpp"
#include "bfp_ops.hpp"
#include "bfp_sched.hpp"

namespace bfp {
namespace {

struct HipExecutor {
  static constexpr int kStreams = 2;
  struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    BatchTask* d_tasks = nullptr;
    BatchChunk* d_chunks = nullptr;
    uint32_t* d_counter = nullptr;
    BatchTask* h_tasks = nullptr;  // pinned staging
    BatchChunk* h_chunks = nullptr;
    size_t cap_tasks = 0, cap_chunks = 0;
    bool busy = false;
    uint64_t seq = 0;
    std::vector<SchedRequest> reqs;
  };
  uint8_t* base = nullptr;  // arena base (device)
  int cap[kBatchClasses] = {};  // resident blocks of each class kernel
  Slot slot[kStreams];
  uint64_t seq = 0;
  std::vector<BatchTask> tasks;
  std::vector<BatchChunk> chunks;

  bool grow(Slot& s, size_t nt, size_t nc) {
    if (nt > s.cap_tasks) {
      size_t cap = s.cap_tasks ? s.cap_tasks : 1024;
      while (cap < nt) cap *= 2;
      if (s.d_tasks) (void)hipFree(s.d_tasks);
      if (s.h_tasks) (void)hipHostFree(s.h_tasks);
      s.d_tasks = nullptr;
      s.h_tasks = nullptr;
      s.cap_tasks = 0;
      if (hipMalloc(&s.d_tasks, cap * sizeof(BatchTask)) != hipSuccess) return false;
      if (hipHostMalloc(&s.h_tasks, cap * sizeof(BatchTask), hipHostMallocDefault) != hipSuccess) return false;
      s.cap_tasks = cap;
    }
    if (nc > s.cap_chunks) {
      size_t cap = s.cap_chunks ? s.cap_chunks : 16384;
      while (cap < nc) cap *= 2;
      if (s.d_chunks) (void)hipFree(s.d_chunks);
      if (s.h_chunks) (void)hipHostFree(s.h_chunks);
      s.d_chunks = nullptr;
      s.h_chunks = nullptr;
      s.cap_chunks = 0;
      if (hipMalloc(&s.d_chunks, cap * sizeof(BatchChunk)) != hipSuccess) return false;
      if (hipHostMalloc(&s.h_chunks, cap * sizeof(BatchChunk), hipHostMallocDefault) != hipSuccess) return false;
      s.cap_chunks = cap;
    }
    return true;
  }

  bool init() {
    for (int c = 0; c < kBatchClasses; ++c) {
      cap[c] = batch_resident_blocks(c);
      if (cap[c] <= 0) return false;
    }
    for (Slot& s : slot) {
      if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) return false;
      if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) return false;
      if (hipMalloc(&s.d_counter, 256) != hipSuccess) return false;
      if (!grow(s, 1024, 16384)) return false;
    }
    return true;
  }

  void shutdown() {
    for (Slot& s : slot) {
      if (s.stream) (void)hipStreamSynchronize(s.stream);
      if (s.d_tasks) (void)hipFree(s.d_tasks);
      if (s.d_chunks) (void)hipFree(s.d_chunks);
      if (s.d_counter) (void)hipFree(s.d_counter);
      if (s.h_tasks) (void)hipHostFree(s.h_tasks);
      if (s.h_chunks) (void)hipHostFree(s.h_chunks);
      if (s.done) (void)hipEventDestroy(s.done);
      if (s.stream) (void)hipStreamDestroy(s.stream);
      s = Slot();
    }
  }

  int launch(const std::vector<SchedRequest>& reqs) {
    Slot* s = nullptr;
    for (Slot& c : slot)
      if (!c.busy) {
        s = &c;
        break;
      }
    if (!s) return BFP_E_ARG;
    tasks.resize(reqs.size());
    for (size_t i = 0; i < reqs.size(); ++i) {
      const SchedRequest& r = reqs[i];
      bfp_format f;
      f.e = r.e;
      f.m = r.m;
      f.round = r.round;
      f.pad = 0;
      if (!batch_task(base + r.a_off, r.na, base + r.b_off, r.nb, base + r.c_off, r.n, f, r.op, &tasks[i]))
        return BFP_E_FORMAT;
    }
    batch_chunks(tasks, &chunks);
    if (!grow(*s, tasks.size(), chunks.size())) return BFP_E_NOMEM;
    std::memcpy(s->h_tasks, tasks.data(), tasks.size() * sizeof(BatchTask));
    std::memcpy(s->h_chunks, chunks.data(), chunks.size() * sizeof(BatchChunk));
    if (hipMemcpyAsync(s->d_tasks, s->h_tasks, tasks.size() * sizeof(BatchTask), hipMemcpyHostToDevice,
                       s->stream) != hipSuccess ||
        hipMemcpyAsync(s->d_chunks, s->h_chunks, chunks.size() * sizeof(BatchChunk), hipMemcpyHostToDevice,
                       s->stream) != hipSuccess)
      return BFP_E_HIP;
    const BatchSplit split = batch_split(tasks, chunks, cap);
    if (batch_launch(s->d_tasks, s->d_chunks, split, s->d_counter, s->stream) != hipSuccess) return BFP_E_HIP;
    if (hipEventRecord(s->done, s->stream) != hipSuccess) return BFP_E_HIP;
    s->busy = true;
    s->seq = ++seq;
    s->reqs = reqs;
    return BFP_OK;
  }

  // Oldest finished tick first.
  bool poll_done(std::vector<SchedRequest>* out) {
    Slot* oldest = nullptr;
    for (Slot& c : slot)
      if (c.busy && (!oldest || c.seq < oldest->seq)) oldest = &c;
    if (!oldest) return false;
    const hipError_t q = hipEventQuery(oldest->done);
    if (q == hipErrorNotReady) return false;
    for (SchedRequest& r : oldest->reqs) {
      if (q != hipSuccess) r.status = BFP_E_HIP;
      out->push_back(r);
    }
    oldest->reqs.clear();
    oldest->busy = false;
    return true;
  }
};

}  // namespace
}  // namespace bfp

using namespace bfp;

struct bfp_server {
  int device = 0;
  uint64_t budget = 0;
  void* arena = nullptr;
  HipExecutor ex;
  Scheduler<HipExecutor>* sched = nullptr;
  std::thread worker;
  std::atomic<bool> stop{false};
  std::condition_variable cv;
  std::atomic<uint64_t> next_id{1};
};

namespace {

void worker_loop(bfp_server* s) {
  (void)hipSetDevice(s->device);
  serve_loop(*s->sched, s->ex, s->stop, s->cv);
}

uint64_t bitslice_bytes_of(uint8_t e, uint8_t m, uint64_t n) {
  return (uint64_t)(1 + e + m) * bfp_plane_stride_words(n) * 4u;
}

}  // namespace

extern "C" {

bfp_status bfp_server_create(uint64_t hbm_budget_bytes, int32_t slots, bfp_server** out) {
  if (!out) return BFP_E_NULL;
  *out = nullptr;
  if (hbm_budget_bytes < Arena::kAlign || slots < 1 || slots > (1 << 20)) return BFP_E_ARG;
  bfp_server* s = new (std::nothrow) bfp_server();
  if (!s) return BFP_E_NOMEM;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return BFP_E_NODEV;
  }
  s->budget = hbm_budget_bytes / Arena::kAlign * Arena::kAlign;
  if (hipMalloc(&s->arena, s->budget) != hipSuccess) {
    delete s;
    return BFP_E_NOMEM;
  }
  if (!s->ex.init()) {
    s->ex.shutdown();
    (void)hipFree(s->arena);
    delete s;
    return BFP_E_HIP;
  }
  s->ex.base = static_cast<uint8_t*>(s->arena);
  s->sched = new Scheduler<HipExecutor>(s->ex, s->budget, slots);
  s->worker = std::thread(worker_loop, s);
  *out = s;
  return BFP_OK;
}

void bfp_server_destroy(bfp_server* s) {
  if (!s) return;
  s->stop.store(true);
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  s->ex.shutdown();
  delete s->sched;
  if (s->arena) (void)hipFree(s->arena);
  delete s;
}

bfp_status bfp_server_put(bfp_server* s, bfp_format f, const void* std_dev, uint64_t n, void* stream,
                          bfp_handle* handle) {
  if (!s || !std_dev || !handle) return BFP_E_NULL;
  if (!bfp_format_supported(f)) return BFP_E_FORMAT;
  if (n == 0 || n > (1ull << 36)) return BFP_E_ARG;
  uint64_t off;
  bfp_handle h;
  {
    std::lock_guard<std::mutex> lk(s->sched->mutex());
    if (!s->sched->alloc_resident(bitslice_bytes_of(f.e, f.m, n), f.e, f.m, n, &h, &off)) return BFP_E_BUDGET;
  }
  bfp_status st = bfp_pack(f, std_dev, static_cast<uint8_t*>(s->arena) + off, n, stream);
  if (st == BFP_OK && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) st = BFP_E_HIP;
  if (st != BFP_OK) {
    std::lock_guard<std::mutex> lk(s->sched->mutex());
    s->sched->free_resident(h);
    return st;
  }
  *handle = h;
  return BFP_OK;
}

bfp_status bfp_server_submit(bfp_server* s, int op, bfp_format f, bfp_handle a, bfp_handle b, uint64_t n,
                             uint64_t* req_id) {
  if (!s || !req_id) return BFP_E_NULL;
  if (!op_valid(op)) return BFP_E_OP;
  if (!bfp_format_supported(f) || !batch_format_ok(f)) return BFP_E_FORMAT;
  SchedRequest r;
  r.op = op;
  r.e = f.e;
  r.m = f.m;
  r.round = f.round;
  r.n = n;
  r.c_bytes = n ? bitslice_bytes_of(f.e, f.m, n) : 0;
  {
    std::lock_guard<std::mutex> lk(s->sched->mutex());
    r.id = s->next_id.fetch_add(1);
    const int st = s->sched->submit(r, a, b);
    if (st != BFP_OK) return st;
    *req_id = r.id;
  }
  s->cv.notify_one();
  return BFP_OK;
}

bfp_status bfp_server_cancel(bfp_server* s, uint64_t req_id) {
  if (!s) return BFP_E_NULL;
  std::lock_guard<std::mutex> lk(s->sched->mutex());
  return s->sched->cancel(req_id);
}

bfp_status bfp_server_set_tick_limit(bfp_server* s, uint64_t max_bytes) {
  if (!s) return BFP_E_NULL;
  std::lock_guard<std::mutex> lk(s->sched->mutex());
  s->sched->set_tick_limit(max_bytes);
  return BFP_OK;
}

bfp_status bfp_server_set_queue_timeout(bfp_server* s, int64_t timeout_ns) {
  if (!s) return BFP_E_NULL;
  std::lock_guard<std::mutex> lk(s->sched->mutex());
  s->sched->set_queue_timeout(timeout_ns);
  return BFP_OK;
}

bfp_status bfp_server_set_autofree(bfp_server* s, int32_t on) {
  if (!s) return BFP_E_NULL;
  std::lock_guard<std::mutex> lk(s->sched->mutex());
  s->sched->set_autofree(on != 0);
  return BFP_OK;
}

bfp_status bfp_server_replay(bfp_server* s, const bfp_request* reqs, uint32_t count, uint64_t* first_id) {
  if (!s || (count && !reqs)) return BFP_E_NULL;
  // check everything first so a bad entry cannot leave a half-submitted schedule
  for (uint32_t i = 0; i < count; ++i) {
    const bfp_request& r = reqs[i];
    if (!op_valid(r.op)) return BFP_E_OP;
    if (!bfp_format_supported(r.f) || !batch_format_ok(r.f)) return BFP_E_FORMAT;
    if (r.arrival_ns < 0 || (i && r.arrival_ns < reqs[i - 1].arrival_ns)) return BFP_E_ARG;
  }
  const int64_t t0 = now_ns();
  for (uint32_t i = 0; i < count; ++i) {
    const int64_t due = t0 + reqs[i].arrival_ns;
    for (;;) {  // sleep while far from the arrival time, spin close to it
      const int64_t left = due - now_ns();
      if (left <= 0) break;
      if (left > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(left - 100000));
      else std::this_thread::yield();
    }
    uint64_t id;
    const bfp_status st = bfp_server_submit(s, reqs[i].op, reqs[i].f, reqs[i].a, reqs[i].b, reqs[i].n, &id);
    if (st != BFP_OK) return st;
    if (i == 0 && first_id) *first_id = id;
  }
  return BFP_OK;
}

bfp_status bfp_server_poll(bfp_server* s, bfp_completion* out, uint32_t max, uint32_t* count) {
  if (!s || !count || (max && !out)) return BFP_E_NULL;
  std::vector<SchedRequest> tmp(max);
  size_t k;
  {
    std::lock_guard<std::mutex> lk(s->sched->mutex());
    k = s->sched->take_completed(tmp.data(), max);
  }
  for (size_t i = 0; i < k; ++i) {
    const SchedRequest& r = tmp[i];
    out[i].req_id = r.id;
    out[i].result = r.c_handle;
    out[i].status = r.status;
    out[i].n = r.n;
    out[i].t_submit_ns = r.t_submit;
    out[i].t_admit_ns = r.t_admit;
    out[i].t_launch_ns = r.t_launch;
    out[i].t_done_ns = r.t_done;
  }
  *count = (uint32_t)k;
  return BFP_OK;
}

bfp_status bfp_server_wait_idle(bfp_server* s, int64_t timeout_ms) {
  if (!s) return BFP_E_NULL;
  const int64_t deadline = now_ns() + timeout_ms * 1000000;
  for (;;) {
    {
      std::lock_guard<std::mutex> lk(s->sched->mutex());
      if (s->sched->idle()) return BFP_OK;
    }
    if (now_ns() > deadline) return BFP_E_TIMEOUT;
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
}

bfp_status bfp_server_view(bfp_server* s, bfp_handle handle, void** bitslice_dev, uint64_t* n) {
  if (!s || !bitslice_dev || !n) return BFP_E_NULL;
  std::lock_guard<std::mutex> lk(s->sched->mutex());
  const Resident* r = s->sched->resident(handle);
  if (!r) return BFP_E_ARG;
  *bitslice_dev = static_cast<uint8_t*>(s->arena) + r->off;
  *n = r->n;
  return BFP_OK;
}

bfp_status bfp_server_get(bfp_server* s, bfp_handle handle, bfp_format f, void* std_dev_out, void* stream) {
  if (!s || !std_dev_out) return BFP_E_NULL;
  uint32_t slot;
  uint64_t off, n;
  {
    std::lock_guard<std::mutex> lk(s->sched->mutex());
    const Resident* r = s->sched->resident(handle);
    if (!r) return BFP_E_ARG;
    if (r->e != f.e || r->m != f.m) return BFP_E_FORMAT;
    off = r->off;
    n = r->n;
    slot = s->sched->pin(handle);  // a concurrent free waits for the unpack
  }
  bfp_status st = bfp_unpack(f, static_cast<uint8_t*>(s->arena) + off, std_dev_out, n, stream);
  if (st == BFP_OK && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) st = BFP_E_HIP;
  {
    std::lock_guard<std::mutex> lk(s->sched->mutex());
    s->sched->unpin(slot);
  }
  return st;
}

bfp_status bfp_server_free(bfp_server* s, bfp_handle handle) {
  if (!s) return BFP_E_NULL;
  std::lock_guard<std::mutex> lk(s->sched->mutex());
  return s->sched->free_resident(handle) ? BFP_OK : BFP_E_ARG;
}

bfp_status bfp_server_stats_get(bfp_server* s, bfp_server_stats* out) {
  if (!s || !out) return BFP_E_NULL;
  std::lock_guard<std::mutex> lk(s->sched->mutex());
  const SchedStats& st = s->sched->stats();
  out->budget = s->sched->capacity();
  out->used = s->sched->used();
  out->high_water = s->sched->high_water();
  out->submitted = st.submitted;
  out->admitted = st.admitted;
  out->completed = st.completed;
  out->ticks = st.ticks;
  out->max_tick_requests = st.max_tick_requests;
  out->max_inflight_ticks = st.max_inflight_ticks;
  out->deferred_budget = st.deferred_budget;
  out->pending = s->sched->pending();
  out->inflight = (uint64_t)s->sched->inflight_requests();
  out->deferred_frees = st.deferred_frees;
  out->cancelled = st.cancelled;
  out->timed_out = st.timed_out;
  out->live_vectors = s->sched->live_residents();
  out->table_slots = s->sched->resident_slots();
  return BFP_OK;
}

}  // extern "C"
