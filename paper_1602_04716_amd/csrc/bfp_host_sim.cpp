// bfp_host_sim.cpp -- the circuits of bfp_circuits.hpp instantiated for the
// host CPU (32- and 64-bit words), to test the netlists against the oracle
// without a GPU, and the gate-count model.  Test-only library: the GPU
// library never loads it and nothing falls back to it.
#include <stdint.h>
#include <string.h>

#include "bfp_circuits.hpp"
#include "bfp_formats.hpp"

// A build may narrow the formats and integer widths it instantiates (the
// sanitizer builds of the tests do, to keep their compile time short); the
// calls return -1 for the others.
#ifndef BFP_SIM_FORMATS
#define BFP_SIM_FORMATS(X) BFP_FOR_EACH_FORMAT(X)
#endif
#ifndef BFP_SIM_WIDE_FORMATS
#define BFP_SIM_WIDE_FORMATS(X) BFP_FOR_EACH_WIDE_FORMAT(X)
#endif
#ifndef BFP_SIM_INT_K
#define BFP_SIM_INT_K(X) BFP_FOR_EACH_INT_K(X)
#endif

namespace {

template <class W>
constexpr int kBits = sizeof(W) * 8;

// Run one circuit over n standard patterns (low 1+e+m bits of uint32 or
// uint64 words).
template <int E, int M, bool RZ, class W, class P>
void run(int op, const P* a, const P* b, P* c, uint64_t n) {
  constexpr int B = 1 + E + M;
  constexpr int WB = kBits<W>;
  const W negb = (op == 1) ? bfp::WordTraits<W>::ones() : bfp::WordTraits<W>::zero();
  for (uint64_t base = 0; base < n; base += WB) {
    W x[B], y[B], z[B];
    for (int k = 0; k < B; ++k) {
      W wx = 0, wy = 0;
      for (int j = 0; j < WB && base + j < n; ++j) {
        wx |= (W)((a[base + j] >> k) & 1u) << j;
        wy |= (W)((b[base + j] >> k) & 1u) << j;
      }
      x[k] = wx;
      y[k] = wy;
    }
    if (op == 2)
      bfp::fp_mul<E, M, RZ, W>(x, y, z);
    else if (op == 3)
      bfp::fp_div<E, M, RZ, W>(x, y, z);
    else
      bfp::fp_add<E, M, RZ, W>(x, y, negb, z);
    for (int j = 0; j < WB && base + j < n; ++j) {
      P v = 0;
      for (int k = 0; k < B; ++k) v |= (P)((z[k] >> j) & 1u) << k;
      c[base + j] = v;
    }
  }
}

template <int E, int M, bool RZ>
unsigned long gates(int op) {
  using bfp::CountW;
  constexpr int B = 1 + E + M;
  CountW x[B], y[B], z[B];
  CountW::counter() = 0;
  if (op == 2)
    bfp::fp_mul<E, M, RZ, CountW>(x, y, z);
  else if (op == 3)
    bfp::fp_div<E, M, RZ, CountW>(x, y, z);
  else
    bfp::fp_add<E, M, RZ, CountW>(x, y, CountW{}, z);
  return CountW::counter();
}

}  // namespace

extern "C" {

// op: 0 add, 1 sub, 2 mul, 3 div; mode: 0 nearest-even, 1 toward zero; wbits 32/64.
// Returns 0, or -1 for a format that is not compiled.
int bfpsim_binop(int op, int e, int m, int mode, int wbits, const uint32_t* a, const uint32_t* b,
                 uint32_t* c, uint64_t n) {
#define BFP_SIM_CASE(EE, MM)                                                             \
  if (e == EE && m == MM) {                                                              \
    if (wbits == 64) {                                                                   \
      if (mode) run<EE, MM, true, uint64_t>(op, a, b, c, n);                             \
      else run<EE, MM, false, uint64_t>(op, a, b, c, n);                                 \
    } else {                                                                             \
      if (mode) run<EE, MM, true, uint32_t>(op, a, b, c, n);                             \
      else run<EE, MM, false, uint32_t>(op, a, b, c, n);                                 \
    }                                                                                    \
    return 0;                                                                            \
  }
  BFP_SIM_FORMATS(BFP_SIM_CASE)
#undef BFP_SIM_CASE
  return -1;
}

// The wide formats on uint64 patterns.
int bfpsim_binop64(int op, int e, int m, int mode, int wbits, const uint64_t* a, const uint64_t* b, uint64_t* c,
                   uint64_t n) {
#define BFP_SIM_CASE(EE, MM)                                                             \
  if (e == EE && m == MM) {                                                              \
    if (wbits == 64) {                                                                   \
      if (mode) run<EE, MM, true, uint64_t>(op, a, b, c, n);                             \
      else run<EE, MM, false, uint64_t>(op, a, b, c, n);                                 \
    } else {                                                                             \
      if (mode) run<EE, MM, true, uint32_t>(op, a, b, c, n);                             \
      else run<EE, MM, false, uint32_t>(op, a, b, c, n);                                 \
    }                                                                                    \
    return 0;                                                                            \
  }
  BFP_SIM_WIDE_FORMATS(BFP_SIM_CASE)
#undef BFP_SIM_CASE
  return -1;
}

// Gates of one circuit instance (one word group), constants folded.
long bfpsim_gate_count(int op, int e, int m, int mode) {
#define BFP_GC_CASE(EE, MM) \
  if (e == EE && m == MM) return (long)(mode ? gates<EE, MM, true>(op) : gates<EE, MM, false>(op));
  BFP_SIM_FORMATS(BFP_GC_CASE)
  BFP_SIM_WIDE_FORMATS(BFP_GC_CASE)
#undef BFP_GC_CASE
  return -1;
}

// Figure 2: 13-bit bitslice integer adder over 32 lanes.  a, b, r hold 13
// plane words each (plane k = bit k of the 32 lane values).
void bfpsim_ripple_add13(const uint32_t* a, const uint32_t* b, uint32_t* r) {
  bfp::ripple_add<13, uint32_t>(a, b, r);
}

}  // extern "C"

#include "bfp_int_circuits.hpp"

namespace {
template <int K, int OP, int KIND, class W>
void run_int(const uint32_t* a, const uint32_t* b, uint32_t* c, uint64_t n) {
  constexpr int WB = kBits<W>;
  for (uint64_t base = 0; base < n; base += WB) {
    W x[K], y[K], z[K];
    for (int k = 0; k < K; ++k) {
      W wx = 0, wy = 0;
      for (int j = 0; j < WB && base + j < n; ++j) {
        wx |= (W)((a[base + j] >> k) & 1u) << j;
        wy |= (W)((b[base + j] >> k) & 1u) << j;
      }
      x[k] = wx;
      y[k] = wy;
    }
    bfp::int_circuit<K, OP, KIND, W>(x, y, z);
    for (int j = 0; j < WB && base + j < n; ++j) {
      uint32_t v = 0;
      for (int k = 0; k < K; ++k) v |= (uint32_t)((z[k] >> j) & 1u) << k;
      c[base + j] = v;
    }
  }
}

template <int K, int OP, int KIND>
long int_gates() {
  bfp::CountW x[K], y[K], z[K];
  bfp::CountW::counter() = 0;
  bfp::int_circuit<K, OP, KIND, bfp::CountW>(x, y, z);
  return (long)bfp::CountW::counter();
}
}  // namespace

extern "C" {
// k-bit integer op (0 add, 1 sub, 2 mul), kind 0 wrap / 1 unsigned / 2 signed
// saturation, on 32- or 64-bit host words.  Returns 0, or -1 for bad k/op/kind.
int bfpsim_int_binop(int op, int k, int kind, int wbits, const uint32_t* a, const uint32_t* b, uint32_t* c,
                     uint64_t n) {
  if (op < 0 || op > 2 || kind < 0 || kind > 2) return -1;
#define BFP_SIM_INT_OPK(KK, OP, KD)                                      \
  if (op == OP && kind == KD) {                                          \
    if (wbits == 64) run_int<KK, OP, KD, uint64_t>(a, b, c, n);          \
    else run_int<KK, OP, KD, uint32_t>(a, b, c, n);                      \
    return 0;                                                            \
  }
#define BFP_SIM_INT_CASE(KK)                                                                          \
  if (k == KK) {                                                                                      \
    BFP_SIM_INT_OPK(KK, 0, 0) BFP_SIM_INT_OPK(KK, 0, 1) BFP_SIM_INT_OPK(KK, 0, 2)                    \
    BFP_SIM_INT_OPK(KK, 1, 0) BFP_SIM_INT_OPK(KK, 1, 1) BFP_SIM_INT_OPK(KK, 1, 2)                    \
    BFP_SIM_INT_OPK(KK, 2, 0) BFP_SIM_INT_OPK(KK, 2, 1) BFP_SIM_INT_OPK(KK, 2, 2)                    \
  }
  BFP_SIM_INT_K(BFP_SIM_INT_CASE)
#undef BFP_SIM_INT_CASE
#undef BFP_SIM_INT_OPK
  return -1;
}

long bfpsim_int_gate_count(int op, int k, int kind) {
#define BFP_GC_INT_OPK(KK, OP, KD) \
  if (op == OP && kind == KD) return int_gates<KK, OP, KD>();
#define BFP_GC_INT_CASE(KK)                                                                 \
  if (k == KK) {                                                                            \
    BFP_GC_INT_OPK(KK, 0, 0) BFP_GC_INT_OPK(KK, 0, 1) BFP_GC_INT_OPK(KK, 0, 2)             \
    BFP_GC_INT_OPK(KK, 1, 0) BFP_GC_INT_OPK(KK, 1, 1) BFP_GC_INT_OPK(KK, 1, 2)             \
    BFP_GC_INT_OPK(KK, 2, 0) BFP_GC_INT_OPK(KK, 2, 1) BFP_GC_INT_OPK(KK, 2, 2)             \
  }
  BFP_SIM_INT_K(BFP_GC_INT_CASE)
#undef BFP_GC_INT_CASE
#undef BFP_GC_INT_OPK
  return -1;
}
}  // extern "C"

#include "bfp_transpose.hpp"

extern "C" {
// 32 elements of C bytes (8C dwords) <-> 8C plane words, as the GPU kernels do it.
int bfpsim_transpose(int C, int inverse, const uint32_t* in, uint32_t* out) {
  switch (C * 2 + (inverse ? 1 : 0)) {
    case 2: bfp::transpose_pack<1>(in, out); return 0;
    case 3: bfp::transpose_unpack<1>(in, out); return 0;
    case 4: bfp::transpose_pack<2>(in, out); return 0;
    case 5: bfp::transpose_unpack<2>(in, out); return 0;
    case 8: bfp::transpose_pack<4>(in, out); return 0;
    case 9: bfp::transpose_unpack<4>(in, out); return 0;
    default: return -1;
  }
}
}

// ---------------------------------------------------------------------------
// Serving scheduler core with a fake executor whose ticks complete only when
// the test releases them (the host forces every condition: full budget, full
// slots, both streams busy, launch failure).
// ---------------------------------------------------------------------------
#include <deque>

#include "bfp_layout.hpp"
#include "bfp_sched.hpp"

namespace {
struct FakeExecutor {
  static constexpr int kStreams = 2;
  std::deque<std::vector<bfp::SchedRequest>> running;
  int releasable = 0;
  int fail_next = 0;
  int launch(const std::vector<bfp::SchedRequest>& reqs) {
    if (fail_next) {
      fail_next = 0;
      return -5;
    }
    running.push_back(reqs);
    return 0;
  }
  bool poll_done(std::vector<bfp::SchedRequest>* out) {
    if (running.empty() || releasable <= 0) return false;
    *out = running.front();
    running.pop_front();
    releasable--;
    return true;
  }
};
struct SimServer {
  FakeExecutor ex;
  bfp::Scheduler<FakeExecutor> sched;
  uint64_t next_id = 1;
  std::vector<bfp::SchedRequest> batch;  // collected, not yet launched
  SimServer(uint64_t budget, int slots) : sched(ex, budget, slots) {}
};
}  // namespace

extern "C" {
void* simsrv_create(uint64_t budget, int slots) { return new SimServer(budget, slots); }
void simsrv_destroy(void* p) { delete static_cast<SimServer*>(p); }
// A resident vector of format (5,10) with n elements taking `bytes`; 0 if
// the arena is full.
uint64_t simsrv_put(void* p, uint64_t bytes, uint64_t n) {
  auto* s = static_cast<SimServer*>(p);
  uint64_t h, off;
  return s->sched.alloc_resident(bytes, 5, 10, n, &h, &off) ? h : 0;
}
int simsrv_free(void* p, uint64_t h) { return static_cast<SimServer*>(p)->sched.free_resident(h) ? 0 : -1; }
// Arena offset of a live handle, or -1.
int64_t simsrv_offset(void* p, uint64_t h) {
  const bfp::Resident* r = static_cast<SimServer*>(p)->sched.resident(h);
  return r ? (int64_t)r->off : -1;
}
// Queue a (5,10) add of the first n elements of a and b with a result of
// c_bytes; returns the request id, or the negative status of a rejected
// submission.
int64_t simsrv_submit(void* p, uint64_t a, uint64_t b, uint64_t n, uint64_t c_bytes) {
  auto* s = static_cast<SimServer*>(p);
  bfp::SchedRequest r;
  r.id = s->next_id;
  r.e = 5;
  r.m = 10;
  r.n = n;
  r.c_bytes = c_bytes;
  const int st = s->sched.submit(r, a, b);
  if (st != 0) return st;
  return (int64_t)s->next_id++;
}
int simsrv_cancel(void* p, uint64_t id) { return static_cast<SimServer*>(p)->sched.cancel(id); }
void simsrv_set_timeout(void* p, int64_t ns) { static_cast<SimServer*>(p)->sched.set_queue_timeout(ns); }
void simsrv_set_tick_limit(void* p, uint64_t bytes) { static_cast<SimServer*>(p)->sched.set_tick_limit(bytes); }
int simsrv_step(void* p) { return static_cast<SimServer*>(p)->sched.step() ? 1 : 0; }
// The serving worker's split step: collect (returns the batch size), then,
// after any number of other calls, launch the batch and commit it.
int simsrv_collect(void* p) {
  auto* s = static_cast<SimServer*>(p);
  s->sched.collect(&s->batch);
  return (int)s->batch.size();
}
void simsrv_launch_commit(void* p) {
  auto* s = static_cast<SimServer*>(p);
  if (s->batch.empty()) return;
  const int st = s->ex.launch(s->batch);
  s->sched.commit(&s->batch, st);
}
void simsrv_release(void* p, int k) { static_cast<SimServer*>(p)->ex.releasable += k; }
void simsrv_fail_next(void* p) { static_cast<SimServer*>(p)->ex.fail_next = 1; }
int simsrv_running_ticks(void* p) { return (int)static_cast<SimServer*>(p)->ex.running.size(); }
// Arena offsets read by the running ticks' requests (a and b of each), up to
// max; returns the count.
int simsrv_running_operands(void* p, uint64_t* offs, int max) {
  auto* s = static_cast<SimServer*>(p);
  int k = 0;
  for (const auto& tick : s->ex.running)
    for (const auto& r : tick) {
      if (k < max) offs[k] = r.a_off;
      k++;
      if (k < max) offs[k] = r.b_off;
      k++;
    }
  return k;
}
// completions: ids[i], handles[i], status[i]; returns count
int simsrv_take(void* p, uint64_t* ids, uint64_t* handles, int32_t* status, int max) {
  auto* s = static_cast<SimServer*>(p);
  std::vector<bfp::SchedRequest> tmp((size_t)max);
  const size_t k = s->sched.take_completed(tmp.data(), (size_t)max);
  for (size_t i = 0; i < k; ++i) {
    ids[i] = tmp[i].id;
    handles[i] = tmp[i].c_handle;
    status[i] = tmp[i].status;
  }
  return (int)k;
}
// used, high_water, capacity, pending, inflight requests, ticks, max_tick_requests,
// max_inflight_ticks, deferred_budget, admitted, completed, deferred_frees,
// cancelled, timed_out, live vectors, table slots
void simsrv_stats(void* p, uint64_t* out) {
  auto* s = static_cast<SimServer*>(p);
  const bfp::SchedStats& st = s->sched.stats();
  out[0] = s->sched.used();
  out[1] = s->sched.high_water();
  out[2] = s->sched.capacity();
  out[3] = s->sched.pending();
  out[4] = (uint64_t)s->sched.inflight_requests();
  out[5] = st.ticks;
  out[6] = st.max_tick_requests;
  out[7] = st.max_inflight_ticks;
  out[8] = st.deferred_budget;
  out[9] = st.admitted;
  out[10] = st.completed;
  out[11] = st.deferred_frees;
  out[12] = st.cancelled;
  out[13] = st.timed_out;
  out[14] = s->sched.live_residents();
  out[15] = s->sched.resident_slots();
}

// Layout rules as the kernels use them.
uint64_t simlayout_gpad(uint64_t n) { return bfp::gpad_of(n); }
uint64_t simlayout_data_words(uint64_t n) { return bfp::data_words(n); }
uint32_t simlayout_word_mask(uint64_t w, uint64_t n) { return bfp::word_mask(w, n); }

// Arena alone
void* simarena_create(uint64_t cap) { return new bfp::Arena(cap); }
void simarena_destroy(void* a) { delete static_cast<bfp::Arena*>(a); }
int64_t simarena_alloc(void* a, uint64_t bytes) {
  uint64_t off;
  return static_cast<bfp::Arena*>(a)->alloc(bytes, &off) ? (int64_t)off : -1;
}
uint64_t simarena_release(void* a, uint64_t off) { return static_cast<bfp::Arena*>(a)->release(off); }
void simarena_stats(void* a, uint64_t* out) {
  auto* ar = static_cast<bfp::Arena*>(a);
  out[0] = ar->used();
  out[1] = ar->high_water();
  out[2] = ar->capacity();
  out[3] = ar->live_count();
  out[4] = ar->free_ranges();
}
}
