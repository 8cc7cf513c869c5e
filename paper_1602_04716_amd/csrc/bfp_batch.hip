// bfp_batch.hip -- many vectors of mixed formats and lengths in one
// persistent kernel, captured once in a HIP graph.
//
// Plan (host): every task (a op b -> c on bitslice vectors of one format) is
// cut into chunks of at most kChunkWords words per plane; chunks are grouped
// by circuit variant so that consecutive chunks run the same code (one
// instruction-cache footprint at a time), the variants taken in decreasing
// time per word so that the slowest chunks start first and the grid drains
// on short ones, and, within a variant, longest task first.  Descriptors go
// to device memory once.
//
// Device: two persistent kernels, one for the add/sub and mul circuits and
// one for the dividers (whose registers would otherwise lower the first
// kernel's occupancy), each compiled for a fixed occupancy and launched on a
// grid sized to the GPU's resident capacity for it.  Each block takes the
// next chunk index of its class from an atomic counter, reads the chunk's
// task, and switches (block-uniformly) to the compiled circuit of the task's
// (e, m, operation class, rounding mode).  The counters are cleared by a
// one-thread kernel at the head of the graph, so each replay starts at chunk 0.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "bfp.h"
#include "bfp_formats.hpp"
#include "bfp_batch.hpp"
#include "bfp_kernels.hpp"
#include "bfp_layout.hpp"

namespace bfp {

// One chunk of one task: the block's threads stride over the chunk's words,
// one word per lane (two would double every circuit's registers).
//
// A task may compute a prefix of longer operands (the serving loop does),
// and the operands' plane strides need not cover the result's: the stride
// rule is not monotonic in the length.  So operand words are read only up to
// the last word holding an element below n, which every operand plane holds:
// words past it read that word again, and their results are cleared.  Bits
// of elements at or past n are cleared in every result word, so c's padding
// is zero whatever the operands hold there (division would otherwise map
// zero padding to NaN).  The clamp and the mask are branch-free: a branch
// around the loads, or around the mask, raised the kernel's registers from
// about 130 to 235 VGPRs (measured on the (8,23) multiplier).
template <int E, int M, bool RZ, int OPC>
__device__ __forceinline__ void batch_chunk(const BatchTask& tk, uint64_t w0, uint32_t nw) {
  constexpr int B = 1 + E + M;
  constexpr int R = 1;
  // word offsets fit in 32 bits: n <= 2^36 elements gives at most 2^31 + 256 words per plane
  const uint32_t end = (uint32_t)w0 + nw;
  const uint32_t wlast = (uint32_t)(data_words(tk.n) - 1);  // last word holding an element below n
  const uint32_t wfull = (uint32_t)(tk.n >> 5);              // words wholly below n
  const uint32_t tail = (1u << (uint32_t)(tk.n & 31u)) - 1u;  // elements below n in word wfull
  for (uint32_t off = (uint32_t)w0 + threadIdx.x; off < end; off += blockDim.x) {
    const uint32_t src = off < wlast ? off : wlast;
    WordR<R> x[B], y[B], z[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      x[k] = ld_words<R>(tk.a + (uint64_t)k * tk.sa + src);
      y[k] = ld_words<R>(tk.b + (uint64_t)k * tk.sb + src);
    }
    circuit<E, M, RZ, OPC, R>(x, y, tk.negb, z);
    const uint32_t mk = off < wfull ? 0xFFFFFFFFu : (off == wfull ? tail : 0u);
#pragma unroll
    for (int k = 0; k < B; ++k) z[k].w[0] &= mk;
#pragma unroll
    for (int k = 0; k < B; ++k) st_words<R>(tk.c + (uint64_t)k * tk.sc + off, z[k]);
  }
}

__global__ void k_batch_reset(uint32_t* counter) {
  if (threadIdx.x < kBatchClasses && blockIdx.x == 0) counter[threadIdx.x] = 0u;
}

// Waves per SIMD each class kernel is compiled for.
// Waves per SIMD each class kernel is compiled for.  Without the target
// the compiler schedules the merged switch of 160 circuits for one wave per
// SIMD (256 VGPRs); at three, the add/sub/mul kernel keeps 168 VGPRs and
// spills a few registers of its heaviest circuits to scratch, which measured
// no slower than the unspilled alternatives.
template <int CLS>
struct ClassWaves {
  static constexpr int value = CLS == 0 ? 3 : 2;
};

// Persistent kernel of register class CLS over chunks [first, first +
// nchunks) of the chunk table, or, when `index` is not null, over the
// index's chunks of class CLS: task t owns chunks [prefix[t], prefix[t+1]),
// cut at kChunkWords words in task order.  Thread 0 takes the next chunk from
// the counter and resolves it; the block then runs it.
template <int CLS>
__global__ void __launch_bounds__(kBatchBlock) __attribute__((amdgpu_waves_per_eu(ClassWaves<CLS>::value)))
k_batch(const BatchTask* tasks, const BatchChunk* chunks, uint32_t first, uint32_t nchunks, uint32_t* counter,
        const BatchIndex* index, const uint64_t* prefix) {
  __shared__ BatchChunk s_ch;
  __shared__ uint32_t s_next;
  const uint64_t total = index ? index->total[CLS] : nchunks;
  for (;;) {
    if (threadIdx.x == 0) {
      const uint32_t ci = atomicAdd(counter, 1u);
      s_next = ci;
      if (ci < total) {
        if (index) {
          uint32_t lo = 0, hi = index->ntasks;  // largest t with prefix[t] <= ci
          while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) / 2;
            if (prefix[mid] <= ci) lo = mid;
            else hi = mid;
          }
          const uint64_t w0 = (ci - prefix[lo]) * (uint64_t)kChunkWords;
          s_ch.task = lo;
          s_ch.w0 = w0;
          s_ch.nwords = (uint32_t)min((uint64_t)kChunkWords, tasks[lo].words - w0);
        } else {
          s_ch = chunks[first + ci];
        }
      }
    }
    __syncthreads();
    const uint32_t ci = s_next;
    const BatchChunk ch = s_ch;
    __syncthreads();
    if (ci >= total) break;  // every block sees the counter pass the total and leaves
    const BatchTask tk = tasks[ch.task];
    switch (tk.variant) {
#define BFP_BATCH_VARIANT(EE, MM, OPC, RZ)                                          \
  case (format_index(EE, MM) * kOpClasses + OPC) * 2 + RZ:                          \
    if constexpr (variant_class(MM, OPC) == CLS) batch_chunk<EE, MM, RZ, OPC>(tk, ch.w0, ch.nwords); \
    break;
#define BFP_BATCH_CASE(EE, MM)                                                                           \
  BFP_BATCH_VARIANT(EE, MM, 0, false) BFP_BATCH_VARIANT(EE, MM, 0, true) BFP_BATCH_VARIANT(EE, MM, 1, false) \
  BFP_BATCH_VARIANT(EE, MM, 1, true) BFP_BATCH_VARIANT(EE, MM, 2, false) BFP_BATCH_VARIANT(EE, MM, 2, true)
      BFP_FOR_EACH_FORMAT(BFP_BATCH_CASE)
#undef BFP_BATCH_CASE
#undef BFP_BATCH_VARIANT
      default: break;
    }
  }
}

constexpr int kBatchFormats = 40;  // format_index covers 5 exponent x 8 mantissa widths

bool batch_format_ok(const bfp_format& f) { return format_index(f.e, f.m) >= 0 && f.round <= 1; }

bool batch_task(const void* a, uint64_t na, const void* b, uint64_t nb, void* c, uint64_t n, bfp_format f, int op,
                BatchTask* out) {
  if (!op_valid(op)) return false;
  return make_batch_task(a, na, b, nb, c, n, f, op, out);
}

// Relative time per word of each variant's circuit: the larger of its HBM
// traffic (two operands and a result of B planes, 4 bytes a plane-word, at
// 8 TB/s: 1.5 ps per plane) and its gates (one 32-bit lane operation each, at
// 256 CUs x 64 lanes x 2.4 GHz: 0.025 ps per gate), so one plane of traffic
// weighs as much as 59 gates.  Computed once, from the circuits' gate counts.
static const std::vector<uint32_t>& variant_cost() {
  static const std::vector<uint32_t> cost = [] {
    std::vector<uint32_t> c(kBatchFormats * kOpClasses * 2, 0);
    const int ops[kOpClasses] = {BFP_ADD, BFP_MUL, BFP_DIV};
#define BFP_COST_CASE(EE, MM)                                                          \
  for (int oc = 0; oc < kOpClasses; ++oc)                                              \
    for (int rz = 0; rz < 2; ++rz) {                                                   \
      const long g = bfp_gate_count(ops[oc], bfp_format{EE, MM, (uint8_t)rz, 0});      \
      c[(format_index(EE, MM) * kOpClasses + oc) * 2 + rz] =                           \
          (uint32_t)std::max<long>(59L * (1 + EE + MM), g);                            \
    }
    BFP_FOR_EACH_FORMAT(BFP_COST_CASE)
#undef BFP_COST_CASE
    return c;
  }();
  return cost;
}

int task_class(const BatchTask& t) {
  const uint32_t fo = t.variant / 2;  // format index * kOpClasses + op class
  static const int kM[8] = {1, 2, 3, 5, 7, 10, 15, 23};
  return variant_class(kM[(fo / kOpClasses) % 8], (int)(fo % kOpClasses));
}

void batch_chunks(const std::vector<BatchTask>& dt, std::vector<BatchChunk>* out) {
  // tasks by kernel class, then variants by decreasing time per word (ties
  // by variant); within a variant, longer tasks first, then by position; each
  // task's chunks follow in word order (sorting the tasks, not the chunks,
  // keeps the host's share of a serving tick small)
  const std::vector<uint32_t>& cost = variant_cost();
  std::vector<uint32_t> order(dt.size());
  std::vector<int> cls(dt.size());
  for (uint32_t i = 0; i < (uint32_t)dt.size(); ++i) {
    order[i] = i;
    cls[i] = task_class(dt[i]);
  }
  std::sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
    const uint32_t vx = dt[x].variant, vy = dt[y].variant;
    if (cls[x] != cls[y]) return cls[x] < cls[y];
    if (cost[vx] != cost[vy]) return cost[vx] > cost[vy];
    if (vx != vy) return vx < vy;
    if (dt[x].words != dt[y].words) return dt[x].words > dt[y].words;
    return x < y;
  });
  std::vector<BatchChunk>& chunks = *out;
  chunks.clear();
  for (uint32_t i : order) {
    for (uint64_t w = 0; w < dt[i].words; w += kChunkWords) {
      BatchChunk ch;
      ch.w0 = w;
      ch.task = i;
      ch.nwords = (uint32_t)std::min<uint64_t>(kChunkWords, dt[i].words - w);
      chunks.push_back(ch);
    }
  }
}

template <int CLS>
static int resident_blocks_of(int cus) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<CLS>, kBatchBlock, 0) != hipSuccess) return 0;
  return (per_cu < 1 ? 1 : per_cu) * cus;
}

int batch_resident_blocks(int c) {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  switch (c) {
    case 0: return resident_blocks_of<0>(prop.multiProcessorCount);
    case 1: return resident_blocks_of<1>(prop.multiProcessorCount);
    default: return 0;
  }
}

BatchSplit batch_split(const std::vector<BatchTask>& tasks, const std::vector<BatchChunk>& chunks, const int* cap) {
  BatchSplit sp;
  for (const BatchChunk& ch : chunks) sp.n[task_class(tasks[ch.task])]++;
  uint32_t first = 0;
  for (int c = 0; c < kBatchClasses; ++c) {
    sp.first[c] = first;
    first += sp.n[c];
    sp.grid[c] = (unsigned)std::min<uint64_t>((uint64_t)std::max(cap[c], 1), sp.n[c]);
  }
  return sp;
}

template <int CLS>
static void launch_class(const BatchTask* d_tasks, const BatchChunk* d_chunks, const BatchSplit& sp,
                         uint32_t* d_counter, hipStream_t s) {
  if (sp.n[CLS] > 0)
    hipLaunchKernelGGL((k_batch<CLS>), dim3(sp.grid[CLS]), dim3(kBatchBlock), 0, s, d_tasks, d_chunks,
                       sp.first[CLS], sp.n[CLS], d_counter + CLS, nullptr, nullptr);
}

hipError_t batch_launch(const BatchTask* d_tasks, const BatchChunk* d_chunks, const BatchSplit& sp,
                        uint32_t* d_counter, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, d_counter);
  launch_class<0>(d_tasks, d_chunks, sp, d_counter, s);
  launch_class<1>(d_tasks, d_chunks, sp, d_counter, s);
  return hipGetLastError();
}

}  // namespace bfp

using namespace bfp;

struct bfp_batch_plan {
  int device = 0;
  std::vector<bfp_task> tasks;  // as given (for the per-vector baseline)
  BatchTask* d_tasks = nullptr;
  BatchChunk* d_chunks = nullptr;
  uint32_t* d_counter = nullptr;
  uint32_t nchunks = 0;
  BatchSplit split;
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t pv_graph = nullptr;      // the per-vector launches, captured on first use
  hipGraphExec_t pv_exec = nullptr;
  uint64_t words_total = 0;  // sum over tasks of B * gpad (per operand)
  std::mutex mu;
};

namespace {

void plan_free(bfp_batch_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->pv_exec) (void)hipGraphExecDestroy(p->pv_exec);
  if (p->pv_graph) (void)hipGraphDestroy(p->pv_graph);
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  if (p->d_tasks) (void)hipFree(p->d_tasks);
  if (p->d_chunks) (void)hipFree(p->d_chunks);
  if (p->d_counter) (void)hipFree(p->d_counter);
  delete p;
}

}  // namespace

extern "C" {

bfp_status bfp_batch_plan_create(const bfp_task* tasks, uint32_t count, bfp_batch_plan** out) {
  if (!out) return BFP_E_NULL;
  *out = nullptr;
  if (count == 0 || !tasks) return count == 0 ? BFP_E_ARG : BFP_E_NULL;
  std::vector<BatchTask> dt(count);
  std::vector<BatchChunk> chunks;
  uint64_t words_total = 0;
  for (uint32_t i = 0; i < count; ++i) {
    const bfp_task& t = tasks[i];
    if (!bfp_format_supported(t.f)) return BFP_E_FORMAT;
    if (!op_valid(t.op)) return BFP_E_OP;
    if (t.n == 0 || t.n > (1ull << 36)) return BFP_E_ARG;
    if (!t.a || !t.b || !t.c) return BFP_E_NULL;
    if (((uintptr_t)t.a | (uintptr_t)t.b | (uintptr_t)t.c) & 15u) return BFP_E_ALIGN;
    if (!batch_task(t.a, t.n, t.b, t.n, t.c, t.n, t.f, t.op, &dt[i])) return BFP_E_FORMAT;
    words_total += (uint64_t)(1 + t.f.e + t.f.m) * dt[i].words;
  }
  batch_chunks(dt, &chunks);
  if (chunks.size() >= 0xFFFFFFF0ull) return BFP_E_ARG;

  bfp_batch_plan* p = new (std::nothrow) bfp_batch_plan();
  if (!p) return BFP_E_NOMEM;
  p->tasks.assign(tasks, tasks + count);
  p->nchunks = (uint32_t)chunks.size();
  p->words_total = words_total;
  if (hipGetDevice(&p->device) != hipSuccess) {
    plan_free(p);
    return BFP_E_NODEV;
  }
  if (hipMalloc(&p->d_tasks, sizeof(BatchTask) * dt.size()) != hipSuccess ||
      hipMalloc(&p->d_chunks, sizeof(BatchChunk) * chunks.size()) != hipSuccess ||
      hipMalloc(&p->d_counter, 256) != hipSuccess) {
    plan_free(p);
    return BFP_E_NOMEM;
  }
  if (hipMemcpy(p->d_tasks, dt.data(), sizeof(BatchTask) * dt.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->d_chunks, chunks.data(), sizeof(BatchChunk) * chunks.size(), hipMemcpyHostToDevice) !=
          hipSuccess) {
    plan_free(p);
    return BFP_E_HIP;
  }
  // resident grids: as many blocks of each class kernel as fit on the device at once
  int cap[kBatchClasses];
  for (int c = 0; c < kBatchClasses; ++c) {
    cap[c] = batch_resident_blocks(c);
    if (cap[c] <= 0) {
      plan_free(p);
      return BFP_E_HIP;
    }
  }
  p->split = batch_split(dt, chunks, cap);
  // capture reset + persistent kernel once
  if (hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking) != hipSuccess) {
    plan_free(p);
    return BFP_E_HIP;
  }
  hipError_t e = hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const hipError_t le = batch_launch(p->d_tasks, p->d_chunks, p->split, p->d_counter, p->capture_stream);
    e = hipStreamEndCapture(p->capture_stream, &p->graph);
    if (le != hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    plan_free(p);
    return BFP_E_HIP;
  }
  *out = p;
  return BFP_OK;
}

bfp_status bfp_batch_run(bfp_batch_plan* plan, void* stream) {
  if (!plan) return BFP_E_NULL;
  std::lock_guard<std::mutex> lk(plan->mu);
  return hipGraphLaunch(plan->exec, (hipStream_t)stream) == hipSuccess ? BFP_OK : BFP_E_HIP;
}

bfp_status bfp_batch_run_eager(bfp_batch_plan* plan, void* stream) {
  if (!plan) return BFP_E_NULL;
  std::lock_guard<std::mutex> lk(plan->mu);
  return batch_launch(plan->d_tasks, plan->d_chunks, plan->split, plan->d_counter, (hipStream_t)stream) ==
                 hipSuccess
             ? BFP_OK
             : BFP_E_HIP;
}

bfp_status bfp_batch_run_per_vector(bfp_batch_plan* plan, void* stream) {
  if (!plan) return BFP_E_NULL;
  for (const bfp_task& t : plan->tasks) {
    const bfp_status st = bfp_binop(t.op, t.f, t.a, t.b, t.c, t.n, stream);
    if (st != BFP_OK) return st;
  }
  return BFP_OK;
}

bfp_status bfp_batch_run_per_vector_graph(bfp_batch_plan* plan, void* stream) {
  if (!plan) return BFP_E_NULL;
  std::lock_guard<std::mutex> lk(plan->mu);
  if (!plan->pv_exec) {
    // capture the per-vector launches once, on the plan's own stream
    hipError_t e = hipStreamBeginCapture(plan->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return BFP_E_HIP;
    bfp_status st = BFP_OK;
    for (const bfp_task& t : plan->tasks) {
      st = bfp_binop(t.op, t.f, t.a, t.b, t.c, t.n, plan->capture_stream);
      if (st != BFP_OK) break;
    }
    e = hipStreamEndCapture(plan->capture_stream, &plan->pv_graph);
    if (st != BFP_OK) return st;
    if (e == hipSuccess) e = hipGraphInstantiate(&plan->pv_exec, plan->pv_graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return BFP_E_HIP;
  }
  return hipGraphLaunch(plan->pv_exec, (hipStream_t)stream) == hipSuccess ? BFP_OK : BFP_E_HIP;
}

bfp_status bfp_batch_plan_info(const bfp_batch_plan* plan, uint32_t* nchunks, uint32_t* grid,
                               uint64_t* words_per_operand) {
  if (!plan) return BFP_E_NULL;
  if (nchunks) *nchunks = plan->nchunks;
  if (grid) {
    unsigned g = 0;
    for (int c = 0; c < kBatchClasses; ++c) g = plan->split.grid[c] > g ? plan->split.grid[c] : g;
    *grid = g;
  }
  if (words_per_operand) *words_per_operand = plan->words_total;
  return BFP_OK;
}

void bfp_batch_plan_destroy(bfp_batch_plan* plan) { plan_free(plan); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free batched launch: descriptors built on the device into a
// static scratch array, for callers that cannot allocate.
// ---------------------------------------------------------------------------
namespace bfp {
namespace {

constexpr uint32_t kNoallocMaxTasks = 16384;
constexpr size_t kNoallocTasksOff = 256;  // after the BatchIndex header
constexpr size_t kNoallocPrefixOff = kNoallocTasksOff + sizeof(BatchTask) * kNoallocMaxTasks;
constexpr size_t kNoallocPrefixWords = kNoallocMaxTasks + 1;  // per class
constexpr size_t kNoallocBytes = kNoallocPrefixOff + kBatchClasses * sizeof(uint64_t) * kNoallocPrefixWords;
static_assert(sizeof(BatchIndex) <= kNoallocTasksOff, "index header must fit before the tasks");
static_assert(kNoallocPrefixOff % 256 == 0, "prefix arrays 256-byte aligned");
// Chunk counters must stay below 2^32 (uint32 counters).
constexpr uint64_t kNoallocMaxChunks = 0xFFF00000ull;

// Index header, task table and the class kernels' chunk prefix arrays: about
// 1.4 MB per device, held until the process ends.  In host code this name
// is a stand-in, not a device address: host code uses the address from
// hipGetSymbolAddress (noalloc_device).
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

// First invalid task's error, checked in the same order as
// bfp_batch_plan_create checks a task on the host.
__device__ int32_t task_error(const bfp_task& t) {
  if (t.f.pad != 0 || t.f.round > 1 || format_index(t.f.e, t.f.m) < 0) return BFP_E_FORMAT;
  if (t.op != BFP_ADD && t.op != BFP_SUB && t.op != BFP_MUL && t.op != BFP_DIV) return BFP_E_OP;
  if (t.n == 0 || t.n > (1ull << 36)) return BFP_E_ARG;
  if (!t.a || !t.b || !t.c) return BFP_E_NULL;
  if (((uintptr_t)t.a | (uintptr_t)t.b | (uintptr_t)t.c) & 15u) return BFP_E_ALIGN;
  return BFP_OK;
}

// One block: validate the tasks, write their descriptors and each class's
// exclusive chunk prefix (block scan in tiles of 1024 tasks with a running
// carry), reset the counters, and report the status.  Any invalid task
// leaves every total 0, so nothing runs.
__global__ void __launch_bounds__(1024) k_noalloc_setup(const bfp_task* in, uint32_t count, unsigned char* scr,
                                                        int32_t* status_out) {
  BatchIndex* idx = reinterpret_cast<BatchIndex*>(scr);
  BatchTask* tasks = reinterpret_cast<BatchTask*>(scr + kNoallocTasksOff);
  uint64_t* prefix = reinterpret_cast<uint64_t*>(scr + kNoallocPrefixOff);  // [class][count + 1]
  __shared__ uint64_t s_scan[kBatchClasses][1024];
  __shared__ uint64_t s_carry[kBatchClasses];
  __shared__ uint32_t s_bad;
  const uint32_t tid = threadIdx.x;
  if (tid < kBatchClasses) s_carry[tid] = 0;
  if (tid == 0) s_bad = count;
  __syncthreads();
  for (uint32_t base = 0; base < count; base += 1024) {
    const uint32_t i = base + tid;
    uint64_t cnt[kBatchClasses] = {};
    if (i < count) {
      const bfp_task t = in[i];
      BatchTask bt;
      if (task_error(t) != BFP_OK || !make_batch_task(t.a, t.n, t.b, t.n, t.c, t.n, t.f, t.op, &bt)) {
        atomicMin(&s_bad, i);
      } else {
        tasks[i] = bt;
        const int opc = t.op == BFP_MUL ? 1 : (t.op == BFP_DIV ? 2 : 0);
        cnt[variant_class(t.f.m, opc)] = (bt.words + kChunkWords - 1) / kChunkWords;
      }
    }
#pragma unroll
    for (int c = 0; c < kBatchClasses; ++c) s_scan[c][tid] = cnt[c];
    __syncthreads();
    for (uint32_t d = 1; d < 1024; d <<= 1) {  // inclusive Hillis-Steele scan
      uint64_t x[kBatchClasses];
#pragma unroll
      for (int c = 0; c < kBatchClasses; ++c) x[c] = tid >= d ? s_scan[c][tid - d] : 0;
      __syncthreads();
#pragma unroll
      for (int c = 0; c < kBatchClasses; ++c) s_scan[c][tid] += x[c];
      __syncthreads();
    }
    if (i < count) {
#pragma unroll
      for (int c = 0; c < kBatchClasses; ++c) prefix[c * kNoallocPrefixWords + i] = s_carry[c] + s_scan[c][tid] - cnt[c];
    }
    __syncthreads();
    if (tid < kBatchClasses) s_carry[tid] += s_scan[tid][1023];
    __syncthreads();
  }
  if (tid == 0) {
    int32_t st = BFP_OK;
    if (s_bad < count) {
      st = task_error(in[s_bad]);
      if (st == BFP_OK) st = BFP_E_FORMAT;  // a task the batch kernels do not compile
    }
    for (int c = 0; c < kBatchClasses; ++c) {
      prefix[c * kNoallocPrefixWords + count] = s_carry[c];
      if (s_carry[c] >= kNoallocMaxChunks && st == BFP_OK) st = BFP_E_ARG;
    }
    for (int c = 0; c < kBatchClasses; ++c) {
      idx->counter[c] = 0u;
      idx->total[c] = st == BFP_OK ? s_carry[c] : 0;
    }
    idx->ntasks = count;
    idx->status = st;
    *status_out = st;
  }
}

struct NoallocDevice {
  unsigned char* ptr = nullptr;  // device address of `scratch` on this device
  int cap[kBatchClasses] = {};
  bool ready = false;
};
std::mutex g_noalloc_mu;
NoallocDevice g_noalloc[64];

// Scratch address and resident grids of the current device, set up once per
// device with that device current.
bool noalloc_device(NoallocDevice* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  NoallocDevice& d = g_noalloc[dev];
  if (!d.ready) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return false;
    for (int c = 0; c < kBatchClasses; ++c) {
      d.cap[c] = batch_resident_blocks(c);
      if (d.cap[c] <= 0) return false;
    }
    d.ptr = static_cast<unsigned char*>(p);
    d.ready = true;
  }
  *out = d;
  return true;
}

template <int CLS>
void launch_indexed(const NoallocDevice& d, hipStream_t s) {
  BatchIndex* idx = reinterpret_cast<BatchIndex*>(d.ptr);
  const BatchTask* tasks = reinterpret_cast<const BatchTask*>(d.ptr + kNoallocTasksOff);
  const uint64_t* prefix = reinterpret_cast<const uint64_t*>(d.ptr + kNoallocPrefixOff) + CLS * kNoallocPrefixWords;
  hipLaunchKernelGGL((k_batch<CLS>), dim3(d.cap[CLS]), dim3(kBatchBlock), 0, s, tasks, nullptr, 0u, 0u,
                     &idx->counter[CLS], idx, prefix);
}

}  // namespace
}  // namespace bfp

extern "C" bfp_status bfp_batch_run_noalloc(const bfp_task* tasks_dev, uint32_t count, int32_t* status_dev,
                                            void* stream) {
  if (!tasks_dev || !status_dev) return BFP_E_NULL;
  if (count == 0 || count > kNoallocMaxTasks) return BFP_E_ARG;
  if (((uintptr_t)tasks_dev & 7u) || ((uintptr_t)status_dev & 3u)) return BFP_E_ALIGN;
  NoallocDevice d;
  if (!noalloc_device(&d)) return BFP_E_HIP;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(1024), 0, s, tasks_dev, count, d.ptr, status_dev);
  launch_indexed<0>(d, s);
  launch_indexed<1>(d, s);
  return hipGetLastError() == hipSuccess ? BFP_OK : BFP_E_HIP;
}
