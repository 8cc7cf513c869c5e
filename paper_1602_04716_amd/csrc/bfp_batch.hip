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
// Device: a grid sized to the GPU's resident capacity; each block takes the
// next chunk index from an atomic counter, reads the chunk's task, and
// switches (block-uniformly) to the compiled circuit of the task's
// (e, m, operation class, rounding mode).  Division chunks go to a second
// persistent kernel after the first, so that the divider's registers do not
// lower the first kernel's occupancy.  The counters are cleared by a
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

namespace bfp {

// variant = ((format index) * kOpClasses + opclass) * 2 + rz, format index in
// the order of BFP_FOR_EACH_FORMAT

__host__ __device__ constexpr int format_index(int e, int m) {
  const int ei = e == 3 ? 0 : e == 4 ? 1 : e == 5 ? 2 : e == 6 ? 3 : e == 8 ? 4 : -1;
  const int mi = m == 1 ? 0 : m == 2 ? 1 : m == 3 ? 2 : m == 5 ? 3 : m == 7 ? 4 : m == 10 ? 5
               : m == 15 ? 6 : m == 23 ? 7 : -1;
  return (ei < 0 || mi < 0) ? -1 : ei * 8 + mi;
}

// One chunk of one task: the block's threads stride over the chunk's words.
// One word per lane: two would double the registers of the light circuits,
// and any two-word instance raises the whole kernel's register allocation
// (measured: 131 -> 176 VGPRs), cutting resident waves from 3 to 2 per SIMD.
template <int E, int M, bool RZ, int OPC>
__device__ __forceinline__ void batch_chunk(const BatchTask& tk, uint64_t w0, uint32_t nw) {
  constexpr int B = 1 + E + M;
  constexpr int R = 1;
  const uint64_t end = w0 + nw;
  for (uint64_t off = w0 + (uint64_t)threadIdx.x * R; off < end; off += (uint64_t)blockDim.x * R) {
    WordR<R> x[B], y[B], z[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      x[k] = ld_words<R>(tk.a + (uint64_t)k * tk.sa + off);
      y[k] = ld_words<R>(tk.b + (uint64_t)k * tk.sb + off);
    }
    circuit<E, M, RZ, OPC, R>(x, y, tk.negb, z);
    mask_padding<OPC, R, B>(z, off, tk.n);
#pragma unroll
    for (int k = 0; k < B; ++k) st_words<R>(tk.c + (uint64_t)k * tk.sc + off, z[k]);
  }
}

constexpr bool variant_is_div(uint32_t v) { return (v / 2) % kOpClasses == 2; }

__global__ void k_batch_reset(uint32_t* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    counter[0] = 0u;
    counter[1] = 0u;
  }
}

// Persistent kernel over chunks [first, first + nchunks).  DIV selects the
// division variants; the other kernel holds add/sub and mul.
template <bool DIV>
__global__ void __launch_bounds__(kBatchBlock) k_batch(const BatchTask* tasks, const BatchChunk* chunks,
                                                       uint32_t first, uint32_t nchunks, uint32_t* counter) {
  __shared__ uint32_t s_next;
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t ci = s_next;
    __syncthreads();
    if (ci >= nchunks) break;  // every block sees the counter pass nchunks and leaves
    const BatchChunk ch = chunks[first + ci];
    const BatchTask tk = tasks[ch.task];
    if constexpr (DIV) {
      switch (tk.variant) {
#define BFP_BATCH_VARIANT(EE, MM, OPC, RZ) \
  case (format_index(EE, MM) * kOpClasses + OPC) * 2 + RZ: batch_chunk<EE, MM, RZ, OPC>(tk, ch.w0, ch.nwords); break;
#define BFP_BATCH_CASE(EE, MM) BFP_BATCH_VARIANT(EE, MM, 2, false) BFP_BATCH_VARIANT(EE, MM, 2, true)
        BFP_FOR_EACH_FORMAT(BFP_BATCH_CASE)
#undef BFP_BATCH_CASE
        default: break;
      }
    } else {
      switch (tk.variant) {
#define BFP_BATCH_CASE(EE, MM)                                                                           \
  BFP_BATCH_VARIANT(EE, MM, 0, false) BFP_BATCH_VARIANT(EE, MM, 0, true) BFP_BATCH_VARIANT(EE, MM, 1, false) \
  BFP_BATCH_VARIANT(EE, MM, 1, true)
        BFP_FOR_EACH_FORMAT(BFP_BATCH_CASE)
#undef BFP_BATCH_CASE
#undef BFP_BATCH_VARIANT
        default: break;
      }
    }
  }
}

constexpr int kBatchFormats = 40;  // format_index covers 5 exponent x 8 mantissa widths

bool batch_format_ok(const bfp_format& f) { return format_index(f.e, f.m) >= 0 && f.round <= 1; }

bool batch_task(const void* a, uint64_t na, const void* b, uint64_t nb, void* c, uint64_t n, bfp_format f, int op,
                BatchTask* out) {
  const int fi = format_index(f.e, f.m);
  if (fi < 0 || f.round > 1 || !op_valid(op)) return false;
  if (na < n || nb < n) return false;
  out->a = static_cast<const uint32_t*>(a);
  out->b = static_cast<const uint32_t*>(b);
  out->c = static_cast<uint32_t*>(c);
  out->sa = bfp_plane_stride_words(na);
  out->sb = bfp_plane_stride_words(nb);
  out->sc = bfp_plane_stride_words(n);
  out->words = out->sc;
  out->n = n;
  out->negb = op == BFP_SUB ? 0xFFFFFFFFu : 0u;
  out->variant = (uint32_t)((fi * kOpClasses + opclass_of(op)) * 2 + f.round);
  return true;
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

void batch_chunks(const std::vector<BatchTask>& dt, std::vector<BatchChunk>* out) {
  std::vector<BatchChunk>& chunks = *out;
  chunks.clear();
  for (uint32_t i = 0; i < (uint32_t)dt.size(); ++i) {
    for (uint64_t w = 0; w < dt[i].words; w += kChunkWords) {
      BatchChunk ch;
      ch.w0 = w;
      ch.task = i;
      ch.nwords = (uint32_t)std::min<uint64_t>(kChunkWords, dt[i].words - w);
      chunks.push_back(ch);
    }
  }
  // division last, then variants by decreasing time per word (ties by
  // variant); within a variant, longer tasks first, then by position
  const std::vector<uint32_t>& cost = variant_cost();
  std::stable_sort(chunks.begin(), chunks.end(), [&](const BatchChunk& x, const BatchChunk& y) {
    const uint32_t vx = dt[x.task].variant, vy = dt[y.task].variant;
    if (variant_is_div(vx) != variant_is_div(vy)) return variant_is_div(vy);
    if (cost[vx] != cost[vy]) return cost[vx] > cost[vy];
    if (vx != vy) return vx < vy;
    if (dt[x.task].words != dt[y.task].words) return dt[x.task].words > dt[y.task].words;
    if (x.task != y.task) return x.task < y.task;
    return x.w0 < y.w0;
  });
}

int batch_resident_blocks(bool div) {
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  const hipError_t e = div ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<true>, kBatchBlock, 0)
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<false>, kBatchBlock, 0);
  if (e != hipSuccess) return 0;
  if (per_cu < 1) per_cu = 1;
  return per_cu * prop.multiProcessorCount;
}

BatchSplit batch_split(const std::vector<BatchTask>& tasks, const std::vector<BatchChunk>& chunks, int cap_main,
                       int cap_div) {
  BatchSplit sp;
  for (const BatchChunk& ch : chunks) {
    if (variant_is_div(tasks[ch.task].variant)) ++sp.n_div;
    else ++sp.n_main;
  }
  sp.grid_main = (unsigned)std::min<uint64_t>((uint64_t)std::max(cap_main, 1), sp.n_main);
  sp.grid_div = (unsigned)std::min<uint64_t>((uint64_t)std::max(cap_div, 1), sp.n_div);
  return sp;
}

hipError_t batch_launch(const BatchTask* d_tasks, const BatchChunk* d_chunks, const BatchSplit& sp,
                        uint32_t* d_counter, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, d_counter);
  if (sp.n_main > 0)
    hipLaunchKernelGGL((k_batch<false>), dim3(sp.grid_main), dim3(kBatchBlock), 0, s, d_tasks, d_chunks, 0u,
                       sp.n_main, d_counter);
  if (sp.n_div > 0)
    hipLaunchKernelGGL((k_batch<true>), dim3(sp.grid_div), dim3(kBatchBlock), 0, s, d_tasks, d_chunks, sp.n_main,
                       sp.n_div, d_counter + 1);
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
  uint64_t words_total = 0;  // sum over tasks of B * gpad (per operand)
  std::mutex mu;
};

namespace {

void plan_free(bfp_batch_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
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
  // resident grids: as many blocks as fit on the device at once
  const int cap_main = batch_resident_blocks(false), cap_div = batch_resident_blocks(true);
  if (cap_main <= 0 || cap_div <= 0) {
    plan_free(p);
    return BFP_E_HIP;
  }
  p->split = batch_split(dt, chunks, cap_main, cap_div);
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

bfp_status bfp_batch_plan_info(const bfp_batch_plan* plan, uint32_t* nchunks, uint32_t* grid,
                               uint64_t* words_per_operand) {
  if (!plan) return BFP_E_NULL;
  if (nchunks) *nchunks = plan->nchunks;
  if (grid) *grid = plan->split.grid_main > plan->split.grid_div ? plan->split.grid_main : plan->split.grid_div;
  if (words_per_operand) *words_per_operand = plan->words_total;
  return BFP_OK;
}

void bfp_batch_plan_destroy(bfp_batch_plan* plan) { plan_free(plan); }

}  // extern "C"
