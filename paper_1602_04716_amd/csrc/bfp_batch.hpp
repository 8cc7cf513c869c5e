// bfp_batch.hpp -- descriptors and helpers of the batched persistent kernel,
// shared by the batch plan (bfp_batch.hip) and the serving loop
// (bfp_server.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "bfp.h"
#include "bfp_layout.hpp"
#include "bfp_ops.hpp"

namespace bfp {

// Index of the 40 sweep formats (e in {3,4,5,6,8} x m in
// {1,2,3,5,7,10,15,23}, in the order of BFP_FOR_EACH_FORMAT) or -1.  A
// circuit variant is ((format index) * kOpClasses + opclass) * 2 + rz.
__host__ __device__ constexpr int format_index(int e, int m) {
  const int ei = e == 3 ? 0 : e == 4 ? 1 : e == 5 ? 2 : e == 6 ? 3 : e == 8 ? 4 : -1;
  const int mi = m == 1 ? 0 : m == 2 ? 1 : m == 3 ? 2 : m == 5 ? 3 : m == 7 ? 4 : m == 10 ? 5
               : m == 15 ? 6 : m == 23 ? 7 : -1;
  return (ei < 0 || mi < 0) ? -1 : ei * 8 + mi;
}

struct BatchTask {
  const uint32_t* a;
  const uint32_t* b;
  uint32_t* c;
  uint64_t sa, sb, sc;  // plane strides of a, b, c in 32-bit words
  uint64_t words;       // words per plane to compute (a multiple of 64)
  uint64_t n;           // elements of c (division masks lanes at and above n)
  uint32_t negb;
  uint32_t variant;
};

struct BatchChunk {
  uint64_t w0;      // first word of the chunk within each plane
  uint32_t task;    // index into the task table
  uint32_t nwords;  // words per plane in this chunk (multiple of 64)
};

// Words per plane of one chunk: 1024 (four per lane of a 256-thread block)
// measured 1-2% faster than 2048 on the 4096-vector batch (a finer tail and
// balance), 512 7% slower and 4096 1% slower (per-chunk costs).
constexpr uint32_t kChunkWords = 1024;
constexpr int kBatchBlock = 256;

// Kernel classes of the circuit variants: 0 add/sub and mul, 1 division.
// Each class runs in a persistent kernel of its own, so the divider's
// registers do not set the occupancy of the kernel that runs everything
// else.  (Splitting further, by the registers of the add/sub/mul circuits,
// measured slower: a kernel that mixes VALU-bound wide multipliers with
// HBM-bound light circuits overlaps the two, 0.70 ms for the 4096-vector
// batch against 0.78-0.80 ms for three register classes run one after
// another.)
constexpr int kBatchClasses = 2;
__host__ __device__ constexpr int variant_class(int m, int opc) { return opc == 2 ? 1 : 0; }

// Chunks of a batch whose descriptors were built on the device (by the
// allocation-free entry point): the class kernels' chunk totals and counters.
struct BatchIndex {
  uint32_t counter[kBatchClasses];  // next chunk of each class kernel
  uint32_t ntasks;
  int32_t status;
  uint64_t total[kBatchClasses];    // chunks of each class
};

// Descriptor of c = a op b on the first n elements (a and b have na, nb >= n
// elements; each plane stride follows from its vector's length), for the
// batch kernels' formats.  False if the format or the lengths do not fit;
// op must be valid.
__host__ __device__ inline bool make_batch_task(const void* a, uint64_t na, const void* b, uint64_t nb, void* c,
                                                uint64_t n, bfp_format f, int op, BatchTask* out) {
  const int fi = format_index(f.e, f.m);
  if (fi < 0 || f.round > 1) return false;
  if (na < n || nb < n) return false;
  const int opc = op == BFP_MUL ? 1 : (op == BFP_DIV ? 2 : 0);
  out->a = static_cast<const uint32_t*>(a);
  out->b = static_cast<const uint32_t*>(b);
  out->c = static_cast<uint32_t*>(c);
  out->sa = gpad_of(na);
  out->sb = gpad_of(nb);
  out->sc = gpad_of(n);
  out->words = out->sc;
  out->n = n;
  out->negb = op == BFP_SUB ? 0xFFFFFFFFu : 0u;
  out->variant = (uint32_t)((fi * kOpClasses + opc) * 2 + f.round);
  return true;
}

// Fill a task descriptor for c = a op b on the first n elements, format f;
// a and b have na and nb elements (na, nb >= n: their plane strides follow
// from those lengths), c has n.  Returns false if the format or op is not
// compiled.
bool batch_task(const void* a, uint64_t na, const void* b, uint64_t nb, void* c, uint64_t n, bfp_format f, int op,
                BatchTask* out);

// Formats the persistent batch kernels compile (the 40 sweep formats).
bool batch_format_ok(const bfp_format& f);

// Cut tasks into chunks of at most kChunkWords words, grouped by register
// class and then by circuit variant, variants in decreasing time per word
// (the larger of the circuit's plane traffic and its gate count) and, within
// a variant, longest task first.
void batch_chunks(const std::vector<BatchTask>& tasks, std::vector<BatchChunk>* out);

// Register class of a task's circuit.
int task_class(const BatchTask& t);

// Chunks of each class kernel: class c runs chunks [first[c], first[c] +
// n[c]) of the sorted table on grid[c] blocks.
struct BatchSplit {
  uint32_t first[kBatchClasses] = {};
  uint32_t n[kBatchClasses] = {};
  unsigned grid[kBatchClasses] = {};
};

// Blocks of class c's persistent kernel that fit on the current device at
// once; 0 on error.
int batch_resident_blocks(int c);

// Split of sorted chunks with grids capped at the resident block counts
// cap[c].
BatchSplit batch_split(const std::vector<BatchTask>& tasks, const std::vector<BatchChunk>& chunks,
                       const int* cap);

// Enqueue the counter reset and the class kernels that have chunks on `s`.
// d_counter holds kBatchClasses counters.
hipError_t batch_launch(const BatchTask* d_tasks, const BatchChunk* d_chunks, const BatchSplit& split,
                        uint32_t* d_counter, hipStream_t s);

}  // namespace bfp
