// bfp_batch.hpp -- descriptors and helpers of the batched persistent kernel,
// shared by the batch plan (bfp_batch.hip) and the serving loop
// (bfp_server.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "bfp.h"

namespace bfp {

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

constexpr uint32_t kChunkWords = 2048;
constexpr int kBatchBlock = 256;

// Fill a task descriptor for c = a op b on the first n elements, format f;
// a and b have na and nb elements (na, nb >= n: their plane strides follow
// from those lengths), c has n.  Returns false if the format or op is not
// compiled.
bool batch_task(const void* a, uint64_t na, const void* b, uint64_t nb, void* c, uint64_t n, bfp_format f, int op,
                BatchTask* out);

// Formats the persistent batch kernels compile (the 40 sweep formats).
bool batch_format_ok(const bfp_format& f);

// Cut tasks into chunks of at most kChunkWords words, grouped by circuit
// variant, variants in decreasing time per word (the larger of the circuit's
// plane traffic and its gate count) and, within a variant, longest task
// first; chunks of the division circuit come last.
void batch_chunks(const std::vector<BatchTask>& tasks, std::vector<BatchChunk>* out);

// Division chunks run in a persistent kernel of their own: the divider's
// register demand would otherwise set the register allocation, and so lower
// the occupancy, of the kernel that runs every other circuit.
struct BatchSplit {
  uint32_t n_main = 0;  // chunks [0, n_main): add/sub/mul kernel
  uint32_t n_div = 0;   // chunks [n_main, n_main + n_div): division kernel
  unsigned grid_main = 0, grid_div = 0;
};

// Blocks of the persistent kernel (division kernel if div) that fit on the
// current device at once; 0 on error.
int batch_resident_blocks(bool div);

// Split of sorted chunks with grids capped at the resident block counts.
BatchSplit batch_split(const std::vector<BatchTask>& tasks, const std::vector<BatchChunk>& chunks, int cap_main,
                       int cap_div);

// Enqueue the counter reset and the persistent kernels that have chunks on
// `s`.  d_counter holds two counters.
hipError_t batch_launch(const BatchTask* d_tasks, const BatchChunk* d_chunks, const BatchSplit& split,
                        uint32_t* d_counter, hipStream_t s);

}  // namespace bfp
