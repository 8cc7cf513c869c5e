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

// Cut tasks into chunks of at most kChunkWords words, sorted by circuit
// variant and, within a variant, longest task first.
void batch_chunks(const std::vector<BatchTask>& tasks, std::vector<BatchChunk>* out);

// Blocks of the persistent kernel that fit on the current device at once.
int batch_resident_blocks();

// Enqueue counter reset + persistent kernel on `s`.
hipError_t batch_launch(const BatchTask* d_tasks, const BatchChunk* d_chunks, uint32_t nchunks, uint32_t* d_counter,
                        unsigned grid, hipStream_t s);

}  // namespace bfp
