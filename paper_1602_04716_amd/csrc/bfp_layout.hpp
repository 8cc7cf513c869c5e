// bfp_layout.hpp -- the bitslice layout's size rules, shared by the HIP
// library and the CPU tests (no HIP types).
//
// Plane k of a vector of n elements is G_pad consecutive 32-bit words; element
// i sits in word i/32 at bit i%32 (Section 2, Figure 1, plane-major).
#pragma once
#include <stdint.h>

#include "bfp_word.hpp"

namespace bfp {

// Plane stride: whole 64-word (256-byte) tiles, skewed by 256 words when it
// would be a multiple of 2048 words: planes 8 KiB-multiples apart put every
// plane of a word group on the same HBM channels (measured: unpack of 2^26
// elements 10% slower at an 8 MiB stride than at 8 MiB + 1 KiB).  Because of
// the skew the stride is not monotonic in n: stride(65000) = 2304 words but
// stride(66000) = 2112.
BFP_FN uint64_t gpad_of(uint64_t n) {
  const uint64_t g = (n + 31) / 32;
  const uint64_t gp = (g + 63) / 64 * 64;
  return gp % 2048 == 0 ? gp + 256 : gp;
}

// Words per plane that hold any element below n.  A kernel computing the
// first n elements of operands of na >= n elements reads only these words of
// each operand plane: ceil(n/32) <= ceil(na/32) <= gpad_of(na), so the reads
// stay inside the operand whatever its stride.
BFP_FN uint64_t data_words(uint64_t n) { return (n + 31) / 32; }

// Mask of the elements below n in word w of a plane.
BFP_FN uint32_t word_mask(uint64_t w, uint64_t n) {
  const uint64_t full = n >> 5;
  return w < full ? 0xFFFFFFFFu : (w == full ? (1u << (uint32_t)(n & 31u)) - 1u : 0u);
}

}  // namespace bfp
