// bfp_int_kernels.hpp -- kernels of the k-bit integer vectors: c = a op b
// on resident bitslice vectors, every word of every plane.
#pragma once
#include "bfp_int_circuits.hpp"
#include "bfp_kernels.hpp"

namespace bfp {

// Words per lane: two for the circuits that move more bytes than they
// compute, one for the quadratic multipliers from k = 13 up.
template <int K, int OP>
constexpr int int_words_per_lane() {
  return (OP == 2 && K > 12) ? 1 : 2;
}

// Padding elements are 0 op 0 = 0 for every op and kind, so the zero padding
// of c needs no mask.
template <int K, int OP, int KIND, int R>
__global__ void __launch_bounds__(512) k_ibinop(const uint32_t* a, const uint32_t* b, uint32_t* c, uint64_t gpad) {
  const uint64_t nt = gpad / R;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += stride) {
    const uint64_t off = t * R;
    WordR<R> x[K], y[K], z[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      x[k] = ld_words<R>(a + (uint64_t)k * gpad + off);
      y[k] = ld_words<R>(b + (uint64_t)k * gpad + off);
    }
    int_circuit<K, OP, KIND, WordR<R>>(x, y, z);
#pragma unroll
    for (int k = 0; k < K; ++k) st_words<R>(c + (uint64_t)k * gpad + off, z[k]);
  }
}

using IntLauncher = hipError_t (*)(const void* a, const void* b, void* c, uint64_t gpad, unsigned grid,
                                   unsigned block, hipStream_t s);

struct IntRegistry {
  IntLauncher op[kMaxIntBits + 1][3][3] = {};  // [k][op][kind]
  int words[kMaxIntBits + 1][3] = {};          // words per lane compiled for [k][op]
};
IntRegistry& int_registry();

template <int K, int OP, int KIND>
hipError_t launch_ibinop(const void* a, const void* b, void* c, uint64_t gpad, unsigned grid, unsigned block,
                         hipStream_t s) {
  constexpr int R = int_words_per_lane<K, OP>();
  hipLaunchKernelGGL((k_ibinop<K, OP, KIND, R>), dim3(grid > 0 ? grid : 1), dim3(block), 0, s,
                     static_cast<const uint32_t*>(a), static_cast<const uint32_t*>(b), static_cast<uint32_t*>(c),
                     gpad);
  return hipGetLastError();
}

template <int K>
void register_int() {
  IntRegistry& r = int_registry();
#define BFP_INT_REG(OP)                                        \
  r.words[K][OP] = int_words_per_lane<K, OP>();            \
  r.op[K][OP][kIntWrap] = launch_ibinop<K, OP, kIntWrap>; \
  r.op[K][OP][kIntSatU] = launch_ibinop<K, OP, kIntSatU>; \
  r.op[K][OP][kIntSatS] = launch_ibinop<K, OP, kIntSatS>;
  BFP_INT_REG(0)
  BFP_INT_REG(1)
  BFP_INT_REG(2)
#undef BFP_INT_REG
}

}  // namespace bfp
