// bfp_chain.hpp -- two-op chains on resident bitslice vectors in one kernel:
// d = (a op1 b) op2 c, the intermediate kept in registers.
//
// Section 4 merges successive steps of one operation so that intermediate
// results are not stored; the same idea applied across operations removes
// the store and reload of the intermediate vector: 4 vectors move through
// HBM instead of 6.  Each op still rounds on its own, so the result equals
// the two single-op calls bit for bit.
#pragma once
#include "bfp_kernels.hpp"

namespace bfp {

// Plane k of a vector whose every element is the pattern `alpha`.
template <int R>
__device__ __forceinline__ WordR<R> splat_plane(uint32_t alpha, int k) {
  WordR<R> v;
  const uint32_t w = ((alpha >> k) & 1u) ? 0xFFFFFFFFu : 0u;
#pragma unroll
  for (int r = 0; r < R; ++r) v.w[r] = w;
  return v;
}

// a == nullptr broadcasts the pattern alpha in place of a.  Outputs of
// elements at and above n are masked to zero: a broadcast operand makes the
// padding lanes compute alpha op1 0, which need not be +0.
template <int E, int M, bool RZ, int OPC1, int OPC2, int R>
__global__ void __launch_bounds__(512) k_chain2(const uint32_t* a, uint32_t alpha, const uint32_t* b,
                                                const uint32_t* c, uint32_t* d, uint64_t gpad, uint64_t n,
                                                uint32_t negb1, uint32_t negb2) {
  constexpr int B = 1 + E + M;
  const uint64_t nt = gpad / R;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += stride) {
    const uint64_t off = t * R;
    WordR<R> x[B], y[B], z[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      x[k] = a ? ld_words<R>(a + (uint64_t)k * gpad + off) : splat_plane<R>(alpha, k);
      y[k] = ld_words<R>(b + (uint64_t)k * gpad + off);
    }
    circuit<E, M, RZ, OPC1, R>(x, y, negb1, z);
#pragma unroll
    for (int k = 0; k < B; ++k) y[k] = ld_words<R>(c + (uint64_t)k * gpad + off);
    circuit<E, M, RZ, OPC2, R>(z, y, negb2, x);
    uint32_t mk[R];
    valid_mask<R>(off, n, mk);
#pragma unroll
    for (int k = 0; k < B; ++k) {
#pragma unroll
      for (int r = 0; r < R; ++r) x[k].w[r] &= mk[r];
      st_words<R>(d + (uint64_t)k * gpad + off, x[k]);
    }
  }
}

template <int E, int M, bool RZ, int OPC1, int OPC2>
hipError_t launch_chain2(const void* a, uint32_t alpha, const void* b, const void* c, void* d, uint64_t gpad,
                         uint64_t n, uint32_t negb1, uint32_t negb2, unsigned grid, unsigned block, hipStream_t s) {
  hipLaunchKernelGGL((k_chain2<E, M, RZ, OPC1, OPC2, 1>), dim3(grid), dim3(block), 0, s,
                     static_cast<const uint32_t*>(a), alpha, static_cast<const uint32_t*>(b),
                     static_cast<const uint32_t*>(c), static_cast<uint32_t*>(d), gpad, n, negb1, negb2);
  return hipGetLastError();
}

template <int E, int M>
void register_chain() {
  Registry& r = registry();
#define BFP_CHAIN_REG(O1, O2)                                               \
  r.chain[E][M][O1][O2][0] = launch_chain2<E, M, false, O1, O2>; \
  r.chain[E][M][O1][O2][1] = launch_chain2<E, M, true, O1, O2>;
  BFP_CHAIN_REG(0, 0)
  BFP_CHAIN_REG(0, 1)
  BFP_CHAIN_REG(1, 0)
  BFP_CHAIN_REG(1, 1)
#undef BFP_CHAIN_REG
}

}  // namespace bfp
