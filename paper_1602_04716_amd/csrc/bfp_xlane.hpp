// bfp_xlane.hpp -- the layout transposes of Section 4 (standard <-> bitslice,
// Figure 1) done across lanes: the alternative to the per-lane transposes of
// k_pack / k_unpack, for the autotuner to choose between.
//
// A wave works on tiles of 64 groups (2048 elements).  For each of 32 steps
// i, lane l holds one element, 2048 t + 64 i + l, so the 32 lanes of each
// half-wave hold the 32 elements of one group; a 32 x 32 bit transpose
// across those lanes (five delta-swap stages, the partner word fetched with
// ds_swizzle in its xor mode) leaves in lane j the word of plane j for that
// group.  The plane words are gathered in LDS, one row of 64 words per plane
// (rows padded to 65 words so that the 32 lanes' column writes fall in
// distinct banks), and stored a plane row at a time: one coalesced 256-byte
// store per plane per tile.  Unpack runs the same steps backwards (the
// transpose is its own inverse).  Each lane needs one word of the element
// and a few temporaries instead of the 8 C words of a whole group, at the
// price of about 40 instructions per 64 elements against about 8 for the
// per-lane transposes.
#pragma once
#include <hip/hip_runtime.h>

#include "bfp_kernels.hpp"

namespace bfp {

// One delta-swap stage between lane pairs (j, j ^ D) of a half-wave (lane j
// holding row j of the bit matrix): the pair exchanges the off-diagonal
// D x D blocks, the low lane's bits at MASK << D for the high lane's bits at
// MASK.
template <int D, uint32_t MASK>
__device__ __forceinline__ uint32_t xlane_stage(uint32_t w, uint32_t lane) {
  const uint32_t p = (uint32_t)__builtin_amdgcn_ds_swizzle((int)w, 0x1F | (D << 10));  // w of lane ^ D
  const bool low = (lane & D) == 0;
  const uint32_t lo = low ? w : p, hi = low ? p : w;
  const uint32_t t = ((lo >> D) ^ hi) & MASK;
  return w ^ (low ? (t << D) : t);
}

// 32 x 32 bit transpose across the 32 lanes of each half-wave: afterwards
// bit c of lane j's word is bit j of lane c's word before.  Every lane of the
// wave must execute it.
__device__ __forceinline__ uint32_t xlane_transpose32(uint32_t w) {
  const uint32_t lane = threadIdx.x & 31u;
  w = xlane_stage<16, 0x0000FFFFu>(w, lane);
  w = xlane_stage<8, 0x00FF00FFu>(w, lane);
  w = xlane_stage<4, 0x0F0F0F0Fu>(w, lane);
  w = xlane_stage<2, 0x33333333u>(w, lane);
  w = xlane_stage<1, 0x55555555u>(w, lane);
  return w;
}

template <int C>
__device__ __forceinline__ uint32_t load_elem(const uint8_t* src, uint64_t e) {
  if constexpr (C == 1) return src[e];
  else if constexpr (C == 2) return reinterpret_cast<const uint16_t*>(src)[e];
  else return reinterpret_cast<const uint32_t*>(src)[e];
}

template <int C>
__device__ __forceinline__ void store_elem(uint8_t* dst, uint64_t e, uint32_t w) {
  if constexpr (C == 1) dst[e] = (uint8_t)w;
  else if constexpr (C == 2) reinterpret_cast<uint16_t*>(dst)[e] = (uint16_t)w;
  else reinterpret_cast<uint32_t*>(dst)[e] = w;
}

constexpr int kXlaneRow = 65;  // words per LDS plane row (64 + 1 of padding)

// Standard -> bitslice over all gpad words of each plane (padding words get
// zero bits).  Dynamic LDS: (blockDim / 64) * 32 * 65 * 4 bytes.
template <int C>
__global__ void __launch_bounds__(512) k_pack_x(const uint8_t* src, uint32_t* planes, uint64_t n, uint64_t gpad,
                                                int B) {
  extern __shared__ uint32_t xl_pack_lds[];
  const int nw = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int h = lane >> 5, j = lane & 31;
  uint32_t* rows = xl_pack_lds + wave * 32 * kXlaneRow;
  const uint64_t tiles = gpad / 64;  // gpad is a multiple of 64
  const uint64_t block_tiles = (tiles + nw - 1) / nw;
  for (uint64_t bt = blockIdx.x; bt < block_tiles; bt += gridDim.x) {
    const uint64_t t = bt * nw + wave;
    const bool active = t < tiles;  // the same for every lane of the wave
    if (active) {
      for (int i = 0; i < 32; ++i) {
        const uint64_t e = t * 2048 + 64 * i + lane;
        uint32_t w = 0u;
        if (e < n) w = load_elem<C>(src, e);
        w = xlane_transpose32(w);  // lane j of half h: plane j of group 2 i + h
        if (j < B) rows[j * kXlaneRow + 2 * i + h] = w;
      }
    }
    __syncthreads();
    if (active) {
      for (int k = 0; k < B; ++k) planes[(uint64_t)k * gpad + t * 64 + lane] = rows[k * kXlaneRow + lane];
    }
    __syncthreads();
  }
}

// Bitslice -> standard: the n containers (upper bits zero), nothing past n.
// Dynamic LDS as for k_pack_x.
template <int C>
__global__ void __launch_bounds__(512) k_unpack_x(const uint32_t* planes, uint8_t* dst, uint64_t n, uint64_t gpad,
                                                  int B) {
  extern __shared__ uint32_t xl_unpack_lds[];
  const int nw = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int h = lane >> 5, j = lane & 31;
  uint32_t* rows = xl_unpack_lds + wave * 32 * kXlaneRow;
  const uint64_t groups = (n + 31) / 32;
  const uint64_t tiles = (groups + 63) / 64;
  const uint64_t block_tiles = (tiles + nw - 1) / nw;
  for (uint64_t bt = blockIdx.x; bt < block_tiles; bt += gridDim.x) {
    const uint64_t t = bt * nw + wave;
    const bool active = t < tiles;
    if (active) {
      for (int k = 0; k < B; ++k) rows[k * kXlaneRow + lane] = planes[(uint64_t)k * gpad + t * 64 + lane];
    }
    __syncthreads();
    if (active) {
      for (int i = 0; i < 32; ++i) {
        uint32_t w = j < B ? rows[j * kXlaneRow + 2 * i + h] : 0u;
        w = xlane_transpose32(w);  // lane l: element 2048 t + 64 i + l
        const uint64_t e = t * 2048 + 64 * i + lane;
        if (e < n) store_elem<C>(dst, e, w);
      }
    }
    __syncthreads();
  }
}

}  // namespace bfp
