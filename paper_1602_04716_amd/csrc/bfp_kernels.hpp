// bfp_kernels.hpp -- HIP kernels for gfx950 and their launchers.
//
// Data layout (plane-major bitslice, see include/bfp.h): plane k of a vector
// is gpad consecutive 32-bit words.  A lane owns R adjacent words of every
// plane (W = 32 R elements) and reads them with one coalesced load per
// plane: consecutive lanes read consecutive words, so each plane load of a
// wave is one contiguous 256 R-byte segment.  The circuit runs entirely in
// VGPRs; nothing here is a contraction, so there is no MFMA.
//
// Memory policy (measured on MI355X): plane loads are ordinary cached loads,
// plane stores are non-temporal (streaming) stores; the standard-layout side
// of pack uses ordinary loads (a lane's 32 C contiguous bytes span partial
// cache lines that neighbouring lanes' loads reuse), and unpack stages its
// output through LDS so that every global store of a wave writes one
// contiguous 1 KiB segment.
#pragma once
#include <hip/hip_runtime.h>

#include "bfp_circuits.hpp"
#include "bfp_formats.hpp"
#include "bfp_ops.hpp"
#include "bfp_transpose.hpp"

namespace bfp {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int R>
__device__ __forceinline__ WordR<R> ld_words(const uint32_t* p) {
  WordR<R> v;
  if constexpr (R == 1) {
    v.w[0] = *p;
  } else if constexpr (R == 2) {
    const u32x2 t = *reinterpret_cast<const u32x2*>(p);
    v.w[0] = t.x;
    v.w[1] = t.y;
  } else {
    static_assert(R == 4, "R must be 1, 2 or 4");
    const u32x4 t = *reinterpret_cast<const u32x4*>(p);
    v.w[0] = t.x;
    v.w[1] = t.y;
    v.w[2] = t.z;
    v.w[3] = t.w;
  }
  return v;
}

template <int R>
__device__ __forceinline__ void st_words(uint32_t* p, const WordR<R>& v) {
  if constexpr (R == 1) {
    __builtin_nontemporal_store(v.w[0], p);
  } else if constexpr (R == 2) {
    u32x2 t;
    t.x = v.w[0];
    t.y = v.w[1];
    __builtin_nontemporal_store(t, reinterpret_cast<u32x2*>(p));
  } else {
    u32x4 t;
    t.x = v.w[0];
    t.y = v.w[1];
    t.z = v.w[2];
    t.w = v.w[3];
    __builtin_nontemporal_store(t, reinterpret_cast<u32x4*>(p));
  }
}

// One circuit instance on R words per plane.
template <int E, int M, bool RZ, int OPC, int R>
__device__ __forceinline__ void circuit(const WordR<R>* x, const WordR<R>* y, uint32_t negb, WordR<R>* z) {
  if constexpr (OPC == 0) {
    WordR<R> nb;
#pragma unroll
    for (int i = 0; i < R; ++i) nb.w[i] = negb;
    fp_add<E, M, RZ, WordR<R>>(x, y, nb, z);
  } else if constexpr (OPC == 1) {
    fp_mul<E, M, RZ, WordR<R>>(x, y, z);
  } else {
    fp_div<E, M, RZ, WordR<R>>(x, y, z);
  }
}

// Lane mask of R words starting at word `off` of a vector of n elements:
// set for elements below n.  Division maps the zero padding to 0/0 = NaN, so
// its outputs are masked to keep the padding of c zero; the other circuits
// map zero operands to +0 and need no mask.
template <int R>
__device__ __forceinline__ void valid_mask(uint64_t off, uint64_t n, uint32_t* mask) {
  const uint64_t full = n >> 5;
  const uint32_t part = (uint32_t)(n & 31u);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint64_t w = off + r;
    mask[r] = w < full ? 0xFFFFFFFFu : (w == full ? (1u << part) - 1u : 0u);
  }
}

template <int OPC, int R, int B>
__device__ __forceinline__ void mask_padding(WordR<R>* z, uint64_t off, uint64_t n) {
  if constexpr (OPC == 2) {
    uint32_t mk[R];
    valid_mask<R>(off, n, mk);
#pragma unroll
    for (int k = 0; k < B; ++k)
#pragma unroll
      for (int r = 0; r < R; ++r) z[k].w[r] &= mk[r];
  }
}

// c = a op b on resident bitslice vectors of n elements: every word of every
// plane (padding words of c are zero).  A lane takes U units of R adjacent
// words per loop step, the units a grid stride apart: R widens each plane
// load (4, 8 or 16 bytes per lane), U puts independent loads and circuit
// instances side by side; both trade registers for bytes in flight.  A unit
// past the end reads the step's first unit again and is not stored.
// `nb` and `ng` are the block and grid sizes, read by the kernel itself (see
// k_binop).
template <int E, int M, bool RZ, int OPC, int R, int U>
__device__ __forceinline__ void binop_body(const uint32_t* a, const uint32_t* b, uint32_t* c, uint64_t gpad,
                                           uint64_t n, uint32_t negb, unsigned nb, unsigned ng) {
  constexpr int B = 1 + E + M;
  constexpr int RU = R * U;
  const uint64_t nt = gpad / R;
  const uint64_t stride = (uint64_t)ng * nb;
  for (uint64_t t = (uint64_t)blockIdx.x * nb + threadIdx.x; t < nt; t += stride * U) {
    uint64_t off[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t tu = t + (uint64_t)u * stride;
      ok[u] = tu < nt;
      off[u] = (ok[u] ? tu : t) * R;
    }
    WordR<RU> x[B], y[B], z[B];
#pragma unroll
    for (int k = 0; k < B; ++k)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const WordR<R> xa = ld_words<R>(a + (uint64_t)k * gpad + off[u]);
        const WordR<R> yb = ld_words<R>(b + (uint64_t)k * gpad + off[u]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          x[k].w[u * R + r] = xa.w[r];
          y[k].w[u * R + r] = yb.w[r];
        }
      }
    circuit<E, M, RZ, OPC, RU>(x, y, negb, z);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      WordR<R> zu[B];
#pragma unroll
      for (int k = 0; k < B; ++k)
#pragma unroll
        for (int r = 0; r < R; ++r) zu[k].w[r] = z[k].w[u * R + r];
      mask_padding<OPC, R, B>(zu, off[u], n);
      if (ok[u]) {
#pragma unroll
        for (int k = 0; k < B; ++k) st_words<R>(c + (uint64_t)k * gpad + off[u], zu[k]);
      }
    }
  }
}

// The launch dimensions are read here, in the kernel, and passed down: read
// inside the inlined body, the compiler fetched the block size with a vector
// load from the dispatch's hidden arguments and waited for it before the
// first operand load; read here they come from a scalar load with the other
// kernel arguments.
template <int E, int M, bool RZ, int OPC, int R, int U>
__global__ void __launch_bounds__(512) k_binop(const uint32_t* a, const uint32_t* b, uint32_t* c,
                                               uint64_t gpad, uint64_t n, uint32_t negb) {
  binop_body<E, M, RZ, OPC, R, U>(a, b, c, gpad, n, negb, blockDim.x, gridDim.x);
}

// Load the 32 R standard elements starting at element e0 (C bytes each) as
// 8 C R dwords; elements at or past n read as zero.
template <int C, int R>
__device__ __forceinline__ void load_std(const uint8_t* src, uint64_t e0, uint64_t n, uint32_t (*in)[8 * C]) {
  if (e0 + 32 * R <= n) {
    const u32x4* p = reinterpret_cast<const u32x4*>(src + e0 * C);
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int q = 0; q < 2 * C; ++q) {
        const u32x4 v = p[r * 2 * C + q];
        in[r][4 * q + 0] = v.x;
        in[r][4 * q + 1] = v.y;
        in[r][4 * q + 2] = v.z;
        in[r][4 * q + 3] = v.w;
      }
    }
  } else {
    // ragged tail or padding: byte loads, every array index a constant
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int w = 0; w < 8 * C; ++w) {
        uint32_t v = 0u;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int byte = 4 * w + q;
          const uint64_t idx = e0 + 32 * r + byte / C;
          if (idx < n) v |= (uint32_t)src[idx * C + byte % C] << (8 * q);
        }
        in[r][w] = v;
      }
    }
  }
}

// Store 32 R standard elements starting at e0; nothing at or past n.
template <int C, int R>
__device__ __forceinline__ void store_std(uint8_t* dst, uint64_t e0, uint64_t n, uint32_t (*out)[8 * C]) {
  if (e0 + 32 * R <= n) {
    u32x4* p = reinterpret_cast<u32x4*>(dst + e0 * C);
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int q = 0; q < 2 * C; ++q) {
        u32x4 v;
        v.x = out[r][4 * q + 0];
        v.y = out[r][4 * q + 1];
        v.z = out[r][4 * q + 2];
        v.w = out[r][4 * q + 3];
        p[r * 2 * C + q] = v;
      }
    }
  } else {
    // ragged tail: one container store per element below n
#pragma unroll
    for (int j = 0; j < 32 * R; ++j) {
      const uint64_t idx = e0 + j;
      const int r = j >> 5, byte = (j & 31) * C;
      const uint32_t w = out[r][byte >> 2] >> (8 * (byte & 3));
      if (idx < n) {
        if constexpr (C == 1) dst[idx] = (uint8_t)w;
        else if constexpr (C == 2) reinterpret_cast<uint16_t*>(dst)[idx] = (uint16_t)w;
        else if constexpr (C == 4) reinterpret_cast<uint32_t*>(dst)[idx] = w;
        else reinterpret_cast<uint64_t*>(dst)[idx] = ((uint64_t)out[r][(byte >> 2) + 1] << 32) | w;
      }
    }
  }
}

// Standard -> bitslice over all gpad words of each plane (padding words get
// zero bits); B of the 8 C planes computed are stored.  Work goes in wave
// tiles of 64 groups (2048 elements): a tile wholly below n is read with
// coalesced streaming 16-byte loads (each load instruction of the wave covers
// one contiguous 1 KiB) into LDS, XOR-swizzled per lane so that each lane then
// reads its own 32 C bytes without bank conflicts; the ragged last tile and
// padding tiles read element by element.  Plane stores are ordinary stores,
// so the planes stay cache-resident for the operation that follows.  Loops run
// per block so every thread meets the same barriers.  Dynamic LDS:
// (blockDim / 64) * 2048 C bytes.
template <int C>
__global__ void __launch_bounds__(512) k_pack(const uint8_t* src, uint32_t* planes, uint64_t n,
                                              uint64_t gpad, int B) {
  extern __shared__ u32x4 pack_lds[];
  constexpr int CH = 2 * C;  // 16-byte chunks per lane
  const int nw = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  u32x4* tile = pack_lds + wave * 64 * CH;
  const uint64_t tiles = gpad / 64;  // gpad is a multiple of 64
  const uint64_t block_tiles = (tiles + nw - 1) / nw;
  for (uint64_t bt = blockIdx.x; bt < block_tiles; bt += gridDim.x) {
    const uint64_t t = bt * nw + wave;
    const bool active = t < tiles;
    const bool full = (t + 1) * 2048 <= n;
    if (active && full) {
      const u32x4* p = reinterpret_cast<const u32x4*>(src + t * 2048 * C);
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const int idx = lane + 64 * j;
        const int owner = idx / CH, q = idx % CH;
        tile[owner * CH + (q ^ (owner & (CH - 1)))] = __builtin_nontemporal_load(p + idx);
      }
    }
    __syncthreads();
    if (active) {
      const uint64_t g = t * 64 + lane;
      uint32_t in[1][8 * C];
      if (full) {
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          const u32x4 v = tile[lane * CH + (q ^ (lane & (CH - 1)))];
          in[0][4 * q + 0] = v.x;
          in[0][4 * q + 1] = v.y;
          in[0][4 * q + 2] = v.z;
          in[0][4 * q + 3] = v.w;
        }
      } else {
        load_std<C, 1>(src, g * 32, n, in);
      }
      uint32_t pl[8 * C];
      transpose_pack<C>(in[0], pl);
#pragma unroll
      for (int k = 0; k < 8 * C; ++k)
        if (k < B) planes[(uint64_t)k * gpad + g] = pl[k];
    }
    __syncthreads();
  }
}

// Bitslice -> standard.  Work goes in wave tiles of 64 groups (2048
// elements): a lane loads word g of each plane (coalesced) and transposes its
// group in registers.  A tile wholly below n is written through LDS, so that
// each store instruction of the wave covers one contiguous 1 KiB (the lane
// chunks are XOR-swizzled in LDS to spread banks), with non-temporal stores
// (back to back at 2^26 elements: 49.7 us against 52.2 us with ordinary
// stores); the ragged last tile stores element by element.  Loops run per block so that every thread of a
// block meets the same barriers.  Dynamic LDS: (blockDim / 64) * 2048 C bytes.
template <int C>
__global__ void __launch_bounds__(512) k_unpack(const uint32_t* planes, uint8_t* dst, uint64_t n,
                                                uint64_t gpad, int B) {
  extern __shared__ u32x4 unpack_lds[];
  constexpr int CH = 2 * C;  // 16-byte chunks per lane
  const int nw = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  u32x4* tile = unpack_lds + wave * 64 * CH;
  const uint64_t groups = (n + 31) / 32;
  const uint64_t tiles = (groups + 63) / 64;
  const uint64_t block_tiles = (tiles + nw - 1) / nw;
  for (uint64_t bt = blockIdx.x; bt < block_tiles; bt += gridDim.x) {
    const uint64_t t = bt * nw + wave;
    const bool active = t < tiles;
    const bool full = (t + 1) * 2048 <= n;
    uint32_t out[1][8 * C];
    if (active) {
      const uint64_t g = t * 64 + lane;  // < gpad: gpad = 64 * tiles
      uint32_t pl[8 * C];
#pragma unroll
      for (int k = 0; k < 8 * C; ++k) pl[k] = (k < B) ? planes[(uint64_t)k * gpad + g] : 0u;
      transpose_unpack<C>(pl, out[0]);
      if (full) {
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          u32x4 v;
          v.x = out[0][4 * q + 0];
          v.y = out[0][4 * q + 1];
          v.z = out[0][4 * q + 2];
          v.w = out[0][4 * q + 3];
          tile[lane * CH + (q ^ (lane & (CH - 1)))] = v;
        }
      } else {
        store_std<C, 1>(dst, g * 32, n, out);
      }
    }
    __syncthreads();
    if (active && full) {
      u32x4* p = reinterpret_cast<u32x4*>(dst + t * 2048 * C);
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const int idx = lane + 64 * j;
        const int owner = idx / CH, q = idx % CH;
        __builtin_nontemporal_store(tile[owner * CH + (q ^ (owner & (CH - 1)))], p + idx);
      }
    }
    __syncthreads();
  }
}

// Fused standard-in / standard-out op: transposes and circuit in registers.
// `nb` and `ng`: block and grid sizes, read by the kernel (as in k_binop).
template <int E, int M, bool RZ, int OPC>
__device__ __forceinline__ void binop_std_body(const uint8_t* a, const uint8_t* b, uint8_t* c, uint64_t n,
                                               uint32_t negb, unsigned nb, unsigned ng) {
  constexpr int B = 1 + E + M;
  constexpr int C = B <= 8 ? 1 : (B <= 16 ? 2 : (B <= 32 ? 4 : 8));
  const uint64_t groups = (n + 31) / 32;
  const uint64_t stride = (uint64_t)ng * nb;
  for (uint64_t t = (uint64_t)blockIdx.x * nb + threadIdx.x; t < groups; t += stride) {
    uint32_t ia[1][8 * C], ib[1][8 * C];
    load_std<C, 1>(a, t * 32, n, ia);
    load_std<C, 1>(b, t * 32, n, ib);
    uint32_t pa[8 * C], pb[8 * C];
    transpose_pack<C>(ia[0], pa);
    transpose_pack<C>(ib[0], pb);
    WordR<1> x[B], y[B], z[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      x[k].w[0] = pa[k];
      y[k].w[0] = pb[k];
    }
    circuit<E, M, RZ, OPC, 1>(x, y, negb, z);
    uint32_t pz[8 * C];
#pragma unroll
    for (int k = 0; k < 8 * C; ++k) pz[k] = (k < B) ? z[k].w[0] : 0u;
    uint32_t oc[1][8 * C];
    transpose_unpack<C>(pz, oc[0]);
    store_std<C, 1>(c, t * 32, n, oc);
  }
}

template <int E, int M, bool RZ, int OPC>
__global__ void __launch_bounds__(512) k_binop_std(const uint8_t* a, const uint8_t* b, uint8_t* c, uint64_t n,
                                                   uint32_t negb) {
  binop_std_body<E, M, RZ, OPC>(a, b, c, n, negb, blockDim.x, gridDim.x);
}

// The wide formats' fused kernels hold two 64-word operands and their
// transposes at once: blocks of at most 256 threads let the compiler use 512
// registers per lane (accumulation registers included) instead of spilling
// to scratch (measured at (11,52) mul: 234 registers spilled under the
// 512-thread bound).  The bitslice kernels keep the 512-thread bound: for
// them a few spilled registers cost less than halving the resident waves
// (binary64 mul 645 us against 836 us at 2^26 elements).
template <int E, int M, bool RZ, int OPC>
__global__ void __launch_bounds__(256) k_binop_std_w(const uint8_t* a, const uint8_t* b, uint8_t* c, uint64_t n,
                                                     uint32_t negb) {
  binop_std_body<E, M, RZ, OPC>(a, b, c, n, negb, blockDim.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Launchers and the registry of compiled variants
// ---------------------------------------------------------------------------
using BinopLauncher = hipError_t (*)(const void* a, const void* b, void* c, uint64_t gpad, uint64_t n, uint32_t negb,
                                     unsigned grid, unsigned block, hipStream_t s);
using StdLauncher = hipError_t (*)(const void* a, const void* b, void* c, uint64_t n, uint32_t negb,
                                   unsigned grid, unsigned block, hipStream_t s);

using ChainLauncher = hipError_t (*)(const void* a, uint32_t alpha, const void* b, const void* c, void* d,
                                     uint64_t gpad, uint64_t n, uint32_t negb1, uint32_t negb2, unsigned grid,
                                     unsigned block, hipStream_t s);

// Launch shapes of the elementwise kernels: R words per lane in {1, 2, 4}
// (index 0, 1, 2) and U units per loop step in {1, 2} (index 0, 1).
constexpr int kWordChoices = 3;
constexpr int kUnrollChoices = 2;
constexpr int r_index(int r) { return r == 1 ? 0 : (r == 2 ? 1 : (r == 4 ? 2 : -1)); }

// Four words per lane are compiled for the formats of at most 10 bits,
// whose circuits leave the registers for them.
constexpr bool four_words_ok(int e, int m) { return 1 + e + m <= 10; }

struct Registry {
  // [e][m][opclass][rz][r_index(R)][U-1]
  BinopLauncher binop[kMaxE + 1][kMaxM + 1][kOpClasses][2][kWordChoices][kUnrollChoices] = {};
  StdLauncher std_op[kMaxE + 1][kMaxM + 1][kOpClasses][2] = {};
  // two-op chains: [e][m][opclass of op1][opclass of op2][rz], op classes
  // 0 (add/sub) and 1 (mul)
  ChainLauncher chain[kMaxE + 1][kMaxM + 1][2][2][2] = {};
  // largest block the format's binop kernels are compiled for (0: none)
  int max_block[kMaxE + 1][kMaxM + 1] = {};
};
Registry& registry();

template <int E, int M, bool RZ, int OPC, int R, int U>
hipError_t launch_binop(const void* a, const void* b, void* c, uint64_t gpad, uint64_t n, uint32_t negb, unsigned grid,
                        unsigned block, hipStream_t s) {
  hipLaunchKernelGGL((k_binop<E, M, RZ, OPC, R, U>), dim3(grid), dim3(block), 0, s,
                     static_cast<const uint32_t*>(a), static_cast<const uint32_t*>(b),
                     static_cast<uint32_t*>(c), gpad, n, negb);
  return hipGetLastError();
}

template <int E, int M, bool RZ, int OPC>
hipError_t launch_binop_std(const void* a, const void* b, void* c, uint64_t n, uint32_t negb, unsigned grid,
                            unsigned block, hipStream_t s) {
  hipLaunchKernelGGL((k_binop_std<E, M, RZ, OPC>), dim3(grid), dim3(block), 0, s,
                     static_cast<const uint8_t*>(a), static_cast<const uint8_t*>(b), static_cast<uint8_t*>(c),
                     n, negb);
  return hipGetLastError();
}

template <int E, int M, bool RZ, int OPC>
hipError_t launch_binop_std_w(const void* a, const void* b, void* c, uint64_t n, uint32_t negb, unsigned grid,
                              unsigned block, hipStream_t s) {
  hipLaunchKernelGGL((k_binop_std_w<E, M, RZ, OPC>), dim3(grid), dim3(block), 0, s,
                     static_cast<const uint8_t*>(a), static_cast<const uint8_t*>(b), static_cast<uint8_t*>(c),
                     n, negb);
  return hipGetLastError();
}

template <int E, int M, int OPC, bool RZ>
void register_shapes() {
  Registry& r = registry();
  auto& L = r.binop[E][M][OPC][RZ ? 1 : 0];
  L[0][0] = launch_binop<E, M, RZ, OPC, 1, 1>;
  L[1][0] = launch_binop<E, M, RZ, OPC, 2, 1>;
  L[0][1] = launch_binop<E, M, RZ, OPC, 1, 2>;
  if constexpr (four_words_ok(E, M)) L[2][0] = launch_binop<E, M, RZ, OPC, 4, 1>;
}

template <int E, int M>
void register_format() {
  Registry& r = registry();
  r.max_block[E][M] = 512;
  register_shapes<E, M, 0, false>();
  register_shapes<E, M, 0, true>();
  register_shapes<E, M, 1, false>();
  register_shapes<E, M, 1, true>();
  register_shapes<E, M, 2, false>();
  register_shapes<E, M, 2, true>();
  r.std_op[E][M][0][0] = launch_binop_std<E, M, false, 0>;
  r.std_op[E][M][0][1] = launch_binop_std<E, M, true, 0>;
  r.std_op[E][M][1][0] = launch_binop_std<E, M, false, 1>;
  r.std_op[E][M][1][1] = launch_binop_std<E, M, true, 1>;
  r.std_op[E][M][2][0] = launch_binop_std<E, M, false, 2>;
  r.std_op[E][M][2][1] = launch_binop_std<E, M, true, 2>;
}

// Wide formats: one 32-element word per lane (two would double registers
// that the 64-plane circuits already fill), every op class, both modes.
template <int E, int M>
void register_wide_format() {
  Registry& r = registry();
  r.max_block[E][M] = 512;
#define BFP_WIDE_REG(OPC)                                           \
  r.binop[E][M][OPC][0][0][0] = launch_binop<E, M, false, OPC, 1, 1>; \
  r.binop[E][M][OPC][1][0][0] = launch_binop<E, M, true, OPC, 1, 1>;  \
  r.std_op[E][M][OPC][0] = launch_binop_std_w<E, M, false, OPC>;   \
  r.std_op[E][M][OPC][1] = launch_binop_std_w<E, M, true, OPC>;
  BFP_WIDE_REG(0)
  BFP_WIDE_REG(1)
  BFP_WIDE_REG(2)
#undef BFP_WIDE_REG
}

}  // namespace bfp
