// bfp_host_sim.cpp -- the circuits of bfp_circuits.hpp instantiated for the
// host CPU (32- and 64-bit words), to test the netlists against the oracle
// without a GPU, and the gate-count model.  Test-only library: the GPU
// library never loads it and nothing falls back to it.
#include <stdint.h>
#include <string.h>

#include "bfp_circuits.hpp"
#include "bfp_formats.hpp"

namespace {

template <class W>
constexpr int kBits = sizeof(W) * 8;

// Run one circuit over n standard patterns (low 1+e+m bits of uint32 words).
template <int E, int M, bool RZ, class W>
void run(int op, const uint32_t* a, const uint32_t* b, uint32_t* c, uint64_t n) {
  constexpr int B = 1 + E + M;
  constexpr int WB = kBits<W>;
  const W negb = (op == 1) ? bfp::WordTraits<W>::ones() : bfp::WordTraits<W>::zero();
  for (uint64_t base = 0; base < n; base += WB) {
    W x[B], y[B], z[B];
    for (int k = 0; k < B; ++k) {
      W wx = 0, wy = 0;
      for (int j = 0; j < WB && base + j < n; ++j) {
        wx |= (W)((a[base + j] >> k) & 1u) << j;
        wy |= (W)((b[base + j] >> k) & 1u) << j;
      }
      x[k] = wx;
      y[k] = wy;
    }
    if (op == 2)
      bfp::fp_mul<E, M, RZ, W>(x, y, z);
    else
      bfp::fp_add<E, M, RZ, W>(x, y, negb, z);
    for (int j = 0; j < WB && base + j < n; ++j) {
      uint32_t v = 0;
      for (int k = 0; k < B; ++k) v |= (uint32_t)((z[k] >> j) & 1u) << k;
      c[base + j] = v;
    }
  }
}

template <int E, int M, bool RZ>
unsigned long gates(int op) {
  using bfp::CountW;
  constexpr int B = 1 + E + M;
  CountW x[B], y[B], z[B];
  CountW::counter() = 0;
  if (op == 2)
    bfp::fp_mul<E, M, RZ, CountW>(x, y, z);
  else
    bfp::fp_add<E, M, RZ, CountW>(x, y, CountW{}, z);
  return CountW::counter();
}

}  // namespace

extern "C" {

// op: 0 add, 1 sub, 2 mul; mode: 0 nearest-even, 1 toward zero; wbits 32/64.
// Returns 0, or -1 for a format that is not compiled.
int bfpsim_binop(int op, int e, int m, int mode, int wbits, const uint32_t* a, const uint32_t* b,
                 uint32_t* c, uint64_t n) {
#define BFP_SIM_CASE(EE, MM)                                                             \
  if (e == EE && m == MM) {                                                              \
    if (wbits == 64) {                                                                   \
      if (mode) run<EE, MM, true, uint64_t>(op, a, b, c, n);                             \
      else run<EE, MM, false, uint64_t>(op, a, b, c, n);                                 \
    } else {                                                                             \
      if (mode) run<EE, MM, true, uint32_t>(op, a, b, c, n);                             \
      else run<EE, MM, false, uint32_t>(op, a, b, c, n);                                 \
    }                                                                                    \
    return 0;                                                                            \
  }
  BFP_FOR_EACH_FORMAT(BFP_SIM_CASE)
#undef BFP_SIM_CASE
  return -1;
}

// Gates of one circuit instance (one word group), constants folded.
long bfpsim_gate_count(int op, int e, int m, int mode) {
#define BFP_GC_CASE(EE, MM) \
  if (e == EE && m == MM) return (long)(mode ? gates<EE, MM, true>(op) : gates<EE, MM, false>(op));
  BFP_FOR_EACH_FORMAT(BFP_GC_CASE)
#undef BFP_GC_CASE
  return -1;
}

// Figure 2: 13-bit bitslice integer adder over 32 lanes.  a, b, r hold 13
// plane words each (plane k = bit k of the 32 lane values).
void bfpsim_ripple_add13(const uint32_t* a, const uint32_t* b, uint32_t* r) {
  bfp::ripple_add<13, uint32_t>(a, b, r);
}

}  // extern "C"

#include "bfp_transpose.hpp"

extern "C" {
// 32 elements of C bytes (8C dwords) <-> 8C plane words, as the GPU kernels do it.
int bfpsim_transpose(int C, int inverse, const uint32_t* in, uint32_t* out) {
  switch (C * 2 + (inverse ? 1 : 0)) {
    case 2: bfp::transpose_pack<1>(in, out); return 0;
    case 3: bfp::transpose_unpack<1>(in, out); return 0;
    case 4: bfp::transpose_pack<2>(in, out); return 0;
    case 5: bfp::transpose_unpack<2>(in, out); return 0;
    case 8: bfp::transpose_pack<4>(in, out); return 0;
    case 9: bfp::transpose_unpack<4>(in, out); return 0;
    default: return -1;
  }
}
}
