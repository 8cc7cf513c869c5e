// Integer-vector kernel instances for k = 9 .. 16: add, sub, mul, each
// wrapping, unsigned-saturating and signed-saturating.
#include "bfp_formats.hpp"
#include "bfp_int_kernels.hpp"

namespace {
struct RegisterIntK9 {
  RegisterIntK9() {
#define BFP_REG(K) bfp::register_int<K>();
    BFP_FOR_EACH_INT_K_9_16(BFP_REG)
#undef BFP_REG
  }
} register_int_k9;
}  // namespace
