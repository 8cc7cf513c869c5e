// Integer-vector kernel instances for k = 25 .. 32: add, sub, mul, each
// wrapping, unsigned-saturating and signed-saturating.
#include "bfp_formats.hpp"
#include "bfp_int_kernels.hpp"

namespace {
struct RegisterIntK25 {
  RegisterIntK25() {
#define BFP_REG(K) bfp::register_int<K>();
    BFP_FOR_EACH_INT_K_25_32(BFP_REG)
#undef BFP_REG
  }
} register_int_k25;
}  // namespace
