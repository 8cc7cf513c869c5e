// Kernel instances for the wide formats (exponent up to 11 bits, patterns up
// to 64 bits): every operation class, both rounding modes, one word per lane.
#include "bfp_formats.hpp"
#include "bfp_kernels.hpp"

namespace {
struct RegisterWide {
  RegisterWide() {
#define BFP_REG(E, M) bfp::register_wide_format<E, M>();
    BFP_FOR_EACH_WIDE_FORMAT(BFP_REG)
#undef BFP_REG
  }
} register_wide;
}  // namespace
