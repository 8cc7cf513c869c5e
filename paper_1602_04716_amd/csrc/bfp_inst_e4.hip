// Kernel instances for the formats with e = 4 (every compiled m), both
// operation classes, both rounding modes and both word widths.
#include "bfp_formats.hpp"
#include "bfp_kernels.hpp"

namespace {
struct RegisterE4 {
  RegisterE4() {
#define BFP_REG(E, M) bfp::register_format<E, M>();
    BFP_FOR_EACH_M(BFP_REG, 4)
#undef BFP_REG
  }
} register_e4;
}  // namespace
