// Two-op chain kernel instances for the formats with e = 6 (every compiled
// m), op classes add/sub and mul in both positions, both rounding modes.
#include "bfp_chain.hpp"
#include "bfp_formats.hpp"

namespace {
struct RegisterChainE6 {
  RegisterChainE6() {
#define BFP_REG(E, M) bfp::register_chain<E, M>();
    BFP_FOR_EACH_M(BFP_REG, 6)
#undef BFP_REG
  }
} register_chain_e6;
}  // namespace
