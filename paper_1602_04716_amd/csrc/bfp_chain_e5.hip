// Two-op chain kernel instances for the formats with e = 5 (every compiled
// m), op classes add/sub and mul in both positions, both rounding modes.
#include "bfp_chain.hpp"
#include "bfp_formats.hpp"

namespace {
struct RegisterChainE5 {
  RegisterChainE5() {
#define BFP_REG(E, M) bfp::register_chain<E, M>();
    BFP_FOR_EACH_M(BFP_REG, 5)
#undef BFP_REG
  }
} register_chain_e5;
}  // namespace
