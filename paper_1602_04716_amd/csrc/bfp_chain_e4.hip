// Two-op chain kernel instances for the formats with e = 4 (every compiled
// m), op classes add/sub and mul in both positions, both rounding modes.
#include "bfp_chain.hpp"
#include "bfp_formats.hpp"

namespace {
struct RegisterChainE4 {
  RegisterChainE4() {
#define BFP_REG(E, M) bfp::register_chain<E, M>();
    BFP_FOR_EACH_M(BFP_REG, 4)
#undef BFP_REG
  }
} register_chain_e4;
}  // namespace
