// bfp_cost.cpp -- gate counts of the compiled circuits (the cost model of
// Table 1), from the same netlists the kernels run, evaluated on a counting
// word type on the host.  Built with the host compiler into libbfp.
#include "bfp.h"
#include "bfp_circuits.hpp"
#include "bfp_formats.hpp"

namespace {
template <int E, int M, bool RZ>
long count(int op) {
  using bfp::CountW;
  constexpr int B = 1 + E + M;
  CountW x[B], y[B], z[B];
  CountW::counter() = 0;
  if (op == BFP_MUL)
    bfp::fp_mul<E, M, RZ, CountW>(x, y, z);
  else if (op == BFP_DIV)
    bfp::fp_div<E, M, RZ, CountW>(x, y, z);
  else
    bfp::fp_add<E, M, RZ, CountW>(x, y, CountW{}, z);
  return (long)CountW::counter();
}
}  // namespace

extern "C" long bfp_gate_count(int op, bfp_format f) {
  if (op < BFP_ADD || op > BFP_DIV) return -1;
  if (f.round > 1 || f.pad != 0) return -1;
#define BFP_COUNT_CASE(EE, MM) \
  if (f.e == EE && f.m == MM) return f.round ? count<EE, MM, true>(op) : count<EE, MM, false>(op);
  BFP_FOR_EACH_FORMAT(BFP_COUNT_CASE)
  BFP_FOR_EACH_WIDE_FORMAT(BFP_COUNT_CASE)
#undef BFP_COUNT_CASE
  return -1;
}
