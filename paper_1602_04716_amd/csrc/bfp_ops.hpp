// bfp_ops.hpp -- operation codes of the C ABI mapped to compiled circuits.
#pragma once
#include "bfp.h"

namespace bfp {

// Operation classes, one compiled circuit each: 0 add/sub (subtraction runs
// the adder with the second operand's sign flipped), 1 mul, 2 div.
constexpr int kOpClasses = 3;
inline int opclass_of(int op) { return op == BFP_MUL ? 1 : (op == BFP_DIV ? 2 : 0); }
inline bool op_valid(int op) { return op == BFP_ADD || op == BFP_SUB || op == BFP_MUL || op == BFP_DIV; }

}  // namespace bfp
