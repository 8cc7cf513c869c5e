// bfp_formats.hpp -- the (e, m) formats compiled into the library.
//
// The paper's generator emits one library per (exponent bits, mantissa bits,
// rounding mode) configuration (Section 5.1); here every format of the sweep
// e in {3,4,5,6,8} x m in {1,2,3,5,7,10,15,23} is instantiated once per
// operation class and rounding mode, which covers FP8 (4,3), FP16 (5,10) and
// FP32 (8,23) of Section 5.2 and bfloat16 (8,7); four wider formats follow.
#pragma once

// X(e, m) for every compiled format
#define BFP_FOR_EACH_M(X, e) X(e, 1) X(e, 2) X(e, 3) X(e, 5) X(e, 7) X(e, 10) X(e, 15) X(e, 23)
#define BFP_FOR_EACH_FORMAT(X) \
  BFP_FOR_EACH_M(X, 3) BFP_FOR_EACH_M(X, 4) BFP_FOR_EACH_M(X, 5) BFP_FOR_EACH_M(X, 6) BFP_FOR_EACH_M(X, 8)

// X(k) for every integer width of the bitslice integer vectors, 1 <= k <= 32
#define BFP_FOR_EACH_INT_K_1_8(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)
#define BFP_FOR_EACH_INT_K_9_16(X) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
#define BFP_FOR_EACH_INT_K_17_24(X) X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24)
#define BFP_FOR_EACH_INT_K_25_32(X) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)
#define BFP_FOR_EACH_INT_K(X) \
  BFP_FOR_EACH_INT_K_1_8(X) BFP_FOR_EACH_INT_K_9_16(X) BFP_FOR_EACH_INT_K_17_24(X) BFP_FOR_EACH_INT_K_25_32(X)

// Formats wider than the sweep (exponent up to 11 bits, patterns up to 64
// bits in 8-byte containers above 32 bits); (11,52) is IEEE binary64.  They
// have the elementwise ops with 32-element lane words and the fused standard
// path, but no two-op chains and no batch or serving kernels, whose register
// allocation they would set.
#define BFP_FOR_EACH_WIDE_FORMAT(X) X(8, 31) X(11, 20) X(11, 40) X(11, 52)

namespace bfp {
constexpr int kMaxE = 11;
constexpr int kMaxM = 52;
}  // namespace bfp
