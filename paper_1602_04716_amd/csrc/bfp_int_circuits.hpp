// bfp_int_circuits.hpp -- k-bit integer arithmetic on bitslice words
// (Section 3: vectors of elements of any bit length; Figure 2: the ripple
// adder).  An element is a k-bit pattern; plane i holds bit i.  Three kinds:
//   kIntWrap  the result modulo 2^k (Figure 2 with the last carry dropped;
//             the same bits for signed and unsigned operands),
//   kIntSatU  unsigned operands, result clamped to [0, 2^k - 1],
//   kIntSatS  two's complement operands, result clamped to
//             [-2^(k-1), 2^(k-1) - 1].
#pragma once
#include "bfp_circuits.hpp"

namespace bfp {

constexpr int kIntWrap = 0, kIntSatU = 1, kIntSatS = 2;
constexpr int kMaxIntBits = 32;

// r = a + b + cin0 (K bits) with cin0 = 0 (add) or, for a - b = a + ~b + 1,
// the operand b inverted and cin0 = 1.  *c_top receives the carry into bit
// K-1, *c_out the carry out of bit K-1.
template <int K, bool SUB, class W>
BFP_FN void int_addsub_carries(const W* a, const W* b, W* r, W* c_top, W* c_out) {
  W c;
  if constexpr (SUB) {
    *c_top = WordTraits<W>::ones();  // carry into bit 0 (K = 1)
    r[0] = g_xor(a[0], b[0]);        // a ^ ~b ^ 1
    c = g_orn(a[0], b[0]);           // maj(a, ~b, 1)
  } else {
    *c_top = WordTraits<W>::zero();
    r[0] = g_xor(a[0], b[0]);
    c = g_and(a[0], b[0]);
  }
#pragma unroll
  for (int i = 1; i < K; ++i) {
    *c_top = c;
    if constexpr (SUB) {
      r[i] = g3<IMM_XNOR3>(a[i], b[i], c);
      c = g3<IMM_MAJ_NB>(a[i], b[i], c);
    } else {
      r[i] = g_xor3(a[i], b[i], c);
      c = g_maj(a[i], b[i], c);
    }
  }
  *c_out = c;
}

// Clamp to the signed bound of sign s where ov is set: bits below K-1 become
// ~s, bit K-1 becomes s (s = 0: 011..1, s = 1: 100..0).
template <int K, class W>
BFP_FN void int_clamp_signed(W* r, W ov, W s) {
#pragma unroll
  for (int i = 0; i + 1 < K; ++i) r[i] = g3<imm8((TA & ~TB) | (~TA & TC))>(ov, s, r[i]);
  r[K - 1] = g_mux(ov, s, r[K - 1]);
}

// Low K bits of a * b: row j adds (a & b_j) << j, truncated to K bits.
template <int K, class W>
BFP_FN void int_mul_lo(const W* a, const W* b, W* r) {
#pragma unroll
  for (int i = 0; i < K; ++i) r[i] = g_and(a[i], b[0]);
#pragma unroll
  for (int j = 1; j < K; ++j) {
    W c = WordTraits<W>::zero();
#pragma unroll
    for (int i = 0; i + j < K; ++i) {
      const int pos = i + j;
      const W pp = g_and(a[i], b[j]);
      const W x = r[pos];
      if (i == 0) {
        r[pos] = g_xor(x, pp);
        if (pos + 1 < K) c = g_and(x, pp);
      } else {
        r[pos] = g_xor3(x, pp, c);
        if (pos + 1 < K) c = g_maj(x, pp, c);
      }
    }
  }
}

// Full 2K-bit product P = a * b (unsigned): an array multiplier whose
// accumulator stays K + 1 words wide, the low bit retiring after each row.
template <int K, class W>
BFP_FN void int_mul_full(const W* a, const W* b, W* P) {
  W acc[K + 1];
#pragma unroll
  for (int i = 0; i < K; ++i) acc[i] = g_and(a[i], b[0]);
  acc[K] = WordTraits<W>::zero();
#pragma unroll
  for (int j = 1; j < K; ++j) {
    P[j - 1] = acc[0];
    W c = WordTraits<W>::zero();
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const W x = acc[i + 1];
      const W pp = g_and(a[i], b[j]);
      if (i == 0) {
        acc[0] = g_xor(x, pp);
        c = g_and(x, pp);
      } else if (j == 1 && i == K - 1) {  // acc[K] is still zero in the first row
        acc[i] = g_xor(pp, c);
        c = g_and(pp, c);
      } else {
        acc[i] = g_xor3(x, pp, c);
        c = g_maj(x, pp, c);
      }
    }
    acc[K] = c;
  }
#pragma unroll
  for (int i = 0; i <= K; ++i) P[K - 1 + i] = acc[i];
}

// x = s ? -x : x (K bits, modulo 2^K): (x ^ s) + s.
template <int K, class W>
BFP_FN void int_cond_negate(W* x, W s) {
#pragma unroll
  for (int i = 0; i < K; ++i) x[i] = g_xor(x[i], s);
  increment<K>(x, s);
}

// r = a op b; OP 0 add, 1 sub, 2 mul; KIND as above.
template <int K, int OP, int KIND, class W>
BFP_FN void int_circuit(const W* a, const W* b, W* r) {
  static_assert(K >= 1 && K <= kMaxIntBits, "1 <= k <= 32");
  if constexpr (OP == 0 && KIND == kIntWrap) {
    if constexpr (K == 1) r[0] = g_xor(a[0], b[0]);
    else ripple_add<K, W>(a, b, r);  // Figure 2
  } else if constexpr (OP == 1 && KIND == kIntWrap) {
#pragma unroll
    for (int i = 0; i < K; ++i) r[i] = a[i];
    sub_zext<K, K, W>(r, b);
  } else if constexpr (OP <= 1) {
    W c_top, c_out;
    int_addsub_carries<K, OP == 1, W>(a, b, r, &c_top, &c_out);
    if constexpr (KIND == kIntSatU) {
      // add: a carry out means the sum exceeds 2^k - 1; sub: no carry out
      // (a borrow) means a < b
#pragma unroll
      for (int i = 0; i < K; ++i) r[i] = OP == 0 ? g_or(r[i], c_out) : g_and(r[i], c_out);
    } else {
      // signed overflow: the carries into and out of the sign bit differ;
      // the exact result then has the sign of a
      int_clamp_signed<K, W>(r, g_xor(c_top, c_out), a[K - 1]);
    }
  } else if constexpr (KIND == kIntWrap) {
    int_mul_lo<K, W>(a, b, r);
  } else if constexpr (KIND == kIntSatU) {
    W P[2 * K];
    int_mul_full<K, W>(a, b, P);
    const W ov = or_range<K, 2 * K>(P);  // product >= 2^k
#pragma unroll
    for (int i = 0; i < K; ++i) r[i] = g_or(P[i], ov);
  } else {
    // signed: multiply the magnitudes (|-2^(k-1)| = 2^(k-1) fits in k
    // unsigned bits), then negate when the signs differ
    const W s = g_xor(a[K - 1], b[K - 1]);
    W ma[K], mb[K], P[2 * K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      ma[i] = a[i];
      mb[i] = b[i];
    }
    int_cond_negate<K, W>(ma, a[K - 1]);
    int_cond_negate<K, W>(mb, b[K - 1]);
    int_mul_full<K, W>(ma, mb, P);
    // positive results overflow at |P| >= 2^(k-1), negative ones at > 2^(k-1)
    const W hi = or_range<K, 2 * K>(P);
    const W ov_pos = g_or(hi, P[K - 1]);
    W ov_neg = hi;
    if constexpr (K > 1) ov_neg = g3<imm8(TA | (TB & TC))>(hi, P[K - 1], or_range<0, cmax(K - 1, 1)>(P));
    const W ov = g_mux(s, ov_neg, ov_pos);
#pragma unroll
    for (int i = 0; i < K; ++i) r[i] = P[i];
    int_cond_negate<K, W>(r, s);
    int_clamp_signed<K, W>(r, ov, s);
  }
}

}  // namespace bfp
