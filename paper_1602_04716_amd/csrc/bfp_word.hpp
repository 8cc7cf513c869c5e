// bfp_word.hpp -- machine words of a bitslice vector and the gates on them.
//
// A bitslice word holds one bit of 32 elements (Section 2; Figure 3 uses one
// integer per bit of the format).  A lane may hold R adjacent 32-bit words of
// every plane (W = 32 R elements per lane); all gates act on each word alike.
//
// On gfx950 every 3-input boolean function is one instruction,
// v_bitop3_b32, reached through __builtin_amdgcn_bitop3_b32; its 8-bit
// immediate is the truth table indexed by (a << 2) | (b << 1) | c.  The same
// functions evaluate on the host (to test the circuits on the CPU) from the
// truth table, and a counting word type tallies gates for the cost model.
#pragma once
#include <stdint.h>

#ifdef __HIPCC__
#include <hip/hip_runtime.h>
#define BFP_FN __host__ __device__ __forceinline__
#else
#define BFP_FN inline
#endif

namespace bfp {

// Truth tables of the three inputs; a gate's immediate is the same boolean
// expression applied to them, e.g. majority = (A&B)|(A&C)|(B&C) = 0xE8.
constexpr unsigned TA = 0xF0, TB = 0xCC, TC = 0xAA;
constexpr unsigned imm8(unsigned v) { return v & 0xFFu; }

constexpr unsigned IMM_XOR3 = imm8(TA ^ TB ^ TC);                              // 0x96
constexpr unsigned IMM_XNOR3 = imm8(~(TA ^ TB ^ TC));                          // 0x69
constexpr unsigned IMM_MAJ = imm8((TA & TB) | (TA & TC) | (TB & TC));          // 0xE8
constexpr unsigned IMM_MAJ_NA = imm8((~TA & TB) | (~TA & TC) | (TB & TC));     // maj(~a,b,c)
constexpr unsigned IMM_MAJ_NB = imm8((TA & ~TB) | (TA & TC) | (~TB & TC));     // maj(a,~b,c)
constexpr unsigned IMM_MUX = imm8((TA & TB) | (~TA & TC));                     // a ? b : c
constexpr unsigned IMM_OR3 = imm8(TA | TB | TC);
constexpr unsigned IMM_NOR3 = imm8(~(TA | TB | TC));
constexpr unsigned IMM_AND3 = imm8(TA & TB & TC);
constexpr unsigned IMM_AND_OR = imm8(TA & (TB | TC));                          // a & (b | c)
constexpr unsigned IMM_ANDN_OR = imm8((TA & ~TB) | TC);                        // (a & ~b) | c
constexpr unsigned IMM_AND_NOR = imm8(TA & ~(TB | TC));                        // a & ~(b | c)
constexpr unsigned IMM_XOR_AND = imm8((TA ^ TB) & TC);                         // (a ^ b) & c
constexpr unsigned IMM_OR_AND = imm8((TA | TB) & TC);                          // (a | b) & c
constexpr unsigned IMM_AND_XOR = imm8((TA & TB) ^ TC);                         // (a & b) ^ c

// ---------------------------------------------------------------------------
// One 32-bit word
// ---------------------------------------------------------------------------
template <unsigned IMM>
BFP_FN uint32_t bitop3(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_bitop3_b32(a, b, c, IMM);
#else
  uint32_t r = 0;
  for (unsigned idx = 0; idx < 8; ++idx) {
    if ((IMM >> idx) & 1u) {
      uint32_t t = ((idx & 4u) ? a : ~a) & ((idx & 2u) ? b : ~b) & ((idx & 1u) ? c : ~c);
      r |= t;
    }
  }
  return r;
#endif
}

// ---------------------------------------------------------------------------
// R adjacent words per lane (W = 32 R elements)
// ---------------------------------------------------------------------------
template <int R>
struct WordR {
  uint32_t w[R];
};

template <int R>
BFP_FN WordR<R> operator&(WordR<R> a, WordR<R> b) {
  WordR<R> r;
#pragma unroll
  for (int i = 0; i < R; ++i) r.w[i] = a.w[i] & b.w[i];
  return r;
}
template <int R>
BFP_FN WordR<R> operator|(WordR<R> a, WordR<R> b) {
  WordR<R> r;
#pragma unroll
  for (int i = 0; i < R; ++i) r.w[i] = a.w[i] | b.w[i];
  return r;
}
template <int R>
BFP_FN WordR<R> operator^(WordR<R> a, WordR<R> b) {
  WordR<R> r;
#pragma unroll
  for (int i = 0; i < R; ++i) r.w[i] = a.w[i] ^ b.w[i];
  return r;
}
template <int R>
BFP_FN WordR<R> operator~(WordR<R> a) {
  WordR<R> r;
#pragma unroll
  for (int i = 0; i < R; ++i) r.w[i] = ~a.w[i];
  return r;
}
template <unsigned IMM, int R>
BFP_FN WordR<R> bitop3(WordR<R> a, WordR<R> b, WordR<R> c) {
  WordR<R> r;
#pragma unroll
  for (int i = 0; i < R; ++i) r.w[i] = bitop3<IMM>(a.w[i], b.w[i], c.w[i]);
  return r;
}

// Word traits: all-zero / all-one words of a type.
template <class W>
struct WordTraits;
template <>
struct WordTraits<uint32_t> {
  static BFP_FN uint32_t zero() { return 0u; }
  static BFP_FN uint32_t ones() { return ~0u; }
};
template <int R>
struct WordTraits<WordR<R>> {
  static BFP_FN WordR<R> zero() {
    WordR<R> r;
#pragma unroll
    for (int i = 0; i < R; ++i) r.w[i] = 0u;
    return r;
  }
  static BFP_FN WordR<R> ones() {
    WordR<R> r;
#pragma unroll
    for (int i = 0; i < R; ++i) r.w[i] = ~0u;
    return r;
  }
};

#ifndef __HIPCC__
// ---------------------------------------------------------------------------
// Host-only: a 64-bit word (W = 64 on the CPU) and a gate-counting word.
// ---------------------------------------------------------------------------
template <unsigned IMM>
inline uint64_t bitop3(uint64_t a, uint64_t b, uint64_t c) {
  uint64_t r = 0;
  for (unsigned idx = 0; idx < 8; ++idx)
    if ((IMM >> idx) & 1u) r |= ((idx & 4u) ? a : ~a) & ((idx & 2u) ? b : ~b) & ((idx & 1u) ? c : ~c);
  return r;
}
template <>
struct WordTraits<uint64_t> {
  static inline uint64_t zero() { return 0ull; }
  static inline uint64_t ones() { return ~0ull; }
};

// Gate-counting word: each gate whose inputs are not all constant counts one;
// AND/OR/XOR with a constant fold away as they do in the compiled code.
struct CountW {
  static unsigned long &counter() {
    static thread_local unsigned long c = 0;
    return c;
  }
  signed char k = -1;  // -1: variable; 0: constant all-zero; 1: constant all-one
};
inline CountW cw_var() {
  CountW::counter()++;
  return CountW{-1};
}
inline CountW operator&(CountW a, CountW b) {
  if (a.k == 0 || b.k == 0) return CountW{0};
  if (a.k == 1) return b;
  if (b.k == 1) return a;
  return cw_var();
}
inline CountW operator|(CountW a, CountW b) {
  if (a.k == 1 || b.k == 1) return CountW{1};
  if (a.k == 0) return b;
  if (b.k == 0) return a;
  return cw_var();
}
inline CountW operator^(CountW a, CountW b) {
  if (a.k >= 0 && b.k >= 0) return CountW{(signed char)(a.k ^ b.k)};
  if (a.k == 0) return b;
  if (b.k == 0) return a;
  return cw_var();
}
inline CountW operator~(CountW a) {
  if (a.k >= 0) return CountW{(signed char)(1 - a.k)};
  return cw_var();
}
template <unsigned IMM>
inline CountW bitop3(CountW a, CountW b, CountW c) {
  if (a.k >= 0 && b.k >= 0 && c.k >= 0)
    return CountW{(signed char)((IMM >> ((a.k << 2) | (b.k << 1) | c.k)) & 1u)};
  return cw_var();
}
template <>
struct WordTraits<CountW> {
  static inline CountW zero() { return CountW{0}; }
  static inline CountW ones() { return CountW{1}; }
};
#endif

}  // namespace bfp
