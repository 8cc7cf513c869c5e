// bfp_transpose.hpp -- standard <-> bitslice transposes of 32 elements held
// by one lane (the paper's helper transforms, Section 4; layout of Figure 1).
//
// Standard side: 32 elements of C bytes (C = 1, 2, 4), element j at byte
// j*C, i.e. 8*C dwords.  Bitslice side: 8*C plane words, plane k holding bit
// k of element j at bit j.
//
// Method: view the 32 x 8C bit matrix as 4 x C blocks of 8 x 8 bits.  Each
// block (one byte of 8 consecutive elements) is gathered into a 64-bit pair
// of dwords by byte shuffles (v_perm_b32 on gfx9), transposed in three
// delta-swap steps, and its 8 result bytes are scattered to 8 plane words
// by byte shuffles.  Unpack runs the same steps in reverse; the 8 x 8
// transpose is its own inverse.
#pragma once
#include "bfp_word.hpp"

namespace bfp {

BFP_FN uint32_t byte_at(const uint32_t* v, int idx) { return (v[idx >> 2] >> (8 * (idx & 3))) & 0xFFu; }

// 8 x 8 bit transpose: byte t bit i <-> byte i bit t (lo = bytes 0..3).
BFP_FN void transpose8x8(uint32_t& lo, uint32_t& hi) {
  uint32_t t;
  t = (lo ^ (lo >> 7)) & 0x00AA00AAu;
  lo = lo ^ t ^ (t << 7);
  t = (hi ^ (hi >> 7)) & 0x00AA00AAu;
  hi = hi ^ t ^ (t << 7);
  t = (lo ^ (lo >> 14)) & 0x0000CCCCu;
  lo = lo ^ t ^ (t << 14);
  t = (hi ^ (hi >> 14)) & 0x0000CCCCu;
  hi = hi ^ t ^ (t << 14);
  t = (lo ^ (hi << 4)) & 0xF0F0F0F0u;
  lo ^= t;
  hi ^= t >> 4;
}

// in[8C] standard dwords -> pl[8C] plane words
template <int C>
BFP_FN void transpose_pack(const uint32_t* in, uint32_t* pl) {
  uint32_t lo[4][C], hi[4][C];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int b = 0; b < C; ++b) {
      uint32_t l = 0, h = 0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        l |= byte_at(in, (8 * r + t) * C + b) << (8 * t);
        h |= byte_at(in, (8 * r + 4 + t) * C + b) << (8 * t);
      }
      transpose8x8(l, h);
      lo[r][b] = l;
      hi[r][b] = h;
    }
  }
#pragma unroll
  for (int b = 0; b < C; ++b) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      uint32_t w = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t src = (i < 4) ? lo[r][b] : hi[r][b];
        w |= ((src >> (8 * (i & 3))) & 0xFFu) << (8 * r);
      }
      pl[8 * b + i] = w;
    }
  }
}

// pl[8C] plane words -> out[8C] standard dwords
template <int C>
BFP_FN void transpose_unpack(const uint32_t* pl, uint32_t* out) {
  uint32_t lo[4][C], hi[4][C];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int b = 0; b < C; ++b) {
      uint32_t l = 0, h = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        l |= ((pl[8 * b + i] >> (8 * r)) & 0xFFu) << (8 * i);
        h |= ((pl[8 * b + 4 + i] >> (8 * r)) & 0xFFu) << (8 * i);
      }
      transpose8x8(l, h);
      lo[r][b] = l;
      hi[r][b] = h;
    }
  }
#pragma unroll
  for (int w = 0; w < 8 * C; ++w) {
    uint32_t v = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = 4 * w + q;  // byte index in the standard data
      const int j = idx / C, b = idx % C;
      const int r = j >> 3, t = j & 7;
      const uint32_t src = (t < 4) ? lo[r][b] : hi[r][b];
      v |= ((src >> (8 * (t & 3))) & 0xFFu) << (8 * q);
    }
    out[w] = v;
  }
}

}  // namespace bfp
