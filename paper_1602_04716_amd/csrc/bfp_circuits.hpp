// bfp_circuits.hpp -- software circuits for bitslice custom-precision FP.
//
// Every function here is a straight-line netlist of word-wide gates: one
// gate processes one bit of every element held in the word (Section 3,
// Figure 2).  The floating-point operations follow the step lists of
// Table 1 (Section 4):
//   add/sub: sign, alignment shift, add, normalise, round
//   mul:     sign, exponent add, significand multiply, normalise, round
//   div:     sign, exponent subtract, significand divide, normalise, round
// with a logarithmic (barrel) shifter for alignment and normalisation
// (Section 4) and gate count, not depth, as the cost to minimise, which is
// also the cost on a SIMT machine where every lane runs every gate.
//
// Number model (the paper names IEEE binary16/binary32 as its FP16/FP32;
// everything else it leaves open is read the IEEE way): bias 2^(e-1)-1,
// exponent field 0 = zero/subnormal, all ones = Inf (mantissa 0) or NaN;
// results correctly rounded to nearest-even or toward zero; overflow gives
// Inf (nearest) or the largest finite value (toward zero); an exact zero sum
// of opposite-signed operands is +0; NaN results are the canonical quiet NaN
// (sign 0, exponent all ones, mantissa 2^(m-1)).
//
// Plane layout of an operand x[0 .. 1+e+m): x[k] for k < m is mantissa bit
// k, x[m + j] exponent bit j, x[m + e] the sign.
#pragma once
#include "bfp_word.hpp"

namespace bfp {

constexpr int ceil_log2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int cmin(int a, int b) { return a < b ? a : b; }

// ---------------------------------------------------------------------------
// Gates
// ---------------------------------------------------------------------------
template <class W> BFP_FN W g_and(W a, W b) { return a & b; }
template <class W> BFP_FN W g_or(W a, W b) { return a | b; }
template <class W> BFP_FN W g_xor(W a, W b) { return a ^ b; }
template <class W> BFP_FN W g_not(W a) { return ~a; }
template <class W> BFP_FN W g_andn(W a, W b) { return bitop3<imm8(TA & ~TB)>(a, b, b); }  // a & ~b
template <class W> BFP_FN W g_orn(W a, W b) { return bitop3<imm8(TA | ~TB)>(a, b, b); }   // a | ~b
template <class W> BFP_FN W g_xnor(W a, W b) { return bitop3<imm8(~(TA ^ TB))>(a, b, b); } // ~(a ^ b)
template <class W> BFP_FN W g_or3(W a, W b, W c) { return bitop3<IMM_OR3>(a, b, c); }
template <class W> BFP_FN W g_and3(W a, W b, W c) { return bitop3<IMM_AND3>(a, b, c); }
template <class W> BFP_FN W g_xor3(W a, W b, W c) { return bitop3<IMM_XOR3>(a, b, c); }
template <class W> BFP_FN W g_maj(W a, W b, W c) { return bitop3<IMM_MAJ>(a, b, c); }
template <class W> BFP_FN W g_mux(W s, W a, W b) { return bitop3<IMM_MUX>(s, a, b); }  // s ? a : b
template <unsigned IMM, class W> BFP_FN W g3(W a, W b, W c) { return bitop3<IMM>(a, b, c); }

// OR / AND / NOR over x[LO, HI) (HI > LO), with 3-input gates.
template <int LO, int HI, class W>
BFP_FN W or_range(const W* x) {
  static_assert(HI > LO, "empty range");
  W r = x[LO];
  int i = LO + 1;
#pragma unroll
  for (; i + 1 < HI; i += 2) r = g_or3(r, x[i], x[i + 1]);
  if (i < HI) r = g_or(r, x[i]);
  return r;
}
template <int LO, int HI, class W>
BFP_FN W and_range(const W* x) {
  static_assert(HI > LO, "empty range");
  W r = x[LO];
  int i = LO + 1;
#pragma unroll
  for (; i + 1 < HI; i += 2) r = g_and3(r, x[i], x[i + 1]);
  if (i < HI) r = g_and(r, x[i]);
  return r;
}

// OR over x[lo, hi) with bounds that are constants once loops are unrolled.
template <class W>
BFP_FN W or_span(const W* x, int lo, int hi) {
  W r = x[lo];
  int i = lo + 1;
#pragma unroll
  for (; i + 1 < hi; i += 2) r = g_or3(r, x[i], x[i + 1]);
  if (i < hi) r = g_or(r, x[i]);
  return r;
}

// ---------------------------------------------------------------------------
// Figure 2: bitslice ripple-carry adder of two N-bit unsigned vectors,
// result modulo 2^N.  Sum and carry of each full adder are one 3-input gate
// each (xor3, majority).
// ---------------------------------------------------------------------------
template <int N, class W>
BFP_FN void ripple_add(const W* a, const W* b, W* r) {
  W c = g_and(a[0], b[0]);
  r[0] = g_xor(a[0], b[0]);
#pragma unroll
  for (int i = 1; i < N; ++i) {
    r[i] = g_xor3(a[i], b[i], c);
    if (i + 1 < N) c = g_maj(a[i], b[i], c);
  }
}

// r[0 .. N] = a + b (N + 1 bits)
template <int N, class W>
BFP_FN void ripple_add_full(const W* a, const W* b, W* r) {
  W c = g_and(a[0], b[0]);
  r[0] = g_xor(a[0], b[0]);
#pragma unroll
  for (int i = 1; i < N; ++i) {
    r[i] = g_xor3(a[i], b[i], c);
    c = g_maj(a[i], b[i], c);
  }
  r[N] = c;
}

// r = x + cin (N bits, carry out dropped)
template <int N, class W>
BFP_FN void increment(W* x, W cin) {
  W c = cin;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    W t = g_xor(x[i], c);
    if (i + 1 < N) c = g_and(x[i], c);
    x[i] = t;
  }
}

// Logarithmic right shift of v[0, NV) by the amount whose bits are amt[0, NB),
// with sticky: bits shifted to position 0 or below are ORed into v[0].
// Positions 1 .. NV-1 hold data; v[0] is the sticky bit.  A shift by 2^LF or
// more (any amount bit >= LF) moves every data bit into the sticky bit.
template <int NV, int NB, class W>
BFP_FN void shift_right_sticky(W* v, const W* amt) {
  constexpr int LF = ceil_log2(NV - 1);  // 2^LF >= NV - 1: such a shift empties every position
  if constexpr (NB > LF) {
    W hi = (NB - LF == 1) ? amt[LF] : or_range<LF, NB>(amt);
    W any = or_range<1, NV>(v);
    v[0] = g3<imm8((TA & TB) | TC)>(hi, any, v[0]);
#pragma unroll
    for (int i = 1; i < NV; ++i) v[i] = g_andn(v[i], hi);
  }
  constexpr int NS = cmin(NB, LF);
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const int s = 1 << j;
    const W sel = amt[j];
    // bits at positions 1 .. s land at or below 0
    W lost = v[1];
#pragma unroll
    for (int i = 2; i <= s && i < NV; ++i) lost = g_or(lost, v[i]);
    v[0] = g3<imm8((TA & TB) | TC)>(sel, lost, v[0]);
#pragma unroll
    for (int i = 1; i < NV; ++i) v[i] = (i + s < NV) ? g_mux(sel, v[i + s], v[i]) : g_andn(v[i], sel);
  }
}

// x > 2^j for an N-bit unsigned x (j < N)
template <int N, class W>
BFP_FN W gt_pow2(const W* x, int j) {
  const bool above = j + 1 < N, below = j > 0;
  if (!below) return above ? or_span(x, j + 1, N) : WordTraits<W>::zero();
  const W lo = or_span(x, 0, j);
  if (!above) return g_and(x[j], lo);
  return g3<imm8(TA | (TB & TC))>(or_span(x, j + 1, N), x[j], lo);
}

// ---------------------------------------------------------------------------
// Table 1, Add/Sub.  c = a + (b with its sign XORed with negb): negb is all
// ones for subtraction and zero for addition.
// ---------------------------------------------------------------------------
template <int E, int M, bool RZ, class W>
BFP_FN void fp_add(const W* a, const W* b, W negb, W* out) {
  constexpr int F = E + M;   // magnitude field: exponent | mantissa
  constexpr int P = M + 1;   // significand bits with the hidden bit
  constexpr int NA = P + 3;  // aligned: 0 sticky, 1 round, 2 guard, 3.. significand
  const W zero = WordTraits<W>::zero();

  // step 1 (sign): order the operands by magnitude; |a| < |b| is the borrow
  // out of the unsigned subtraction of the E|M fields
  const W sa = a[F];
  const W sb = g_xor(b[F], negb);
  W lt = g_andn(b[0], a[0]);
#pragma unroll
  for (int i = 1; i < F; ++i) lt = g3<IMM_MAJ_NA>(a[i], b[i], lt);
  W big[F], sml[F];
#pragma unroll
  for (int i = 0; i < F; ++i) {
    big[i] = g_mux(lt, b[i], a[i]);
    sml[i] = g_mux(lt, a[i], b[i]);
  }
  const W s_big = g_mux(lt, sb, sa);
  const W eff_sub = g_xor(sa, sb);

  // classification
  const W* Eb = big + M;
  const W* Es = sml + M;
  const W hid_b = or_range<0, E>(Eb);  // exponent nonzero: hidden bit
  const W hid_s = or_range<0, E>(Es);
  const W emax_b = and_range<0, E>(Eb);
  const W emax_s = and_range<0, E>(Es);
  const W mnz_b = or_range<0, M>(big);

  // effective exponents (a subnormal's is 1) and d = E'big - E'small >= 0
  W eb[E], es[E];
  eb[0] = g_orn(Eb[0], hid_b);
  es[0] = g_orn(Es[0], hid_s);
#pragma unroll
  for (int i = 1; i < E; ++i) {
    eb[i] = Eb[i];
    es[i] = Es[i];
  }
  W d[E];
  {
    d[0] = g_xor(eb[0], es[0]);
    W c = g_orn(eb[0], es[0]);  // eb + ~es + 1
#pragma unroll
    for (int i = 1; i < E; ++i) {
      d[i] = g3<IMM_XNOR3>(eb[i], es[i], c);
      if (i + 1 < E) c = g3<IMM_MAJ_NB>(eb[i], es[i], c);
    }
  }

  // step 2 (alignment shift): small significand right by d, with sticky
  W q[NA];
  q[0] = zero;
  q[1] = zero;
  q[2] = zero;
#pragma unroll
  for (int k = 0; k < M; ++k) q[3 + k] = sml[k];
  q[3 + M] = hid_s;
  shift_right_sticky<NA, E>(q, d);

  // step 3 (add): r = 8*big_sig + q, or 8*big_sig - q.  With t the carry
  // (add) or borrow (sub): sum = x ^ q ^ t, t' = maj(x ^ eff_sub, q, t).
  W r[NA + 1];
  W t;
  r[0] = q[0];
  t = g_and(eff_sub, q[0]);
  r[1] = g_xor(q[1], t);
  t = g_maj(eff_sub, q[1], t);
  r[2] = g_xor(q[2], t);
  t = g_maj(eff_sub, q[2], t);
#pragma unroll
  for (int i = 3; i < NA; ++i) {
    const W x = (i - 3 < M) ? big[i - 3] : hid_b;
    r[i] = g_xor3(x, q[i], t);
    t = g_maj(g_xor(x, eff_sub), q[i], t);
  }
  r[NA] = t;  // carry out of a magnitude addition; 0 after a subtraction

  // step 4 (normalise): carry out -> right shift by one, exponent + 1
  const W cout = r[NA];
  W n[NA];
  n[0] = g3<imm8((TA & TB) | TC)>(cout, r[1], r[0]);
#pragma unroll
  for (int i = 1; i < NA; ++i) n[i] = g_mux(cout, r[i + 1], r[i]);
  W ex[E];
#pragma unroll
  for (int i = 0; i < E; ++i) ex[i] = eb[i];
  increment<E>(ex, cout);
  const W ovf = and_range<0, E>(ex);  // only E'big = 2^e - 2 with a carry out gets here

  // cancellation -> left shift by min(leading zeros, ex - 1), greedily by
  // descending powers of two; the clamp yields subnormal results directly
  {
    constexpr int LN = ceil_log2(NA);
#pragma unroll
    for (int j = LN - 1; j >= 0; --j) {
      const int s = 1 << j;
      if (s >= (1 << E) - 2) continue;  // ex - 1 <= 2^e - 3 never allows this shift
      W z = n[NA - 1];
#pragma unroll
      for (int i = NA - 2; i >= NA - s; --i) z = g_or(z, n[i]);
      const W cond = g_andn(gt_pow2<E>(ex, j), z);  // ex > 2^j and top s bits zero
#pragma unroll
      for (int i = NA - 1; i >= s; --i) n[i] = g_mux(cond, n[i - s], n[i]);
#pragma unroll
      for (int i = 0; i < s; ++i) n[i] = g_andn(n[i], cond);
      // ex -= cond * 2^j
      W bw = cond;
#pragma unroll
      for (int i = j; i < E; ++i) {
        W nb = g_xor(ex[i], bw);
        if (i + 1 < E) bw = g_andn(bw, ex[i]);
        ex[i] = nb;
      }
    }
  }

  // step 5 (round): result field X = (exponent if normal else 0) | mantissa;
  // nearest-even adds 1 at the mantissa LSB, and a carry out of the mantissa
  // moves into the exponent, so max-finite + ulp becomes Inf by itself
  const W hid = n[NA - 1];
  W x[F];
#pragma unroll
  for (int k = 0; k < M; ++k) x[k] = n[3 + k];
#pragma unroll
  for (int i = 0; i < E; ++i) x[M + i] = g_and(ex[i], hid);
  if constexpr (!RZ) {
    const W up = g3<IMM_AND_OR>(n[2], g_or(n[3], n[1]), n[0]);  // g & (lsb | r | s)
    increment<F>(x, up);
#pragma unroll
    for (int i = 0; i < E; ++i) x[M + i] = g_or(x[M + i], ovf);
#pragma unroll
    for (int k = 0; k < M; ++k) x[k] = g_andn(x[k], ovf);
  } else {
    x[M] = g_andn(x[M], ovf);  // largest finite: exponent 2^e - 2, mantissa all ones
#pragma unroll
    for (int k = 0; k < M; ++k) x[k] = g_or(x[k], ovf);
  }

  // specials and the sign of zero
  const W nan_o = g_and(emax_b, g3<imm8(TA | (TB & TC))>(mnz_b, emax_s, eff_sub));
  const W sp = emax_b;  // Inf or NaN out
  const W nz = or_range<0, F>(x);
  // sign: NaN -> 0; exact cancellation (eff_sub, zero result) -> 0
  const W kill = g3<imm8(TA | (TB & ~TC))>(nan_o, eff_sub, g_or(nz, sp));
  out[F] = g_andn(s_big, kill);
#pragma unroll
  for (int i = 0; i < E; ++i) out[M + i] = g_or(x[M + i], sp);
#pragma unroll
  for (int k = 0; k < M - 1; ++k) out[k] = g_andn(x[k], sp);
  out[M - 1] = g3<IMM_ANDN_OR>(x[M - 1], sp, nan_o);
}

// ---------------------------------------------------------------------------
// Shared by Mul and Div
// ---------------------------------------------------------------------------

// Two's complement width holding every value in [lo, hi] and also -lo (the
// underflow shift amount).
constexpr int exp_width(int lo, int hi) {
  int w = 2;
  while (!(-(1 << (w - 1)) <= lo && hi < (1 << (w - 1)) && -lo < (1 << (w - 1)))) ++w;
  return w;
}

// x[0, N) -= y[0, NY) (y zero-extended), modulo 2^N: x + ~y + 1.
template <int N, int NY, class W>
BFP_FN void sub_zext(W* x, const W* y) {
  W c = WordTraits<W>::zero();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const W xi = x[i];
    if (i == 0) {  // carry-in 1: sum = x ^ y, carry = x | ~y
      x[0] = g_xor(xi, y[0]);
      c = g_orn(xi, y[0]);
    } else if (i < NY) {
      x[i] = g3<IMM_XNOR3>(xi, y[i], c);
      if (i + 1 < N) c = g3<IMM_MAJ_NB>(xi, y[i], c);
    } else {  // ~y = 1 above its width: x + 1 + c
      x[i] = g_xnor(xi, c);
      if (i + 1 < N) c = g_or(xi, c);
    }
  }
}

// x[0, N) += y[0, NY) (y zero-extended), modulo 2^N.
template <int N, int NY, class W>
BFP_FN void add_zext(W* x, const W* y) {
  W c = WordTraits<W>::zero();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const W xi = x[i];
    if (i == 0) {
      x[0] = g_xor(xi, y[0]);
      c = g_and(xi, y[0]);
    } else if (i < NY) {
      x[i] = g_xor3(xi, y[i], c);
      if (i + 1 < N) c = g_maj(xi, y[i], c);
    } else {
      x[i] = g_xor(xi, c);
      if (i + 1 < N) c = g_and(xi, c);
    }
  }
}

// x[0, N) += K (a constant), modulo 2^N: a constant addend folds to at most
// one gate per bit for the sum and one for the carry.
template <int N, class W>
BFP_FN void add_const(W* x, unsigned K) {
  W c = WordTraits<W>::zero();
  bool c_is_zero = true;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const bool k = (K >> i) & 1u;
    const W xi = x[i];
    if (c_is_zero) {
      if (k) {  // x + 1, carry-in 0
        x[i] = g_not(xi);
        c = xi;
        c_is_zero = false;
      }
    } else if (k) {  // x + 1 + c: sum = ~(x ^ c), carry = x | c
      x[i] = g_xnor(xi, c);
      c = g_or(xi, c);
    } else {         // x + 0 + c
      x[i] = g_xor(xi, c);
      c = g_and(xi, c);
    }
  }
}

// Pre-normalise the P = M + 1 bit significand of x (hidden bit hid): shift it
// left by its leading-zero count, found greedily by descending powers of two;
// lz[0, LP) receives the count.  A normal significand is left unchanged.
template <int M, int LP, class W>
BFP_FN void prenormalise(const W* x, W hid, W* S, W* lz) {
  constexpr int P = M + 1;
#pragma unroll
  for (int k = 0; k < M; ++k) S[k] = x[k];
  S[M] = hid;
#pragma unroll
  for (int j = LP - 1; j >= 0; --j) {
    const int sh = 1 << j;
    W z = S[P - 1];
#pragma unroll
    for (int i = P - 2; i >= P - sh; --i) z = g_or(z, S[i]);
    z = g_not(z);
#pragma unroll
    for (int i = P - 1; i >= sh; --i) S[i] = g_mux(z, S[i - sh], S[i]);
#pragma unroll
    for (int i = 0; i < sh; ++i) S[i] = g_andn(S[i], z);
    lz[j] = z;
  }
}

// Normalised significand v[0, M + 3) (0 sticky, 1 guard, 2 .. M+2 the
// significand, hidden bit on top) and D = E_f - 1 in EW two's complement bits
// -> rounded result.  Underflow (E_f <= 0, i.e. D < 0) shifts right by -D with
// sticky and gives exponent field 0; overflow is E_f >= 2^e - 1.  Then the
// special results: sp forces the all-ones exponent (Inf, or NaN when nan_o),
// zero_o a signed zero.
template <int E, int M, bool RZ, int EW, class W>
BFP_FN void finish_muldiv(W* v, W* D, W s, W nan_o, W sp, W zero_o, W* out) {
  constexpr int F = E + M, P = M + 1, NV = P + 2;
  const W zero = WordTraits<W>::zero();
  const W neg = D[EW - 1];
  W sh[EW];
  {
    // -D = ~D + 1, masked to zero unless D < 0
#pragma unroll
    for (int i = 0; i < EW; ++i) sh[i] = g_not(D[i]);
    increment<EW>(sh, WordTraits<W>::ones());
#pragma unroll
    for (int i = 0; i < EW; ++i) sh[i] = g_and(sh[i], neg);
  }
  shift_right_sticky<NV, EW - 1>(v, sh);
  W ovf;
  {
    W hi_bits = (EW - 1 > E) ? or_range<E, cmax(EW - 1, E + 1)>(D) : zero;
    W top = (E >= 2) ? and_range<1, cmax(E, 2)>(D) : D[0];
    ovf = g3<imm8((TA | TB) & ~TC)>(hi_bits, top, neg);
  }

  // step 5 (round): X = (D + hidden) << m | mantissa, then + round-up; the
  // hidden bit carries D + 1 = E_f into the field for normal results, and D
  // is masked to 0 for subnormal ones
  W x[F];
#pragma unroll
  for (int k = 0; k < M; ++k) x[k] = v[2 + k];
#pragma unroll
  for (int i = 0; i < E; ++i) x[M + i] = g_andn(D[i], neg);
  {
    W c = v[P + 1];  // hidden bit
#pragma unroll
    for (int i = 0; i < E; ++i) {
      W t = g_xor(x[M + i], c);
      if (i + 1 < E) c = g_and(x[M + i], c);
      x[M + i] = t;
    }
  }
  if constexpr (!RZ) {
    const W up = g3<IMM_AND_OR>(v[1], v[2], v[0]);  // g & (lsb | s)
    increment<F>(x, up);
#pragma unroll
    for (int i = 0; i < E; ++i) x[M + i] = g_or(x[M + i], ovf);
#pragma unroll
    for (int k = 0; k < M; ++k) x[k] = g_andn(x[k], ovf);
  } else {
#pragma unroll
    for (int i = 1; i < E; ++i) x[M + i] = g_or(x[M + i], ovf);
    x[M] = g_andn(x[M], ovf);
#pragma unroll
    for (int k = 0; k < M; ++k) x[k] = g_or(x[k], ovf);
  }

  // zero operands, then specials
  out[F] = g_andn(s, nan_o);
#pragma unroll
  for (int i = 0; i < E; ++i) out[M + i] = g3<IMM_ANDN_OR>(x[M + i], zero_o, sp);
#pragma unroll
  for (int k = 0; k < M - 1; ++k) out[k] = g3<imm8(TA & ~(TB | TC))>(x[k], zero_o, sp);
  out[M - 1] = g3<imm8((TA & ~TB) | TC)>(g_andn(x[M - 1], zero_o), sp, nan_o);
}

// ---------------------------------------------------------------------------
// Table 1, Mul.
// ---------------------------------------------------------------------------
template <int E, int M>
struct MulWidths {
  static constexpr int P = M + 1;
  static constexpr int LP = ceil_log2(P);  // pre-normalisation stages (2^LP >= P)
  static constexpr int BIAS = (1 << (E - 1)) - 1;
  // E_f - 1 = E'a + E'b - lza - lzb - bias + cout - 1 spans
  // [2 - 2(P-1) - bias - 1, 2(2^E - 2) - bias]
  static constexpr int LO = 2 - 2 * (P - 1) - BIAS - 1;
  static constexpr int HI = 2 * ((1 << E) - 2) - BIAS;
  static constexpr int EW = cmax(exp_width(LO, HI), E + 2);  // signed width of the exponent datapath
};

template <int E, int M, bool RZ, class W>
BFP_FN void fp_mul(const W* a, const W* b, W* out) {
  using MW = MulWidths<E, M>;
  constexpr int F = E + M, P = MW::P, LP = MW::LP, EW = MW::EW;
  constexpr int NV = P + 2;  // 0 sticky, 1 guard, 2.. significand
  const W zero = WordTraits<W>::zero();

  // step 1 (sign)
  const W s = g_xor(a[F], b[F]);

  // classification and special results
  const W hid_a = or_range<M, F>(a), hid_b = or_range<M, F>(b);
  const W emax_a = and_range<M, F>(a), emax_b = and_range<M, F>(b);
  const W mnz_a = or_range<0, M>(a), mnz_b = or_range<0, M>(b);
  const W nz_a = g_or(hid_a, mnz_a), nz_b = g_or(hid_b, mnz_b);
  // NaN: a NaN operand, or Inf * 0
  const W nan_o = g_or(g3<imm8(TA & (TB | ~TC))>(emax_a, mnz_a, nz_b),
                       g3<imm8(TA & (TB | ~TC))>(emax_b, mnz_b, nz_a));
  const W sp = g_or(emax_a, emax_b);
  const W zero_o = g_not(g_and(nz_a, nz_b));

  // pre-normalise subnormal significands
  W A[P], Bs[P], lza[LP], lzb[LP];
  prenormalise<M, LP>(a, hid_a, A, lza);
  prenormalise<M, LP>(b, hid_b, Bs, lzb);

  // step 2 (exponent add), merged into one datapath of EW signed bits:
  // D = E'a + E'b + (-bias - 1) - (lza + lzb), and + cout after the multiply
  W D[EW];
  {
    W ea[E], eb[E];
    ea[0] = g_orn(a[M], hid_a);
    eb[0] = g_orn(b[M], hid_b);
#pragma unroll
    for (int i = 1; i < E; ++i) {
      ea[i] = a[M + i];
      eb[i] = b[M + i];
    }
    // E'a + E'b (E + 1 bits)
#pragma unroll
    for (int i = 0; i < EW; ++i) D[i] = zero;
    {
      W c = g_and(ea[0], eb[0]);
      D[0] = g_xor(ea[0], eb[0]);
#pragma unroll
      for (int i = 1; i < E; ++i) {
        D[i] = g_xor3(ea[i], eb[i], c);
        c = g_maj(ea[i], eb[i], c);
      }
      D[E] = c;
    }
    // + (-bias - 1) mod 2^EW
    add_const<EW>(D, (unsigned)(-(MW::BIAS + 1)) & ((1u << EW) - 1u));
    // - (lza + lzb) = + ~(lza + lzb) + 1
    W lz[LP + 1];
    if constexpr (LP == 1) {
      lz[0] = g_xor(lza[0], lzb[0]);
      lz[1] = g_and(lza[0], lzb[0]);
    } else {
      ripple_add_full<LP, W>(lza, lzb, lz);
    }
    {
      W c = WordTraits<W>::ones();  // carry-in 1 of the negation
      bool c_is_one = true;
#pragma unroll
      for (int i = 0; i < EW; ++i) {
        if (i <= LP) {
          const W x = D[i], y = lz[i];
          if (c_is_one) {  // x + ~y + 1: sum = x ^ y, carry = x | ~y
            D[i] = g_xor(x, y);
            c = g_orn(x, y);
            c_is_one = false;
          } else {
            D[i] = g3<IMM_XNOR3>(x, y, c);
            c = g3<IMM_MAJ_NB>(x, y, c);
          }
        } else {  // ~y = 1 above the lz width: x + 1 + c
          const W x = D[i];
          D[i] = g_xnor(x, c);
          c = g_or(x, c);
        }
      }
    }
  }

  // step 3 (significand multiply): rows of an array multiplier, least
  // significant multiplier bit first.  After row j the low bit of the
  // accumulator is product bit j-1 and retires: bits 0 .. P-3 only feed the
  // sticky bit, bit P-2 is kept; the accumulator stays P+1 bits wide.
  W acc[P + 1];
#pragma unroll
  for (int i = 0; i < P; ++i) acc[i] = g_and(A[i], Bs[0]);
  acc[P] = zero;
  W sticky = zero;
  W pbit = zero;  // product bit P-2
#pragma unroll
  for (int j = 1; j < P; ++j) {
    const W retired = acc[0];
    if (j - 1 <= P - 3) sticky = (j == 1) ? retired : g_or(sticky, retired);
    else pbit = retired;
    const W bj = Bs[j];
    W c = zero;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const W x = acc[i + 1];
      const W pp = g_and(A[i], bj);
      if (i == 0) {
        acc[0] = g_xor(x, pp);
        c = g_and(x, pp);
      } else if (j == 1 && i == P - 1) {  // acc[P] is still zero in the first row
        acc[i] = g_xor(pp, c);
        c = g_and(pp, c);
      } else {
        acc[i] = g_xor3(x, pp, c);
        c = g_maj(x, pp, c);
      }
    }
    acc[P] = c;
  }
  if constexpr (P == 1) pbit = zero;
  // product bits P-1 .. 2P-1 are acc[0 .. P]; product in [2^(2P-2), 2^(2P))

  // step 4 (normalise): a product >= 2 shifts right by one, exponent + 1
  const W cout = acc[P];
  W v[NV];
  v[0] = g3<imm8(TA | (TB & TC))>(sticky, cout, pbit);
  v[1] = g_mux(cout, acc[0], pbit);
#pragma unroll
  for (int i = 2; i < NV; ++i) v[i] = g_mux(cout, acc[i - 1], acc[i - 2]);
  increment<EW>(D, cout);  // D = E_f - 1
  finish_muldiv<E, M, RZ, EW, W>(v, D, s, nan_o, sp, zero_o, out);
}

// ---------------------------------------------------------------------------
// Table 1, Div.
// ---------------------------------------------------------------------------
template <int E, int M>
struct DivWidths {
  static constexpr int P = M + 1;
  static constexpr int LP = ceil_log2(P);
  static constexpr int BIAS = (1 << (E - 1)) - 1;
  // E_f - 1 = E'a - lza - E'b + lzb + bias - 2 + q0 spans
  // [2 - 2^E - P + bias, 2^E + P + bias - 5]
  static constexpr int LO = 2 - (1 << E) - P + BIAS;
  static constexpr int HI = (1 << E) + P + BIAS - 5;
  static constexpr int EW = cmax(exp_width(LO, HI), E + 2);
};

// c = a / b.  After pre-normalisation both significands A', B' lie in
// [2^(P-1), 2^P), so the quotient A'/B' lies in (1/2, 2).  Restoring division
// produces its bits q_0, q_-1, ..., q_-(P+1), one per step (compare the
// doubled partial remainder with B', subtract when not below), and the final
// remainder's OR is the sticky bit; a quotient below 1 (q_0 = 0) shifts left
// by one and lowers the exponent.
template <int E, int M, bool RZ, class W>
BFP_FN void fp_div(const W* a, const W* b, W* out) {
  using DW = DivWidths<E, M>;
  constexpr int F = E + M, P = DW::P, LP = DW::LP, EW = DW::EW;
  constexpr int NV = P + 2;  // 0 sticky, 1 guard, 2.. significand
  const W zero = WordTraits<W>::zero();

  // step 1 (sign)
  const W s = g_xor(a[F], b[F]);

  // classification and special results
  const W hid_a = or_range<M, F>(a), hid_b = or_range<M, F>(b);
  const W emax_a = and_range<M, F>(a), emax_b = and_range<M, F>(b);
  const W mnz_a = or_range<0, M>(a), mnz_b = or_range<0, M>(b);
  const W nz_a = g_or(hid_a, mnz_a), nz_b = g_or(hid_b, mnz_b);
  const W inf_a = g_andn(emax_a, mnz_a), inf_b = g_andn(emax_b, mnz_b);
  // NaN: a NaN operand, 0/0 or Inf/Inf
  const W nan_o = g_or(g_or3(g_and(emax_a, mnz_a), g_and(emax_b, mnz_b), g_and(inf_a, inf_b)),
                       g3<imm8(~(TA | TB))>(nz_a, nz_b, nz_b));
  // Inf: Inf / finite, or nonzero / 0; zero: 0 / nonzero, or finite / Inf
  const W inf_o = g3<imm8((TA | ~TB) & ~TC)>(inf_a, nz_b, nan_o);
  const W zero_o = g3<imm8((~TA | TB) & ~TC)>(nz_a, inf_b, nan_o);
  const W sp = g_or(nan_o, inf_o);

  // pre-normalise subnormal significands
  W A[P], Bs[P], lza[LP], lzb[LP];
  prenormalise<M, LP>(a, hid_a, A, lza);
  prenormalise<M, LP>(b, hid_b, Bs, lzb);

  // step 2 (exponent subtract): D = E'a - E'b + lzb - lza + bias - 2, then + q_0
  W D[EW];
  {
    W eb[E];
    D[0] = g_orn(a[M], hid_a);  // E' = max(E, 1)
    eb[0] = g_orn(b[M], hid_b);
#pragma unroll
    for (int i = 1; i < E; ++i) {
      D[i] = a[M + i];
      eb[i] = b[M + i];
    }
#pragma unroll
    for (int i = E; i < EW; ++i) D[i] = zero;
    sub_zext<EW, E>(D, eb);
    add_zext<EW, LP>(D, lzb);
    sub_zext<EW, LP>(D, lza);
    add_const<EW>(D, (unsigned)(DW::BIAS - 2) & ((1u << EW) - 1u));
  }

  // step 3 (significand divide).  Q[t] is quotient bit q_-t.  R holds the
  // partial remainder, always below B' < 2^P.
  W Q[P + 2], R[P];
  W nq0;  // ~q_0
  {
    // q_0: A' - B'; the borrow out is A' < B'
    W d[P];
    W bw = g_andn(Bs[0], A[0]);
    d[0] = g_xor(A[0], Bs[0]);
#pragma unroll
    for (int i = 1; i < P; ++i) {
      d[i] = g_xor3(A[i], Bs[i], bw);
      bw = g3<IMM_MAJ_NA>(A[i], Bs[i], bw);
    }
    nq0 = bw;
    Q[0] = g_not(bw);
#pragma unroll
    for (int i = 0; i < P; ++i) R[i] = g_mux(bw, A[i], d[i]);
  }
#pragma unroll
  for (int t = 1; t <= P + 1; ++t) {
    // 2R (P + 1 bits, low bit 0) - B': bit 0 of the difference is B'[0] with
    // borrow B'[0]; the top bit of 2R is R[P-1] against a zero bit of B'
    W d[P];
    W bw = Bs[0];
    d[0] = Bs[0];
#pragma unroll
    for (int i = 1; i < P; ++i) {
      d[i] = g_xor3(R[i - 1], Bs[i], bw);
      bw = g3<IMM_MAJ_NA>(R[i - 1], Bs[i], bw);
    }
    const W q = g_orn(R[P - 1], bw);  // 2R >= B'
    Q[t] = q;
    W Rn[P];
    Rn[0] = g_and(q, d[0]);
#pragma unroll
    for (int i = 1; i < P; ++i) Rn[i] = g_mux(q, d[i], R[i - 1]);
#pragma unroll
    for (int i = 0; i < P; ++i) R[i] = Rn[i];
  }
  const W rem = or_range<0, P>(R);

  // step 4 (normalise): q_0 = 1 keeps q_0 .. q_-(P-1), guard q_-P and sticky
  // q_-(P+1) | rem; q_0 = 0 takes q_-1 .. q_-P, guard q_-(P+1), sticky rem
  W v[NV];
  v[0] = g3<imm8(TA | (~TB & TC))>(rem, nq0, Q[P + 1]);
#pragma unroll
  for (int i = 1; i < NV; ++i) v[i] = g_mux(nq0, Q[P + 2 - i], Q[P + 1 - i]);
  increment<EW>(D, Q[0]);  // D = E_f - 1

  finish_muldiv<E, M, RZ, EW, W>(v, D, s, nan_o, sp, zero_o, out);
}

}  // namespace bfp
