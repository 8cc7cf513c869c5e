/* Native IEEE arithmetic on the host CPU, used to pin the oracle at the
 * formats that hardware implements: (8,23) = binary32 and (5,10) = binary16.
 * Test helper only.  Built with gcc -frounding-math, no fast-math, and with
 * the SSE flush-to-zero / denormals-are-zero bits cleared while it runs. */
#include <fenv.h>
#include <stdint.h>
#include <string.h>
#include <stddef.h>
#include <immintrin.h>

#pragma STDC FENV_ACCESS ON

static unsigned clear_ftz_daz(void) {
    unsigned old = _mm_getcsr();
    _mm_setcsr(old & ~((1u << 15) | (1u << 6)));
    return old;
}

/* op: 0 add, 1 sub, 2 mul, 3 div; mode: 0 nearest-even, 1 toward zero */
void f32_binop(int op, int mode, const uint32_t *a, const uint32_t *b, uint32_t *c, size_t n) {
    unsigned csr = clear_ftz_daz();
    int old = fegetround();
    fesetround(mode == 0 ? FE_TONEAREST : FE_TOWARDZERO);
    for (size_t i = 0; i < n; i++) {
        volatile float x, y, r;
        float tx, ty;
        memcpy(&tx, &a[i], 4);
        memcpy(&ty, &b[i], 4);
        x = tx;
        y = ty;
        if (op == 0) r = x + y;
        else if (op == 1) r = x - y;
        else if (op == 2) r = x * y;
        else r = x / y;
        float tr = r;
        memcpy(&c[i], &tr, 4);
    }
    fesetround(old);
    _mm_setcsr(csr);
}

/* binary16 toward zero: binary16 operands are exact in double, and a sum or
 * product of two of them is exact in double (at most 40 significant bits);
 * double -> float under FE_TOWARDZERO and float -> half with the F16C
 * truncating conversion round toward zero twice on nested grids, which equals
 * one rounding toward zero.  For division the double quotient is rounded
 * (to nearest), but a quotient p/q of binary16 values (q < 2^11 as an integer
 * significand) is either a float or at relative distance at least
 * 2^-24 / q > 2^-35 from every float, far more than the 2^-53 of that
 * rounding, so the rounded quotient stays on the exact quotient's side of
 * every float and half grid point. */
void f16_binop_rz(int op, const uint16_t *a, const uint16_t *b, uint16_t *c, size_t n) {
    unsigned csr = clear_ftz_daz();
    int old = fegetround();
    for (size_t i = 0; i < n; i++) {
        float fa = _cvtsh_ss(a[i]);
        float fb = _cvtsh_ss(b[i]);
        volatile double x = fa, y = fb, r;
        if (op == 0) r = x + y;
        else if (op == 1) r = x - y;
        else if (op == 2) r = x * y;
        else r = x / y;
        fesetround(FE_TOWARDZERO);
        volatile float rf = (float)r;
        fesetround(old);
        c[i] = _cvtss_sh(rf, _MM_FROUND_TO_ZERO | _MM_FROUND_NO_EXC);
    }
    _mm_setcsr(csr);
}

/* d = (a op1 b) op2 c in binary32, each op rounded (the intermediate is
 * stored to a volatile float, so no fused multiply-add can form). */
void f32_chain2(int op1, int op2, int mode, const uint32_t *a, const uint32_t *b, const uint32_t *c,
                uint32_t *d, size_t n) {
    unsigned csr = clear_ftz_daz();
    int old = fegetround();
    fesetround(mode == 0 ? FE_TONEAREST : FE_TOWARDZERO);
    for (size_t i = 0; i < n; i++) {
        volatile float x, y, z, t, r;
        float tx, ty, tz;
        memcpy(&tx, &a[i], 4);
        memcpy(&ty, &b[i], 4);
        memcpy(&tz, &c[i], 4);
        x = tx;
        y = ty;
        z = tz;
        if (op1 == 0) t = x + y;
        else if (op1 == 1) t = x - y;
        else t = x * y;
        if (op2 == 0) r = t + z;
        else if (op2 == 1) r = t - z;
        else r = t * z;
        float tr = r;
        memcpy(&d[i], &tr, 4);
    }
    fesetround(old);
    _mm_setcsr(csr);
}

/* Saturating and wrapping 8- and 16-bit integer arithmetic with SSE2/SSE4.1
 * instructions: add/sub by the saturating adds/subs instructions; products
 * formed exactly in a wider lane and narrowed by the saturating packs
 * (signed) or an unsigned minimum (unsigned).  op: 0 add, 1 sub, 2 mul;
 * kind: 1 unsigned saturation, 2 signed saturation.  Inputs and outputs are
 * held in uint32 arrays (low k bits). */
void int_sat_sse(int op, int k, int kind, const uint32_t *a, const uint32_t *b, uint32_t *c, size_t n) {
    for (size_t i = 0; i < n; i++) {
        uint32_t r = 0;
        if (k == 8) {
            __m128i x = _mm_cvtsi32_si128((int)(a[i] & 0xFF)), y = _mm_cvtsi32_si128((int)(b[i] & 0xFF)), z;
            if (op == 0) z = kind == 1 ? _mm_adds_epu8(x, y) : _mm_adds_epi8(x, y);
            else if (op == 1) z = kind == 1 ? _mm_subs_epu8(x, y) : _mm_subs_epi8(x, y);
            else if (kind == 1) {
                __m128i p = _mm_mullo_epi16(_mm_cvtepu8_epi16(x), _mm_cvtepu8_epi16(y));
                z = _mm_min_epu16(p, _mm_set1_epi16(0xFF));
            } else {
                __m128i p = _mm_mullo_epi16(_mm_cvtepi8_epi16(x), _mm_cvtepi8_epi16(y));
                z = _mm_packs_epi16(p, p);
            }
            r = (uint32_t)_mm_cvtsi128_si32(z) & 0xFF;
        } else {
            __m128i x = _mm_cvtsi32_si128((int)(a[i] & 0xFFFF)), y = _mm_cvtsi32_si128((int)(b[i] & 0xFFFF)), z;
            if (op == 0) z = kind == 1 ? _mm_adds_epu16(x, y) : _mm_adds_epi16(x, y);
            else if (op == 1) z = kind == 1 ? _mm_subs_epu16(x, y) : _mm_subs_epi16(x, y);
            else if (kind == 1) {
                __m128i p = _mm_mullo_epi32(_mm_cvtepu16_epi32(x), _mm_cvtepu16_epi32(y));
                z = _mm_min_epu32(p, _mm_set1_epi32(0xFFFF));
            } else {
                __m128i p = _mm_mullo_epi32(_mm_cvtepi16_epi32(x), _mm_cvtepi16_epi32(y));
                z = _mm_packs_epi32(p, p);
            }
            r = (uint32_t)_mm_cvtsi128_si32(z) & 0xFFFF;
        }
        c[i] = r;
    }
}

/* binary64 under fesetround (nearest-even or toward zero), FTZ/DAZ cleared.
 * op: 0 add, 1 sub, 2 mul, 3 div. */
void f64_binop(int op, int mode, const uint64_t *a, const uint64_t *b, uint64_t *c, size_t n) {
    unsigned csr = clear_ftz_daz();
    int old = fegetround();
    fesetround(mode == 0 ? FE_TONEAREST : FE_TOWARDZERO);
    for (size_t i = 0; i < n; i++) {
        volatile double x, y, r;
        double tx, ty;
        memcpy(&tx, &a[i], 8);
        memcpy(&ty, &b[i], 8);
        x = tx;
        y = ty;
        if (op == 0) r = x + y;
        else if (op == 1) r = x - y;
        else if (op == 2) r = x * y;
        else r = x / y;
        double tr = r;
        memcpy(&c[i], &tr, 8);
    }
    fesetround(old);
    _mm_setcsr(csr);
}
