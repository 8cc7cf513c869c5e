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
