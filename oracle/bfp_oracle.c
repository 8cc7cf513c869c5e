/*
 * bfp_oracle.c -- reference arithmetic for custom-precision floating point
 * (1 sign bit, e exponent bits, m mantissa bits) and for the standard <->
 * bitslice layout transforms.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the oracle: the tests, the smoke
 * check and the CPU-baseline leg of the benchmark call it; the GPU library
 * never does, and it shares no code with the GPU library.
 *
 * Method (plain definition, no circuit): decode each operand to an exact
 * (sign, integer significand, power-of-two exponent), form the exact sum or
 * product with wide unsigned integers, and round once.  The paper fixes the
 * two rounding modes (Section 4: round toward zero, and round to nearest with
 * ties to even) and the three arithmetic operations (Section 4, Table 1:
 * add/sub, mul, div).  Everything the paper leaves open
 * (bias, subnormals, infinities and NaN, overflow, the sign of an exact zero,
 * NaN output bits) follows IEEE 754-2008 binary interchange semantics
 * generalised to (e, m); each such reading is listed in the design notes.
 *
 * Patterns are held in 64-bit words (1 + e + m <= 64, e <= 11, m <= 52).
 * Wide integers: an exact sum needs at most 2^e - 3 + m + 2 <= 2100 bits
 * (e <= 11, m <= 52), so a fixed 2304-bit unsigned integer (36 64-bit limbs,
 * least significant first) is enough; products need at most 106 bits and
 * the scaled quotient at most 164.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define ORACLE_RNE 0
#define ORACLE_RZ 1
#define ORACLE_ADD 0
#define ORACLE_SUB 1
#define ORACLE_MUL 2
#define ORACLE_DIV 3

/* ------------------------------------------------------------------------ */
/* 2304-bit unsigned integers                                                */
/* ------------------------------------------------------------------------ */
#define NLIMB 36
/* Limbs [0, n) hold the value; limbs at and above n are zero by definition
 * and are never read (limb() supplies the zeros), so small formats touch
 * only the few limbs their values need. */
typedef struct { int n; uint64_t w[NLIMB]; } big;

static uint64_t limb(const big *a, int i) { return i < a->n ? a->w[i] : 0; }
static int imax(int a, int b) { return a > b ? a : b; }
static int imin(int a, int b) { return a < b ? a : b; }

static big big_from_u64(uint64_t v) {
    big r;
    r.n = 1;
    r.w[0] = v;
    return r;
}

static big big_from_u128(unsigned __int128 v) {
    big r;
    r.n = 2;
    r.w[0] = (uint64_t)v;
    r.w[1] = (uint64_t)(v >> 64);
    return r;
}

static int big_cmp(const big *a, const big *b) {
    for (int i = imax(a->n, b->n) - 1; i >= 0; i--) {
        uint64_t x = limb(a, i), y = limb(b, i);
        if (x > y) return 1;
        if (x < y) return -1;
    }
    return 0;
}

/* a << s; the operands used here never overflow 2304 bits. */
static big big_shl(const big *a, int s) {
    big r;
    int lw = s / 64, bit = s % 64;
    r.n = imin(NLIMB, a->n + lw + 1);
    for (int i = 0; i < r.n; i++) {
        int src = i - lw;
        uint64_t v = src >= 0 ? limb(a, src) << bit : 0;
        if (bit && src - 1 >= 0) v |= limb(a, src - 1) >> (64 - bit);
        r.w[i] = v;
    }
    return r;
}

/* a >> s */
static big big_shr(const big *a, int s) {
    big r;
    int lw = s / 64, bit = s % 64;
    r.n = imax(1, a->n - lw);
    for (int i = 0; i < r.n; i++) {
        int src = i + lw;
        uint64_t v = limb(a, src) >> bit;
        if (bit) v |= limb(a, src + 1) << (64 - bit);
        r.w[i] = v;
    }
    return r;
}

static big big_add(const big *a, const big *b) {
    big r;
    uint64_t carry = 0;
    r.n = imin(NLIMB, imax(a->n, b->n) + 1);
    for (int i = 0; i < r.n; i++) {
        uint64_t x = limb(a, i), y = limb(b, i);
        uint64_t s = x + y;
        uint64_t c1 = s < x;
        uint64_t t = s + carry;
        uint64_t c2 = t < s;
        r.w[i] = t;
        carry = c1 | c2;
    }
    return r;
}

/* a - b, requires a >= b */
static big big_sub(const big *a, const big *b) {
    big r;
    uint64_t borrow = 0;
    r.n = imax(a->n, b->n);
    for (int i = 0; i < r.n; i++) {
        uint64_t x = limb(a, i), y = limb(b, i);
        uint64_t d = x - y;
        uint64_t b1 = x < y;
        uint64_t t = d - borrow;
        uint64_t b2 = d < borrow;
        r.w[i] = t;
        borrow = b1 | b2;
    }
    return r;
}

/* x / d in place (d > 0, one limb: schoolbook division digit by digit, each
 * step dividing a 128-bit partial remainder); returns the remainder. */
static uint64_t big_divmod_u64(big *x, uint64_t d) {
    unsigned __int128 rem = 0;
    for (int i = x->n - 1; i >= 0; i--) {
        unsigned __int128 cur = (rem << 64) | x->w[i];
        x->w[i] = (uint64_t)(cur / d);
        rem = cur % d;
    }
    return (uint64_t)rem;
}

/* number of significant bits; 0 for zero */
static int big_bitlen(const big *a) {
    for (int i = a->n - 1; i >= 0; i--) {
        if (a->w[i]) {
            int n = 64;
            while (!((a->w[i] >> (n - 1)) & 1)) n--;
            return i * 64 + n;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Number model                                                              */
/* ------------------------------------------------------------------------ */
enum { CLS_ZERO, CLS_FINITE, CLS_INF, CLS_NAN };

typedef struct {
    int s;         /* sign bit */
    uint64_t sig;  /* integer significand */
    int q;         /* value = (-1)^s * sig * 2^q */
    int cls;
} decoded;

static int bias_of(int e) { return (1 << (e - 1)) - 1; }

/* Field layout of a pattern x (low 1+e+m bits): mantissa in bits [0,m),
 * exponent in bits [m,m+e), sign in bit m+e. */
static decoded decode(uint64_t x, int e, int m) {
    decoded d;
    uint64_t M = x & ((1ull << m) - 1u);
    uint64_t E = (x >> m) & ((1ull << e) - 1u);
    d.s = (int)((x >> (e + m)) & 1u);
    d.sig = 0;
    d.q = 0;
    if (E == (1ull << e) - 1u) {
        d.cls = M ? CLS_NAN : CLS_INF;
    } else if (E == 0) {
        d.sig = M;
        d.q = 1 - bias_of(e) - m;
        d.cls = M ? CLS_FINITE : CLS_ZERO;
    } else {
        d.sig = (1ull << m) + M;
        d.q = (int)E - bias_of(e) - m;
        d.cls = CLS_FINITE;
    }
    return d;
}

static uint64_t encode(int s, uint64_t E, uint64_t M, int e, int m) {
    return ((uint64_t)s << (e + m)) | (E << m) | M;
}

static uint64_t canonical_nan(int e, int m) {
    return encode(0, (1ull << e) - 1u, 1ull << (m - 1), e, m);
}

static uint64_t infinity(int s, int e, int m) {
    return encode(s, (1ull << e) - 1u, 0, e, m);
}

/* Round (-1)^s * S * 2^q0 (S > 0) once to the format. */
static uint64_t round_exact(int s, const big *S, int q0, int e, int m, int mode) {
    int bias = bias_of(e);
    int L = big_bitlen(S);
    /* ulp exponent of the result: normal ulp, clamped at the subnormal ulp */
    int top = q0 + L - 1;
    int qt = (top > 1 - bias ? top : 1 - bias) - m;
    uint64_t sig;
    if (qt <= q0) {
        big t = big_shl(S, q0 - qt); /* exact, fits in m+1 bits */
        sig = limb(&t, 0);
    } else {
        int sh = qt - q0;
        big t = big_shr(S, sh);
        sig = limb(&t, 0);
        big back = big_shl(&t, sh);
        big rem = big_sub(S, &back);
        big one = big_from_u64(1);
        big half = big_shl(&one, sh - 1);
        if (mode == ORACLE_RNE) {
            int c = big_cmp(&rem, &half);
            if (c > 0 || (c == 0 && (sig & 1u))) sig += 1;
        }
    }
    if (sig == (1ull << (m + 1))) { /* rounding carried into a new bit */
        sig >>= 1;
        qt += 1;
    }
    uint64_t E, M;
    if (sig < (1ull << m)) { /* subnormal (or zero), qt is the subnormal ulp */
        E = 0;
        M = sig;
    } else {
        long Ev = (long)qt + m + bias;
        if (Ev >= (1L << e) - 1) { /* overflow */
            if (mode == ORACLE_RNE) return infinity(s, e, m);
            return encode(s, (1ull << e) - 2u, (1ull << m) - 1u, e, m);
        }
        E = (uint64_t)Ev;
        M = sig - (1ull << m);
    }
    return encode(s, E, M, e, m);
}

/* ------------------------------------------------------------------------ */
/* Operations                                                                */
/* ------------------------------------------------------------------------ */
static uint64_t op_add(uint64_t a, uint64_t b, int e, int m, int mode) {
    decoded x = decode(a, e, m), y = decode(b, e, m);
    if (x.cls == CLS_NAN || y.cls == CLS_NAN) return canonical_nan(e, m);
    if (x.cls == CLS_INF && y.cls == CLS_INF)
        return x.s == y.s ? infinity(x.s, e, m) : canonical_nan(e, m);
    if (x.cls == CLS_INF) return infinity(x.s, e, m);
    if (y.cls == CLS_INF) return infinity(y.s, e, m);
    if (x.cls == CLS_ZERO && y.cls == CLS_ZERO)
        return encode(x.s == y.s ? x.s : 0, 0, 0, e, m);
    int q0 = x.q < y.q ? x.q : y.q;
    big A0 = big_from_u64(x.sig), B0 = big_from_u64(y.sig);
    big A = big_shl(&A0, x.q - q0);
    big B = big_shl(&B0, y.q - q0);
    big S;
    int s;
    if (x.s == y.s) {
        S = big_add(&A, &B);
        s = x.s;
    } else {
        int c = big_cmp(&A, &B);
        if (c == 0) return encode(0, 0, 0, e, m); /* exact cancellation: +0 */
        if (c > 0) {
            S = big_sub(&A, &B);
            s = x.s;
        } else {
            S = big_sub(&B, &A);
            s = y.s;
        }
    }
    return round_exact(s, &S, q0, e, m, mode);
}

static uint64_t op_mul(uint64_t a, uint64_t b, int e, int m, int mode) {
    decoded x = decode(a, e, m), y = decode(b, e, m);
    int s = x.s ^ y.s;
    if (x.cls == CLS_NAN || y.cls == CLS_NAN) return canonical_nan(e, m);
    if (x.cls == CLS_INF || y.cls == CLS_INF) {
        if (x.cls == CLS_ZERO || y.cls == CLS_ZERO) return canonical_nan(e, m);
        return infinity(s, e, m);
    }
    if (x.cls == CLS_ZERO || y.cls == CLS_ZERO) return encode(s, 0, 0, e, m);
    big S = big_from_u128((unsigned __int128)x.sig * y.sig); /* < 2^106 */
    return round_exact(s, &S, x.q + y.q, e, m, mode);
}

/* a / b.  The exact quotient sig_a / sig_b is represented for rounding as
 * S = 2 * floor(sig_a * 2^k / sig_b) + [remainder != 0] at exponent
 * qa - qb - k - 1: with k chosen so the integer quotient has at least m + 3
 * bits, no rounding boundary of the format lies strictly between the exact
 * quotient and S * 2^(qa-qb-k-1) (both lie in the same open interval between
 * consecutive multiples of 2^(qa-qb-k), and every boundary is a multiple of
 * that unit), so rounding S rounds the exact quotient. */
static uint64_t op_div(uint64_t a, uint64_t b, int e, int m, int mode) {
    decoded x = decode(a, e, m), y = decode(b, e, m);
    int s = x.s ^ y.s; /* sign of the quotient */
    if (x.cls == CLS_NAN || y.cls == CLS_NAN) return canonical_nan(e, m);
    if (x.cls == CLS_INF && y.cls == CLS_INF) return canonical_nan(e, m);
    if (x.cls == CLS_ZERO && y.cls == CLS_ZERO) return canonical_nan(e, m);
    if (x.cls == CLS_INF) return infinity(s, e, m);
    if (y.cls == CLS_INF) return encode(s, 0, 0, e, m);
    if (y.cls == CLS_ZERO) return infinity(s, e, m); /* finite nonzero / 0 */
    if (x.cls == CLS_ZERO) return encode(s, 0, 0, e, m);
    const int k = 2 * m + 6; /* sig_a * 2^k / sig_b >= 2^k / 2^(m+1) = 2^(m+5) */
    big A0 = big_from_u64(x.sig);
    big S = big_shl(&A0, k); /* < 2^(3m+7) <= 2^163 */
    const uint64_t rem = big_divmod_u64(&S, y.sig);
    S = big_shl(&S, 1);
    S.w[0] |= (rem != 0);
    return round_exact(s, &S, x.q - y.q - k - 1, e, m, mode);
}

static int format_ok(int e, int m) { return e >= 2 && e <= 11 && m >= 1 && m <= 52 && 1 + e + m <= 64; }

/* One element.  op: 0 add, 1 sub, 2 mul, 3 div.  mode: 0 RNE, 1 RZ.
 * Returns the result pattern, or all ones (never a result: NaN results have
 * sign 0) for an invalid argument.  Bits above 1+e+m of a and b are ignored. */
uint64_t oracle_op1_64(int op, int e, int m, int mode, uint64_t a, uint64_t b) {
    if (!format_ok(e, m) || (mode != ORACLE_RNE && mode != ORACLE_RZ)) return ~0ull;
    const int B = 1 + e + m;
    const uint64_t mask = B == 64 ? ~0ull : ((1ull << B) - 1u);
    a &= mask;
    b &= mask;
    switch (op) {
    case ORACLE_ADD: return op_add(a, b, e, m, mode);
    case ORACLE_SUB: return op_add(a, b ^ (1ull << (e + m)), e, m, mode); /* a + (-b) */
    case ORACLE_MUL: return op_mul(a, b, e, m, mode);
    case ORACLE_DIV: return op_div(a, b, e, m, mode);
    default: return ~0ull;
    }
}

/* The same for formats of at most 32 bits; 0xFFFFFFFF for an invalid argument. */
uint32_t oracle_op1(int op, int e, int m, int mode, uint32_t a, uint32_t b) {
    if (!format_ok(e, m) || 1 + e + m > 32) return 0xFFFFFFFFu;
    const uint64_t r = oracle_op1_64(op, e, m, mode, a, b);
    return r == ~0ull ? 0xFFFFFFFFu : (uint32_t)r;
}

/* Round a binary64 value once to the format (used to build expected values
 * for pins, never by the GPU path); all ones for an invalid format. */
uint64_t oracle_from_double(int e, int m, int mode, double v) {
    if (!format_ok(e, m)) return ~0ull;
    uint64_t bits;
    memcpy(&bits, &v, sizeof bits);
    int s = (int)(bits >> 63);
    int E = (int)((bits >> 52) & 0x7FF);
    uint64_t F = bits & ((1ull << 52) - 1);
    if (E == 0x7FF) return F ? canonical_nan(e, m) : infinity(s, e, m);
    if (E == 0 && F == 0) return encode(s, 0, 0, e, m);
    uint64_t sig = E ? (F | (1ull << 52)) : F;
    int q = (E ? E : 1) - 1023 - 52;
    big S = big_from_u64(sig);
    return round_exact(s, &S, q, e, m, mode);
}

/* ------------------------------------------------------------------------ */
/* Vector driver with optional threads                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int op, e, m, mode;
    const uint64_t *a, *b;
    uint64_t *c;
    uint64_t lo, hi;
} job;

static void *run_job(void *p) {
    job *j = (job *)p;
    for (uint64_t i = j->lo; i < j->hi; i++)
        j->c[i] = oracle_op1_64(j->op, j->e, j->m, j->mode, j->a[i], j->b[i]);
    return NULL;
}

/* Elementwise c[i] = a[i] op b[i] on patterns held in uint64 words.
 * Returns 0, or -1 for an invalid argument. */
int oracle_binop64(int op, int e, int m, int mode, const uint64_t *a, const uint64_t *b,
                   uint64_t *c, uint64_t n, int nthreads) {
    if (!format_ok(e, m) || op < 0 || op > 3 || (mode != 0 && mode != 1)) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((uint64_t)nthreads > n) nthreads = n ? (int)n : 1;
    job jobs[256];
    pthread_t tids[256];
    uint64_t chunk = (n + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; t++) {
        uint64_t lo = chunk * t, hi = lo + chunk;
        if (lo > n) lo = n;
        if (hi > n) hi = n;
        jobs[t] = (job){op, e, m, mode, a, b, c, lo, hi};
    }
    if (nthreads == 1) {
        run_job(&jobs[0]);
        return 0;
    }
    for (int t = 0; t < nthreads; t++) pthread_create(&tids[t], NULL, run_job, &jobs[t]);
    for (int t = 0; t < nthreads; t++) pthread_join(tids[t], NULL);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Layout transforms (Section 2, Figure 1; Section 4 helper transforms)       */
/* ------------------------------------------------------------------------ */
/* Bitslice layout: plane k (0 <= k < B) holds bit k of every element's
 * standard pattern; element i sits in word i / 32 of the plane at bit
 * i % 32.  Planes are gpad 32-bit words apart. */
static uint64_t load_container(const void *x, int cbytes, uint64_t i) {
    if (cbytes == 1) return ((const uint8_t *)x)[i];
    if (cbytes == 2) return ((const uint16_t *)x)[i];
    if (cbytes == 4) return ((const uint32_t *)x)[i];
    return ((const uint64_t *)x)[i];
}

static void store_container(void *x, int cbytes, uint64_t i, uint64_t v) {
    if (cbytes == 1) ((uint8_t *)x)[i] = (uint8_t)v;
    else if (cbytes == 2) ((uint16_t *)x)[i] = (uint16_t)v;
    else if (cbytes == 4) ((uint32_t *)x)[i] = (uint32_t)v;
    else ((uint64_t *)x)[i] = v;
}

static int layout_ok(int B, int cbytes) {
    return B >= 1 && B <= 64 && B <= 8 * cbytes && (cbytes == 1 || cbytes == 2 || cbytes == 4 || cbytes == 8);
}

int oracle_pack(int B, int cbytes, const void *x, uint32_t *planes, uint64_t n, uint64_t gpad) {
    if (!layout_ok(B, cbytes) || gpad * 32 < n) return -1;
    memset(planes, 0, (size_t)B * gpad * sizeof(uint32_t));
    for (uint64_t i = 0; i < n; i++) {
        uint64_t v = load_container(x, cbytes, i);
        for (int k = 0; k < B; k++)
            if ((v >> k) & 1u) planes[(uint64_t)k * gpad + i / 32] |= 1u << (i % 32);
    }
    return 0;
}

int oracle_unpack(int B, int cbytes, const uint32_t *planes, void *x, uint64_t n, uint64_t gpad) {
    if (!layout_ok(B, cbytes) || gpad * 32 < n) return -1;
    for (uint64_t i = 0; i < n; i++) {
        uint64_t v = 0;
        for (int k = 0; k < B; k++)
            if ((planes[(uint64_t)k * gpad + i / 32] >> (i % 32)) & 1u) v |= 1ull << k;
        store_container(x, cbytes, i, v);
    }
    return 0;
}

/* ---- bitslice integer vectors (Section 3, Figure 2; Section 6) ------------
 * An element is a k-bit pattern, 1 <= k <= 32, read as an unsigned value
 * (the pattern) or a signed one (two's complement).  The exact sum,
 * difference or product of the two values is formed in 128-bit integers and
 * mapped to k bits by the kind:
 *   0 wrap: the exact result modulo 2^k (what the ripple adder of Figure 2
 *     gives when its last carry is dropped; the same bits whether the
 *     operands are read signed or unsigned);
 *   1 unsigned saturation: operands unsigned, result clamped to [0, 2^k - 1];
 *   2 signed saturation: operands signed, result clamped to
 *     [-2^(k-1), 2^(k-1) - 1].
 * Bits of a and b above bit k-1 are ignored. */
static __int128 int_value(uint32_t x, int k, int is_signed) {
    uint64_t p = (uint64_t)x & ((1ull << k) - 1);
    if (is_signed && (p >> (k - 1)) & 1) return (__int128)p - ((__int128)1 << k);
    return (__int128)p;
}

static uint32_t int_op(int op, int k, int kind, uint32_t a, uint32_t b) {
    const int is_signed = kind == 2;
    const __int128 x = int_value(a, k, is_signed), y = int_value(b, k, is_signed);
    __int128 v = op == ORACLE_ADD ? x + y : (op == ORACLE_SUB ? x - y : x * y);
    if (kind == 1) {
        const __int128 hi = ((__int128)1 << k) - 1;
        if (v < 0) v = 0;
        if (v > hi) v = hi;
    } else if (kind == 2) {
        const __int128 lo = -((__int128)1 << (k - 1)), hi = ((__int128)1 << (k - 1)) - 1;
        if (v < lo) v = lo;
        if (v > hi) v = hi;
    }
    const __int128 mod = (__int128)1 << k;
    __int128 r = v % mod;
    if (r < 0) r += mod;
    return (uint32_t)r;
}

/* c[i] = a[i] op b[i] for k-bit integers.  op: 0 add, 1 sub, 2 mul; kind as
 * above.  Returns 0, or -1 for an invalid argument. */
int oracle_int_binop(int op, int k, int kind, const uint32_t *a, const uint32_t *b, uint32_t *c, uint64_t n) {
    if (k < 1 || k > 32 || op < 0 || op > 2 || kind < 0 || kind > 2) return -1;
    for (uint64_t i = 0; i < n; i++) c[i] = int_op(op, k, kind, a[i], b[i]);
    return 0;
}
