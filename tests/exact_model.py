"""Independent exact model used to pin the oracle (test helper, not a test).

Written separately from ``oracle/bfp_oracle.c``: values are Python
``fractions.Fraction``/int, rounding is decided by searching the table of
representable values (or by comparing against the two neighbouring patterns),
never by computing an ulp exponent or a bit length.  It shares the number
model only: an IEEE-754-style reading of (1, e, m) with bias 2^(e-1)-1,
subnormals, infinities and NaN (the paper names IEEE binary16/binary32 as
its FP16/FP32 formats, Section 5.2).
"""
from __future__ import annotations

import bisect
from fractions import Fraction


class Fmt:
    def __init__(self, e: int, m: int):
        self.e, self.m = e, m
        self.B = 1 + e + m
        self.bias = 2 ** (e - 1) - 1
        self.sign_bit = 1 << (e + m)
        self.emax_field = 2 ** e - 1
        self.nan = (self.emax_field << m) | (1 << (m - 1))  # canonical NaN
        self.pinf = self.emax_field << m
        self.maxfin = ((self.emax_field - 1) << m) | ((1 << m) - 1)

    def fields(self, x):
        return (x >> (self.e + self.m)) & 1, (x >> self.m) & self.emax_field, x & ((1 << self.m) - 1)

    def is_nan(self, x):
        s, E, M = self.fields(x)
        return E == self.emax_field and M != 0

    def is_inf(self, x):
        s, E, M = self.fields(x)
        return E == self.emax_field and M == 0

    def value(self, x) -> Fraction:
        """Exact value of a finite pattern: textbook formula."""
        s, E, M = self.fields(x)
        assert E != self.emax_field
        if E == 0:
            mag = Fraction(M, 2 ** self.m) * Fraction(2) ** (1 - self.bias)
        else:
            mag = (1 + Fraction(M, 2 ** self.m)) * Fraction(2) ** (E - self.bias)
        return -mag if s else mag


class Table:
    """Sorted non-negative finite values of a format, for table-search rounding.

    Values are kept as integers scaled by 2**shift so comparisons are int
    comparisons.  A virtual entry 2^(emax+1) sits above the largest finite value:
    round-to-nearest that lands on it means overflow to infinity."""

    def __init__(self, f: Fmt, shift: int):
        self.f = f
        self.shift = shift
        pats = [p for p in range(0, f.pinf)]  # +0 .. +maxfinite, in magnitude order
        self.vals = [int(f.value(p) * 2 ** shift) for p in pats]
        assert all(self.vals[i] < self.vals[i + 1] for i in range(len(self.vals) - 1))
        self.pats = pats
        emax = f.emax_field - 1 - f.bias
        self.virtual = int(Fraction(2) ** (emax + 1) * 2 ** shift)

    def round_mag(self, X, mode: int) -> int:
        """Round a non-negative scaled exact magnitude (int or Fraction);
        returns a pattern (sign 0)."""
        f = self.f
        i = bisect.bisect_right(self.vals, X) - 1  # vals[i] <= X
        lo_v, lo_p = self.vals[i], self.pats[i]
        if lo_v == X:
            return lo_p
        if mode == 1:  # toward zero: largest entry <= X (never the virtual entry)
            return lo_p
        if i + 1 < len(self.vals):
            hi_v, hi_p = self.vals[i + 1], self.pats[i + 1]
        else:
            hi_v, hi_p = self.virtual, f.pinf
        d_lo, d_hi = X - lo_v, hi_v - X
        if d_lo < d_hi:
            return lo_p
        if d_hi < d_lo:
            return hi_p
        return lo_p if (lo_p & 1) == 0 else hi_p  # tie: even last bit (virtual Inf has M=0)


def ref_special(f: Fmt, op: str, a: int, b: int):
    """IEEE special-operand rules; returns a pattern, or None if a and b are finite."""
    if op == "sub":
        b ^= f.sign_bit
    if f.is_nan(a) or f.is_nan(b):
        return f.nan
    sa, sb = a >> (f.e + f.m) & 1, b >> (f.e + f.m) & 1
    ia, ib = f.is_inf(a), f.is_inf(b)
    if op in ("add", "sub"):
        if ia and ib:
            return a if sa == sb else f.nan
        if ia:
            return a
        if ib:
            return b
        return None
    za = (a & ~f.sign_bit) == 0
    zb = (b & ~f.sign_bit) == 0
    sgn = (sa ^ sb) << (f.e + f.m)
    if op == "div":
        if (ia and ib) or (za and zb):
            return f.nan
        if ia or zb:
            return f.pinf | sgn       # Inf / x, and x / 0 for finite nonzero x
        if ib or za:
            return sgn                # x / Inf, 0 / x: signed zero
        return None
    if ia or ib:
        if za or zb:
            return f.nan
        return f.pinf | sgn
    return None


def exact_result(f: Fmt, op: str, a: int, b: int):
    """Exact Fraction of a op b for finite operands, and the sign to give an exact zero."""
    if op == "sub":
        b ^= f.sign_bit
    va, vb = f.value(a), f.value(b)
    sa, sb = a >> (f.e + f.m) & 1, b >> (f.e + f.m) & 1
    if op in ("add", "sub"):
        x = va + vb
        zsign = sa if sa == sb else 0  # exact zero: +0 unless both addends are -0-signed
        return x, zsign
    if op == "div":
        return va / vb, sa ^ sb
    return va * vb, sa ^ sb


def table_round(f: Fmt, tab_add: Table, tab_mul: Table, op: str, mode: int, a: int, b: int) -> int:
    sp = ref_special(f, op, a, b)
    if sp is not None:
        return sp
    x, zsign = exact_result(f, op, a, b)
    tab = tab_mul if op == "mul" else tab_add
    if x == 0:
        return zsign << (f.e + f.m)
    X = abs(x) * 2 ** tab.shift
    if op != "div":
        assert X.denominator == 1
        X = int(X)
    p = tab.round_mag(X, mode)
    neg = x < 0
    return p | (f.sign_bit if neg else 0)


def tables(f: Fmt):
    qmin = 1 - f.bias - f.m
    return Table(f, -qmin), Table(f, -2 * qmin)


def check_correctly_rounded(f: Fmt, op: str, mode: int, a: int, b: int, r: int) -> str | None:
    """Neighbour test: r is the correctly rounded a op b iff no adjacent
    representable value is a better (or, at a tie, an even) answer.  Uses
    only the monotone order of non-negative patterns.  Returns an error text
    or None."""
    sp = ref_special(f, op, a, b)
    if sp is not None:
        return None if r == sp else "special: want %#x got %#x" % (sp, r)
    x, zsign = exact_result(f, op, a, b)
    if f.is_nan(r):
        return "NaN for finite operands"
    if x == 0:
        want = zsign << (f.e + f.m)
        return None if r == want else "exact zero: want %#x got %#x" % (want, r)
    neg = x < 0
    rs = r >> (f.e + f.m) & 1
    mag = r & ~f.sign_bit
    if rs != int(neg):
        return "sign"
    ax = abs(x)
    emax = f.emax_field - 1 - f.bias
    if f.is_inf(r):
        if mode == 1:
            return "RZ must not overflow to Inf"
        big = Fraction(2) ** emax * (2 - Fraction(1, 2 ** (f.m + 1)))  # max + half ulp
        return None if ax >= big else "Inf below overflow threshold"
    vr = f.value(mag)
    lower = f.value(mag - 1) if mag > 0 else None
    upper = f.value(mag + 1) if mag + 1 < f.pinf else Fraction(2) ** (emax + 1)
    if mode == 1:
        # RZ: vr <= |x| < next; above the largest finite value RZ stays there
        if mag == f.maxfin:
            return None if vr <= ax else "RZ bracket fails"
        if not (vr <= ax < upper):
            return "RZ bracket fails"
        return None
    # RNE
    if ax == vr:
        return None
    if ax > vr:
        d_me, d_other = ax - vr, upper - ax
        if upper <= ax:
            return "RNE: above next"
    else:
        if lower is None or lower >= ax:
            return "RNE: below previous"
        d_me, d_other = vr - ax, ax - lower
    if d_me > d_other:
        return "RNE: not nearest"
    if d_me == d_other and (mag & 1):
        return "RNE: tie not even"
    if mag == f.maxfin and ax >= Fraction(2) ** emax * (2 - Fraction(1, 2 ** (f.m + 1))):
        return "RNE: should overflow"
    return None


def edge_patterns(f: Fmt):
    """Interesting positive patterns; callers add signs."""
    m = f.m
    one = f.bias << m
    pts = {0, 1, 2, 3, (1 << m) - 1, (1 << m) - 2, 1 << m, (1 << m) + 1,
           one, one + 1, one - 1, one + (1 << (m - 1)), f.maxfin, f.maxfin - 1,
           f.pinf, f.nan, f.pinf | 1, (2 << m), (2 << m) | ((1 << m) - 1)}
    for E in (2, f.bias - 1, f.bias + 1, f.emax_field - 2, f.emax_field // 2):
        if 0 < E < f.emax_field:
            pts.add(E << m)
            pts.add((E << m) | ((1 << m) - 1))
            pts.add((E << m) | 1)
    return sorted(p for p in pts if 0 <= p <= f.pinf | ((1 << m) - 1))


def sweep_formats():
    return [(e, m) for e in (3, 4, 5, 6, 8) for m in (1, 2, 3, 5, 7, 10, 15, 23)]


def wide_formats():
    """Formats wider than the sweep: exponents up to 11 bits, patterns up to
    64 bits (8-byte containers above 32 bits); (11,52) is binary64."""
    return [(8, 31), (11, 20), (11, 40), (11, 52)]
