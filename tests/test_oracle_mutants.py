"""The pins must catch plausible mistakes in the oracle.

Each mutant is a copy of ``oracle/bfp_oracle.c`` with one planted mistake
(a dropped term, a wrong sign, an off-by-one, a wrong tie rule ...), built in
a temporary directory.  The planted copy must disagree with the exact model
(exhaustive on small formats) or with the hand-derived golden cases.  The
committed oracle itself is never modified."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from tests.exact_model import Fmt, check_correctly_rounded, table_round, tables

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "bfp_oracle.c")

MUTANTS = [
    ("tie ignores evenness", "(c == 0 && (sig & 1u))", "(c == 0)"),
    ("rounds up on any remainder", "if (c > 0 || (c == 0 && (sig & 1u))) sig += 1;",
     "if (c >= 0 || (c == 0 && (sig & 1u))) sig += 1;"),
    ("cancellation keeps sign", "return encode(0, 0, 0, e, m); /* exact", "return encode(x.s, 0, 0, e, m); /* exact"),
    ("overflow threshold off by one", "if (Ev >= (1L << e) - 1)", "if (Ev > (1L << e) - 1)"),
    ("no subnormal clamp", "int qt = (top > 1 - bias ? top : 1 - bias) - m;", "int qt = top - m;"),
    ("subnormal exponent off by one", "d.q = 1 - bias_of(e) - m;", "d.q = 0 - bias_of(e) - m;"),
    ("RZ overflow gives Inf", "if (mode == ORACLE_RNE) return infinity(s, e, m);", "return infinity(s, e, m);"),
    ("carry renormalisation dropped", "sig >>= 1;\n        qt += 1;", "qt += 0;"),
    ("mul sign not xor", "int s = x.s ^ y.s;\n", "int s = x.s;\n"),
    ("sub does not negate", "return op_add(a, b ^ (1ull << (e + m)), e, m, mode);", "return op_add(a, b, e, m, mode);"),
    ("inf*0 not NaN", "if (x.cls == CLS_ZERO || y.cls == CLS_ZERO) return canonical_nan(e, m);", ""),
    ("wrong bias", "static int bias_of(int e) { return (1 << (e - 1)) - 1; }",
     "static int bias_of(int e) { return (1 << (e - 1)); }"),
    ("borrow dropped in sub", "borrow = b1 | b2;", "borrow = b1;"),
    ("min exponent alignment", "int q0 = x.q < y.q ? x.q : y.q;", "int q0 = x.q > y.q ? y.q : y.q + 1;"),
    ("div sticky dropped", "S.w[0] |= (rem != 0);", ""),
    ("div exponent off by one", "x.q - y.q - k - 1, e, m, mode", "x.q - y.q - k, e, m, mode"),
    ("div sign not xor", "int s = x.s ^ y.s; /* sign of the quotient */", "int s = x.s;"),
    ("x/0 gives NaN", "if (y.cls == CLS_ZERO) return infinity(s, e, m);",
     "if (y.cls == CLS_ZERO) return canonical_nan(e, m);"),
    ("0/0 not NaN", "if (x.cls == CLS_ZERO && y.cls == CLS_ZERO) return canonical_nan(e, m);", ""),
    ("x/Inf gives Inf", "if (y.cls == CLS_INF) return encode(s, 0, 0, e, m);",
     "if (y.cls == CLS_INF) return infinity(s, e, m);"),
    ("div guard bits too few", "const int k = 2 * m + 6;", "const int k = 1;"),
    ("wide integers too narrow for binary64 alignment", "#define NLIMB 36", "#define NLIMB 6"),
    ("binary64 product truncated to 64 bits", "big S = big_from_u128((unsigned __int128)x.sig * y.sig);",
     "big S = big_from_u64(x.sig * y.sig);"),
]


def _build(tmp_path, src_text, name):
    c = tmp_path / (name + ".c")
    c.write_text(src_text)
    so = tmp_path / (name + ".so")
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-pthread", "-w", str(c), "-o", str(so)])
    L = ctypes.CDLL(str(so))
    L.oracle_binop64.restype = ctypes.c_int
    L.oracle_binop64.argtypes = [ctypes.c_int] * 4 + [ctypes.c_void_p] * 3 + [ctypes.c_uint64, ctypes.c_int]
    return L


def _wide_gap_pairs():
    """(8,23) pairs whose exact sums span several 64-bit limbs: a power of two
    (or a value just above one) minus a value 60..200 binades smaller."""
    rng = np.random.default_rng(3)
    ea = rng.integers(200, 254, 64)
    gap = rng.integers(60, 200, 64)
    a = (ea << 23) | rng.integers(0, 2, 64)
    b = (1 << 31) | ((ea - gap) << 23) | rng.integers(1, 1 << 23, 64)
    return a.astype(np.uint32), b.astype(np.uint32)


def _run(L, op, e, m, mode, a, b, nthreads=1):
    a64 = np.ascontiguousarray(np.asarray(a, dtype=np.uint64))
    b64 = np.ascontiguousarray(np.asarray(b, dtype=np.uint64))
    c = np.empty_like(a64)
    L.oracle_binop64(op, e, m, mode, a64.ctypes.data, b64.ctypes.data, c.ctypes.data, a64.size, nthreads)
    return c


def _small_dividend_quotients_disagree(L):
    """binary16 subnormal / lowest-binade quotients against numpy's float16
    division (round to nearest even): the fewest bits below the rounding point."""
    a = np.repeat(np.arange(1, 1024, dtype=np.uint32), 1024)
    b = np.tile(np.arange(1024, 2048, dtype=np.uint32), 1023)
    c = _run(L, 3, 5, 10, 0, a, b, 8)
    ha, hb = a.astype(np.uint16).view(np.float16), b.astype(np.uint16).view(np.float16)
    return not np.array_equal(c, (ha / hb).view(np.uint16).astype(np.uint64))


def _binary64_wide_gaps_disagree(L):
    """binary64 sums and differences across exponent gaps of up to ~2000
    binades (exact sums up to ~2100 bits wide), and products and quotients,
    against numpy's float64 (round to nearest even)."""
    rng = np.random.default_rng(8)
    n = 4000
    ea = rng.integers(1000, 2046, n).astype(np.uint64)
    eb = np.maximum(ea.astype(np.int64) - rng.integers(0, 2000, n), 0).astype(np.uint64)
    a = (ea << np.uint64(52)) | rng.integers(0, 1 << 52, n, dtype=np.uint64)
    b = (eb << np.uint64(52)) | rng.integers(0, 1 << 52, n, dtype=np.uint64)
    b[::2] |= np.uint64(1 << 63)
    fa, fb = a.view(np.float64), b.view(np.float64)
    with np.errstate(all="ignore"):
        for op, r in ((0, fa + fb), (2, fa * fb), (3, fa / fb)):
            if not np.array_equal(_run(L, op, 11, 52, 0, a, b, 8), r.view(np.uint64)):
                return True
    return False


def _disagrees(L):
    if _small_dividend_quotients_disagree(L) or _binary64_wide_gaps_disagree(L):
        return True
    f = Fmt(8, 23)
    a, b = _wide_gap_pairs()
    for mode in (0, 1):
        c = _run(L, 0, 8, 23, mode, a, b)
        for i in range(a.size):
            if check_correctly_rounded(f, "add", mode, int(a[i]), int(b[i]), int(c[i])) is not None:
                return True
    for (e, m) in [(5, 2), (4, 3), (3, 1)]:
        f = Fmt(e, m)
        ta, tm = tables(f)
        n = 1 << f.B
        a = np.repeat(np.arange(n, dtype=np.uint32), n)
        b = np.tile(np.arange(n, dtype=np.uint32), n)
        for opi, op in enumerate(("add", "sub", "mul", "div")):
            for mode in (0, 1):
                c = _run(L, opi, e, m, mode, a, b)
                for i in range(0, a.size, 5):
                    if int(c[i]) != table_round(f, ta, tm, op, mode, int(a[i]), int(b[i])):
                        return True
    return False


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, "mutation site not found: " + name
    L = _build(tmp_path, text.replace(old, new), "mutant")
    assert _disagrees(L), "planted mistake survived the pins: " + name


def test_unmutated_copy_agrees(tmp_path):
    """The same harness finds no disagreement for the committed oracle."""
    L = _build(tmp_path, open(SRC).read(), "clean")
    assert not _disagrees(L)


INT_MUTANTS = [
    ("signed read as unsigned", "if (is_signed && (p >> (k - 1)) & 1)", "if (0 && (p >> (k - 1)) & 1)"),
    ("unsigned floor not clamped", "if (v < 0) v = 0;", ""),
    ("signed max off by one", "hi = ((__int128)1 << (k - 1)) - 1;", "hi = ((__int128)1 << (k - 1));"),
    ("signed min off by one", "const __int128 lo = -((__int128)1 << (k - 1)),", "const __int128 lo = 1 - ((__int128)1 << (k - 1)),"),
    ("negative remainder not lifted", "if (r < 0) r += mod;", ""),
    ("sub as add", "(op == ORACLE_SUB ? x - y : x * y)", "(op == ORACLE_SUB ? x + y : x * y)"),
    ("unsigned ceiling off by one", "const __int128 hi = ((__int128)1 << k) - 1;", "const __int128 hi = ((__int128)1 << k) - 2;"),
]


def _int_disagrees(L):
    from tests.test_oracle_int import _table_search
    L.oracle_int_binop.restype = ctypes.c_int
    L.oracle_int_binop.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p] * 3 + [ctypes.c_uint64]
    for k in (1, 3, 4):
        n = 1 << k
        a = np.repeat(np.arange(n, dtype=np.uint32), n)
        b = np.tile(np.arange(n, dtype=np.uint32), n)
        c = np.empty_like(a)
        for opi, op in enumerate(("add", "sub", "mul")):
            for kd, kind in enumerate(("wrap", "satu", "sats")):
                L.oracle_int_binop(opi, k, kd, a.ctypes.data, b.ctypes.data, c.ctypes.data, a.size)
                for i in range(a.size):
                    if int(c[i]) != _table_search(k, kind, op, int(a[i]), int(b[i])):
                        return True
    return False


@pytest.mark.parametrize("name,old,new", INT_MUTANTS, ids=[m[0] for m in INT_MUTANTS])
def test_int_mutant_is_caught(tmp_path, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, "mutation site not found: " + name
    L = _build(tmp_path, text.replace(old, new), "mutant")
    assert _int_disagrees(L), "planted mistake survived the pins: " + name


def test_int_unmutated_copy_agrees(tmp_path):
    L = _build(tmp_path, open(SRC).read(), "clean")
    assert not _int_disagrees(L)
