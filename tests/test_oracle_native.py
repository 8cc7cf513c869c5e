"""Pin the oracle against native IEEE arithmetic on the host (no GPU).

(8,23) is binary32, (5,10) binary16 and (8,7) bfloat16 under the IEEE-style
reading of the format.  NaN results are compared for NaN-ness only (x86 and
numpy propagate payloads and signs; the oracle returns its canonical NaN).
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def native():
    flags = open("/proc/cpuinfo").read()
    if " f16c" not in flags:
        pytest.skip("host CPU lacks F16C")
    so = os.path.join(HERE, "_native_pins.so")
    src = os.path.join(HERE, "native_pins.c")
    if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O1", "-frounding-math", "-fno-fast-math", "-mf16c",
                               "-msse4.1", "-fPIC", "-shared", src, "-o", so + ".tmp"])
        os.replace(so + ".tmp", so)
    L = ctypes.CDLL(so)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    L.f32_binop.argtypes = [i32, i32, vp, vp, vp, sz]
    L.f16_binop_rz.argtypes = [i32, vp, vp, vp, sz]
    L.f32_chain2.argtypes = [i32, i32, i32, vp, vp, vp, vp, sz]
    L.f64_binop.argtypes = [i32, i32, vp, vp, vp, sz]
    return L


def _nan_mask(x, e, m):
    x = x.astype(np.uint64)
    E = (x >> m) & ((1 << e) - 1)
    M = x & ((1 << m) - 1)
    return (E == (1 << e) - 1) & (M != 0)


def _compare(e, m, got, want, a, b, what):
    gn, wn = _nan_mask(got, e, m), _nan_mask(want, e, m)
    assert np.array_equal(gn, wn), (what, np.flatnonzero(gn != wn)[:5])
    canon = ((1 << e) - 1) << m | (1 << (m - 1))
    assert np.all(got[gn] == canon)
    ok = (got == want) | wn
    bad = np.flatnonzero(~ok)
    assert bad.size == 0, [(what, hex(a[i]), hex(b[i]), hex(got[i]), hex(want[i])) for i in bad[:5]]


def _operands(rng, e, m, n):
    """Uniform patterns, near-cancellation pairs, subnormal-heavy pairs, small exponent gaps."""
    B = 1 + e + m
    top = 1 << B
    a = rng.integers(0, top, n, dtype=np.uint64)
    b = rng.integers(0, top, n, dtype=np.uint64)
    q = n // 4
    # near cancellation: b = -(a +- small)
    b[:q] = ((a[:q] + rng.integers(0, 5, q).astype(np.uint64)) % top) ^ (1 << (e + m))
    # subnormal / tiny exponents
    mmask = (1 << m) - 1
    a[q:2 * q] = (rng.integers(0, 3, q).astype(np.uint64) << m) | (a[q:2 * q] & mmask) | \
        (a[q:2 * q] & (1 << (e + m)))
    # exponent gap 0 .. m+4
    gap = rng.integers(0, m + 5, q).astype(np.int64)
    ea = ((a[2 * q:3 * q] >> m) & ((1 << e) - 1)).astype(np.int64)
    eb = np.clip(ea - gap, 0, (1 << e) - 2).astype(np.uint64)
    b[2 * q:3 * q] = (b[2 * q:3 * q] & ~np.uint64(((1 << e) - 1) << m)) | (eb << m)
    return a.astype(np.uint32), b.astype(np.uint32)


def _edges(e, m):
    from tests.exact_model import Fmt, edge_patterns
    f = Fmt(e, m)
    pos = edge_patterns(f)
    pats = pos + [p | f.sign_bit for p in pos]
    a = np.array([x for x in pats for _ in pats], dtype=np.uint32)
    b = np.array([y for _ in pats for y in pats], dtype=np.uint32)
    return a, b


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("op", [0, 1, 2, 3])
def test_binary32(oracle_lib, native, op, mode):
    rng = np.random.default_rng(23 + 3 * op + mode)
    a, b = _operands(rng, 8, 23, 200000)
    ea, eb = _edges(8, 23)
    a, b = np.concatenate([a, ea]), np.concatenate([b, eb])
    want = np.empty_like(a)
    native.f32_binop(op, mode, a.ctypes.data, b.ctypes.data, want.ctypes.data, a.size)
    got = oracle_lib.binop(op, 8, 23, mode, a, b, nthreads=4)
    _compare(8, 23, got, want, a, b, ("f32", op, mode))


@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
def test_binary16_rne_numpy(oracle_lib, op):
    rng = np.random.default_rng(16)
    a, b = _operands(rng, 5, 10, 400000)
    ea, eb = _edges(5, 10)
    a, b = np.concatenate([a, ea]), np.concatenate([b, eb])
    ha, hb = a.astype(np.uint16).view(np.float16), b.astype(np.uint16).view(np.float16)
    with np.errstate(all="ignore"):
        r = {"add": ha + hb, "sub": ha - hb, "mul": ha * hb, "div": ha / hb}[op]
    want = r.view(np.uint16).astype(np.uint32)
    got = oracle_lib.binop(op, 5, 10, 0, a, b, nthreads=4)
    _compare(5, 10, got, want, a, b, ("f16 rne", op))


@pytest.mark.parametrize("op", [0, 1, 2, 3])
def test_binary16_rz_f16c(oracle_lib, native, op):
    rng = np.random.default_rng(160 + op)
    a, b = _operands(rng, 5, 10, 400000)
    ea, eb = _edges(5, 10)
    a, b = np.concatenate([a, ea]), np.concatenate([b, eb])
    a16, b16 = a.astype(np.uint16), b.astype(np.uint16)
    w16 = np.empty_like(a16)
    native.f16_binop_rz(op, a16.ctypes.data, b16.ctypes.data, w16.ctypes.data, a16.size)
    got = oracle_lib.binop(op, 5, 10, 1, a, b, nthreads=4)
    _compare(5, 10, got, w16.astype(np.uint32), a, b, ("f16 rz", op))


def test_binary16_exhaustive_slice(oracle_lib):
    """All b against a fixed set of a's (65,536 x 64 pairs), binary16 RNE."""
    bs = np.arange(65536, dtype=np.uint32)
    rng = np.random.default_rng(99)
    for av in rng.integers(0, 65536, 64):
        a = np.full(65536, av, dtype=np.uint32)
        ha, hb = a.astype(np.uint16).view(np.float16), bs.astype(np.uint16).view(np.float16)
        for op in ("add", "mul", "div"):
            with np.errstate(all="ignore"):
                r = {"add": ha + hb, "mul": ha * hb, "div": ha / hb}[op]
            got = oracle_lib.binop(op, 5, 10, 0, a, bs)
            _compare(5, 10, got, r.view(np.uint16).astype(np.uint32), a, bs, ("f16 slice", op))


def test_division_small_dividends(oracle_lib, native):
    """Quotients of a subnormal by a value of the lowest binades: the integer
    quotient then has the fewest bits below the rounding point, so a dropped
    remainder (a tie mistaken for an exact half) shows.  binary16: every
    subnormal against every divisor with biased exponent 1 or 2, both modes;
    binary32: small subnormal dividends against sampled low-binade divisors."""
    a1 = np.arange(1024, dtype=np.uint32)
    b1 = np.arange(1024, 3072, dtype=np.uint32)
    a = np.repeat(a1, b1.size)
    b = np.tile(b1, a1.size) | (np.arange(a.size, dtype=np.uint32) & 1) << 15
    ha, hb = a.astype(np.uint16).view(np.float16), b.astype(np.uint16).view(np.float16)
    with np.errstate(all="ignore"):
        want = (ha / hb).view(np.uint16).astype(np.uint32)
    _compare(5, 10, oracle_lib.binop("div", 5, 10, 0, a, b, nthreads=8), want, a, b, ("f16 div", 0))
    a16, b16 = a.astype(np.uint16), b.astype(np.uint16)
    w16 = np.empty_like(a16)
    native.f16_binop_rz(3, a16.ctypes.data, b16.ctypes.data, w16.ctypes.data, a16.size)
    _compare(5, 10, oracle_lib.binop("div", 5, 10, 1, a, b, nthreads=8), w16.astype(np.uint32),
             a, b, ("f16 div", 1))
    rng = np.random.default_rng(41)
    bs = ((rng.integers(1, 4, 20000) << 23) | rng.integers(0, 1 << 23, 20000)).astype(np.uint32)
    a = np.repeat(np.arange(1, 33, dtype=np.uint32), bs.size)
    b = np.tile(bs, 32)
    for mode in (0, 1):
        want = np.empty_like(a)
        native.f32_binop(3, mode, a.ctypes.data, b.ctypes.data, want.ctypes.data, a.size)
        _compare(8, 23, oracle_lib.binop("div", 8, 23, mode, a, b, nthreads=8), want, a, b,
                 ("f32 div", mode))


@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
def test_bfloat16_rne_torch(oracle_lib, op):
    torch = pytest.importorskip("torch")
    torch.set_flush_denormal(False)
    # torch computes bf16 arithmetic in float32 and rounds once to nearest-even;
    # check that on a tie first: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7.
    one = torch.tensor([0x3F80], dtype=torch.int16).view(torch.bfloat16)
    tiny = torch.tensor([0x3B80], dtype=torch.int16).view(torch.bfloat16)
    assert int((one + tiny).view(torch.int16)) == 0x3F80
    rng = np.random.default_rng(87)
    a, b = _operands(rng, 8, 7, 400000)
    ea, eb = _edges(8, 7)
    a, b = np.concatenate([a, ea]), np.concatenate([b, eb])
    ta = torch.from_numpy(a.astype(np.uint16).view(np.int16)).view(torch.bfloat16)
    tb = torch.from_numpy(b.astype(np.uint16).view(np.int16)).view(torch.bfloat16)
    r = {"add": ta + tb, "sub": ta - tb, "mul": ta * tb, "div": ta / tb}[op]
    want = r.view(torch.int16).numpy().view(np.uint16).astype(np.uint32)
    got = oracle_lib.binop(op, 8, 7, 0, a, b, nthreads=4)
    _compare(8, 7, got, want, a, b, ("bf16", op))


def test_from_double_matches_native_conversions(oracle_lib):
    """oracle_from_double (round a binary64 value once) against numpy's
    binary64 -> binary16 and -> binary32 conversions (nearest-even), over
    random magnitudes spanning subnormals, normals and overflow."""
    rng = np.random.default_rng(64)
    x = rng.standard_normal(20000) * np.exp2(rng.uniform(-160, 140, 20000))
    x = np.concatenate([x, [0.0, -0.0, np.inf, -np.inf, 65520.0, 65519.99, 2.0 ** -25, 2.0 ** -24 * 1.5,
                            -(2.0 ** -149), 2.0 ** -150, 3.4028235677973366e38]])
    with np.errstate(all="ignore"):
        h = x.astype(np.float16).view(np.uint16)
        f = x.astype(np.float32).view(np.uint32)
    for i, v in enumerate(x):
        assert oracle_lib.from_double(5, 10, 0, v) == int(h[i]), v
        assert oracle_lib.from_double(8, 23, 0, v) == int(f[i]), v
    assert oracle_lib.from_double(5, 10, 0, float("nan")) == 0x7E00


@pytest.mark.parametrize("mode", [0, 1])
def test_chain2_binary32(oracle_lib, native, mode):
    """Two-op chains: the oracle's composition against binary32 arithmetic
    with the intermediate rounded to float (every op pair of add/sub/mul)."""
    rng = np.random.default_rng(70 + mode)
    a, b = _operands(rng, 8, 23, 60000)
    c, _ = _operands(rng, 8, 23, 60000)
    ops = ["add", "sub", "mul"]
    for i1, op1 in enumerate(ops):
        for i2, op2 in enumerate(ops):
            want = np.empty_like(a)
            native.f32_chain2(i1, i2, mode, a.ctypes.data, b.ctypes.data, c.ctypes.data, want.ctypes.data, a.size)
            got = oracle_lib.chain2(op1, op2, 8, 23, mode, a, b, c, nthreads=4)
            _compare(8, 23, got, want, a, b, ("f32 chain", op1, op2, mode))


def test_axpy_binary16_numpy(oracle_lib):
    """alpha * x + y in binary16 (numpy float16: each op rounded to nearest)."""
    rng = np.random.default_rng(71)
    x, y = _operands(rng, 5, 10, 100000)
    for alpha in (0x3C00, 0xC100, 0x0001, 0x7BFF, 0x8000, 0x7C00, 0x3555):
        hx, hy = x.astype(np.uint16).view(np.float16), y.astype(np.uint16).view(np.float16)
        ha = np.float16(np.uint16(alpha).view(np.float16))
        with np.errstate(all="ignore"):
            want = (ha * hx + hy).view(np.uint16).astype(np.uint32)
        got = oracle_lib.axpy(5, 10, 0, alpha, x, y, nthreads=4)
        _compare(5, 10, got, want, x, y, ("f16 axpy", hex(alpha)))


def _operands64(rng, n):
    """binary64 patterns: uniform, near-cancelling, subnormal-heavy, small
    exponent gaps and gaps of up to 2000 binades."""
    e, m = 11, 52
    a = rng.integers(0, 1 << 64, n, dtype=np.uint64)
    b = rng.integers(0, 1 << 64, n, dtype=np.uint64)
    q = n // 5
    sign = np.uint64(1 << 63)
    b[:q] = (a[:q] + rng.integers(0, 5, q).astype(np.uint64)) ^ sign
    mmask = np.uint64((1 << m) - 1)
    a[q:2 * q] = (rng.integers(0, 3, q).astype(np.uint64) << np.uint64(m)) | (a[q:2 * q] & mmask) | \
        (a[q:2 * q] & sign)
    ea = ((a[2 * q:3 * q] >> np.uint64(m)) & np.uint64(0x7FF)).astype(np.int64)
    eb = np.clip(ea - rng.integers(0, m + 5, q), 0, 0x7FE).astype(np.uint64)
    b[2 * q:3 * q] = (b[2 * q:3 * q] & ~np.uint64(0x7FF << m)) | (eb << np.uint64(m))
    ea = rng.integers(1000, 2046, q).astype(np.int64)
    eb = np.clip(ea - rng.integers(0, 2000, q), 0, 0x7FE)
    a[3 * q:4 * q] = (a[3 * q:4 * q] & (mmask | sign)) | (ea.astype(np.uint64) << np.uint64(m))
    b[3 * q:4 * q] = (b[3 * q:4 * q] & (mmask | sign)) | (eb.astype(np.uint64) << np.uint64(m))
    return a, b


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("op", [0, 1, 2, 3])
def test_binary64(oracle_lib, native, op, mode):
    """(11,52) is binary64: x86 double arithmetic under fesetround."""
    rng = np.random.default_rng(640 + 4 * op + mode)
    a, b = _operands64(rng, 200000)
    from tests.exact_model import Fmt, edge_patterns
    pos = edge_patterns(Fmt(11, 52))
    pats = pos + [p | (1 << 63) for p in pos]
    a = np.concatenate([a, np.array([x for x in pats for _ in pats], dtype=np.uint64)])
    b = np.concatenate([b, np.array([y for _ in pats for y in pats], dtype=np.uint64)])
    want = np.empty_like(a)
    native.f64_binop(op, mode, a.ctypes.data, b.ctypes.data, want.ctypes.data, a.size)
    got = oracle_lib.binop(op, 11, 52, mode, a, b, nthreads=8)
    _compare(11, 52, got, want, a, b, ("f64", op, mode))


def test_from_double_binary64_is_identity(oracle_lib):
    rng = np.random.default_rng(9)
    x = rng.integers(0, 1 << 64, 2000, dtype=np.uint64)
    for v in x:
        f = float(np.uint64(v).view(np.float64))
        if f != f:
            continue
        assert oracle_lib.from_double(11, 52, 0, f) == int(v)
