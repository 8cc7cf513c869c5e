"""Pin the oracle's k-bit integer operations (no GPU).

* wrap, k = 8, 16, 32: numpy's wrapping uint8/16/32 (and int8/16/32)
  arithmetic;
* unsigned and signed saturation, k = 8, 16: the x86 saturating add/sub
  instructions, and products formed exactly in wider lanes narrowed by the
  saturating packs (signed) or an unsigned minimum (unsigned);
* every k <= 6, all pairs, all ops and kinds: a table search over the k-bit
  patterns (the nearest representable value to the exact result for the
  saturating kinds, the representable value congruent to it modulo 2^k for
  wrap), which computes no clamp or remainder.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
OPS = ["add", "sub", "mul"]


@pytest.fixture(scope="module")
def native():
    so = os.path.join(HERE, "_native_pins.so")
    src = os.path.join(HERE, "native_pins.c")
    if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O1", "-frounding-math", "-fno-fast-math", "-mf16c",
                               "-msse4.1", "-fPIC", "-shared", src, "-o", so + ".tmp"])
        os.replace(so + ".tmp", so)
    L = ctypes.CDLL(so)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    L.int_sat_sse.argtypes = [i32, i32, i32, vp, vp, vp, sz]
    return L


def _edges(k):
    top = (1 << k) - 1
    e = {0, 1, 2, 3, top, top - 1, top - 2, 1 << (k - 1), (1 << (k - 1)) - 1, (1 << (k - 1)) + 1,
         1 << (k // 2), (1 << (k // 2)) - 1}
    return sorted(x & top for x in e)


def _operands(k, n, seed):
    rng = np.random.default_rng(seed)
    a = rng.integers(0, 1 << k, n, dtype=np.uint64)
    b = rng.integers(0, 1 << k, n, dtype=np.uint64)
    # small magnitudes of either sign, where products do not saturate
    q = n // 4
    a[:q] = rng.integers(0, 1 << max(1, k // 2), q) ^ (rng.integers(0, 2, q) * ((1 << k) - 1))
    b[:q] = rng.integers(0, 1 << max(1, k // 2), q) ^ (rng.integers(0, 2, q) * ((1 << k) - 1))
    ed = _edges(k)
    ea = np.array([x for x in ed for _ in ed], dtype=np.uint64)
    eb = np.array([y for _ in ed for y in ed], dtype=np.uint64)
    top = np.uint64((1 << k) - 1)
    return (np.concatenate([a, ea]) & top).astype(np.uint32), (np.concatenate([b, eb]) & top).astype(np.uint32)


@pytest.mark.parametrize("k", [8, 16, 32])
@pytest.mark.parametrize("op", OPS)
def test_wrap_against_numpy(oracle_lib, k, op):
    a, b = _operands(k, 100000, k + len(op))
    for dt in ({8: np.uint8, 16: np.uint16, 32: np.uint32}[k], {8: np.int8, 16: np.int16, 32: np.int32}[k]):
        ua = a.astype({8: np.uint8, 16: np.uint16, 32: np.uint32}[k]).view(dt)
        ub = b.astype({8: np.uint8, 16: np.uint16, 32: np.uint32}[k]).view(dt)
        with np.errstate(all="ignore"):
            r = {"add": ua + ub, "sub": ua - ub, "mul": ua * ub}[op]
        want = r.view({8: np.uint8, 16: np.uint16, 32: np.uint32}[k]).astype(np.uint32)
        assert np.array_equal(oracle_lib.int_binop(op, k, "wrap", a, b), want), (k, op, dt)


@pytest.mark.parametrize("k", [8, 16])
@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("kind", ["satu", "sats"])
def test_saturation_against_sse(oracle_lib, native, k, op, kind):
    a, b = _operands(k, 100000, 3 * k + len(op) + len(kind))
    want = np.empty_like(a)
    native.int_sat_sse(OPS.index(op), k, 1 if kind == "satu" else 2, a.ctypes.data, b.ctypes.data,
                       want.ctypes.data, a.size)
    got = oracle_lib.int_binop(op, k, kind, a, b)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, [(hex(a[i]), hex(b[i]), hex(got[i]), hex(want[i])) for i in bad[:5]]


def _table_search(k, kind, op, pa, pb):
    """Result pattern by search over all 2^k patterns."""
    signed = kind == "sats"

    def val(p):
        return p - (1 << k) if (signed and p >> (k - 1)) else p

    x, y = val(pa), val(pb)
    exact = x + y if op == "add" else (x - y if op == "sub" else x * y)
    pats = range(1 << k)
    if kind == "wrap":
        hits = [p for p in pats if (p - exact) % (1 << k) == 0]
        assert len(hits) == 1
        return hits[0]
    # nearest representable value (unique: the value set is an interval of integers)
    return min(pats, key=lambda p: abs(val(p) - exact))


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_small_k_exhaustive_table_search(oracle_lib, k):
    n = 1 << k
    a = np.repeat(np.arange(n, dtype=np.uint32), n)
    b = np.tile(np.arange(n, dtype=np.uint32), n)
    for op in OPS:
        for kind in ("wrap", "satu", "sats"):
            got = oracle_lib.int_binop(op, k, kind, a, b)
            for i in range(a.size):
                assert int(got[i]) == _table_search(k, kind, op, int(a[i]), int(b[i])), \
                    (k, op, kind, int(a[i]), int(b[i]))


def test_upper_bits_ignored(oracle_lib):
    a = np.array([0x1F3, 0xFFFFFF05], dtype=np.uint32)
    b = np.array([0x102, 0x7], dtype=np.uint32)
    assert np.array_equal(oracle_lib.int_binop("add", 8, "wrap", a, b),
                          oracle_lib.int_binop("add", 8, "wrap", a & 0xFF, b & 0xFF))
