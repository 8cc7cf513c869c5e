"""The gate-level circuits, instantiated for the host CPU, against the oracle.

``libbfp_hostsim.so`` compiles the same netlists the GPU kernels run
(bfp_circuits.hpp, bfp_transpose.hpp) with 32- and 64-bit host words; these
tests catch netlist mistakes without a GPU.  They are not a fallback: the GPU
library never loads this file.
"""
import ctypes
import os

import numpy as np
import pytest

from paper_1602_04716_amd import build, inputs

FORMATS = inputs.sweep_formats()


@pytest.fixture(scope="module")
def sim():
    if not os.path.exists(build.HOSTSIM):
        build.build()
    L = ctypes.CDLL(build.HOSTSIM)
    L.bfpsim_binop.argtypes = [ctypes.c_int] * 5 + [ctypes.c_void_p] * 3 + [ctypes.c_uint64]
    L.bfpsim_gate_count.restype = ctypes.c_long
    L.bfpsim_gate_count.argtypes = [ctypes.c_int] * 4
    L.bfpsim_ripple_add13.argtypes = [ctypes.c_void_p] * 3
    L.bfpsim_transpose.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    L.bfpsim_int_binop.argtypes = [ctypes.c_int] * 4 + [ctypes.c_void_p] * 3 + [ctypes.c_uint64]
    L.bfpsim_int_gate_count.restype = ctypes.c_long
    L.bfpsim_int_gate_count.argtypes = [ctypes.c_int] * 3
    L.bfpsim_binop64.argtypes = [ctypes.c_int] * 5 + [ctypes.c_void_p] * 3 + [ctypes.c_uint64]
    return L


def _run(L, op, e, m, mode, a, b, w=32):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    b = np.ascontiguousarray(b, dtype=np.uint32)
    c = np.empty_like(a)
    assert L.bfpsim_binop(op, e, m, mode, w, a.ctypes.data, b.ctypes.data, c.ctypes.data, a.size) == 0
    return c


SMALL = [(e, m) for (e, m) in FORMATS if 1 + e + m <= 8]


@pytest.mark.parametrize("e,m", SMALL)
def test_exhaustive_small(sim, oracle_lib, e, m):
    B = 1 + e + m
    a, b = inputs.exhaustive_pairs(B)
    for op in (0, 1, 2, 3):
        for mode in (0, 1):
            assert np.array_equal(_run(sim, op, e, m, mode, a, b), oracle_lib.binop(op, e, m, mode, a, b))


@pytest.mark.parametrize("e,m", FORMATS)
def test_random_and_edges(sim, oracle_lib, e, m):
    from tests.exact_model import Fmt, edge_patterns
    f = Fmt(e, m)
    B = f.B
    rng = np.random.default_rng(e * 31 + m)
    n = 20000
    a = rng.integers(0, 1 << B, n, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 1 << B, n, dtype=np.uint64).astype(np.uint32)
    q = n // 4
    b[:q] = (((a[:q].astype(np.uint64) + rng.integers(0, 3, q).astype(np.uint64)) % (1 << B))
             ^ (1 << (e + m))).astype(np.uint32)
    # subnormal or lowest-binade dividends (and divisors): the quotient's
    # fewest bits below the rounding point, and the pre-normalisation shifts
    low = (1 << (m + 2)) - 1 | (1 << (e + m))
    a[q:2 * q] &= low
    b[2 * q:3 * q] &= low
    pos = edge_patterns(f)
    pats = pos + [p | f.sign_bit for p in pos]
    ea = np.array([x for x in pats for _ in pats], dtype=np.uint32)
    eb = np.array([y for _ in pats for y in pats], dtype=np.uint32)
    a, b = np.concatenate([a, ea]), np.concatenate([b, eb])
    for op in (0, 1, 2, 3):
        for mode in (0, 1):
            want = oracle_lib.binop(op, e, m, mode, a, b, nthreads=4)
            got32 = _run(sim, op, e, m, mode, a, b, 32)
            bad = np.flatnonzero(got32 != want)
            assert bad.size == 0, (op, mode, hex(a[bad[0]]), hex(b[bad[0]]), hex(got32[bad[0]]), hex(want[bad[0]]))
            assert np.array_equal(_run(sim, op, e, m, mode, a, b, 64), got32)  # W = 64 identical


def test_figure2_adder(sim):
    """Figure 2: 32 lanes of 13-bit unsigned addition, result mod 2^13."""
    rng = np.random.default_rng(2)
    for _ in range(50):
        x = rng.integers(0, 1 << 13, 32)
        y = rng.integers(0, 1 << 13, 32)
        ap = np.array([sum(((int(x[j]) >> k) & 1) << j for j in range(32)) for k in range(13)], dtype=np.uint32)
        bp = np.array([sum(((int(y[j]) >> k) & 1) << j for j in range(32)) for k in range(13)], dtype=np.uint32)
        rp = np.zeros(13, dtype=np.uint32)
        sim.bfpsim_ripple_add13(ap.ctypes.data, bp.ctypes.data, rp.ctypes.data)
        got = [sum(((int(rp[k]) >> j) & 1) << k for k in range(13)) for j in range(32)]
        assert got == [int((x[j] + y[j]) % (1 << 13)) for j in range(32)]


def test_table1_cost_growth(sim):
    """Table 1: add costs O(n log n) in the significand width (alignment and
    normalisation shifters), mul and div O(n^2) (the significand multiply,
    the digit-by-digit divide).  Least squares over p = m + 1 at fixed e = 8:
    the p^2 coefficients are ~3 gates per cell (array multiplier: and, sum,
    carry; restoring divider: difference, borrow, restore); add has no
    quadratic term but a positive term in p times the number of log-shifter
    stages."""
    ms = [1, 2, 3, 5, 7, 10, 15, 23]
    p = np.array([m + 1 for m in ms], dtype=float)
    for mode in (0, 1):
        add = np.array([sim.bfpsim_gate_count(0, 8, m, mode) for m in ms], dtype=float)
        mul = np.array([sim.bfpsim_gate_count(2, 8, m, mode) for m in ms], dtype=float)
        A = np.stack([np.ones_like(p), p, p ** 2], axis=1)
        c_mul = np.linalg.lstsq(A, mul, rcond=None)[0]
        assert 2.5 < c_mul[2] < 3.5, c_mul
        div = np.array([sim.bfpsim_gate_count(3, 8, m, mode) for m in ms], dtype=float)
        c_div = np.linalg.lstsq(A, div, rcond=None)[0]
        assert 2.5 < c_div[2] < 3.5, c_div
        c_add_q = np.linalg.lstsq(A, add, rcond=None)[0]
        assert abs(c_add_q[2]) < 0.1 * c_mul[2], c_add_q
        stages = np.ceil(np.log2(p + 3))  # barrel-shifter stages over the aligned width
        L = np.stack([np.ones_like(p), p, p * stages], axis=1)
        c_add, res, *_ = np.linalg.lstsq(L, add, rcond=None)
        assert c_add[2] > 0, c_add
        fit = L @ c_add
        assert np.max(np.abs(fit - add) / add) < 0.05, (fit, add)


def test_round_toward_zero_is_cheaper(sim):
    """Section 5.2: toward-zero rounding needs fewer gates than nearest-even."""
    for (e, m) in FORMATS:
        for op in (0, 2, 3):
            assert sim.bfpsim_gate_count(op, e, m, 1) < sim.bfpsim_gate_count(op, e, m, 0)


@pytest.mark.parametrize("C", [1, 2, 4])
def test_transposes(sim, C):
    rng = np.random.default_rng(C)
    dt = {1: np.uint8, 2: np.uint16, 4: np.uint32}[C]
    for _ in range(100):
        x = rng.integers(0, np.iinfo(dt).max, 32, dtype=np.uint64, endpoint=True).astype(dt)
        inw = np.frombuffer(x.tobytes(), dtype=np.uint32).copy()
        out = np.zeros(8 * C, dtype=np.uint32)
        sim.bfpsim_transpose(C, 0, inw.ctypes.data, out.ctypes.data)
        want = np.array([sum(((int(x[j]) >> k) & 1) << j for j in range(32)) for k in range(8 * C)],
                        dtype=np.uint32)
        assert np.array_equal(out, want)
        back = np.zeros(8 * C, dtype=np.uint32)
        sim.bfpsim_transpose(C, 1, out.ctypes.data, back.ctypes.data)
        assert np.array_equal(back, inw)


def _int_operands(k, n, seed):
    rng = np.random.default_rng(seed)
    if k <= 6:
        a, b = inputs.exhaustive_pairs(k)
        return a.astype(np.uint32), b.astype(np.uint32)
    mask = np.uint64((1 << k) - 1)
    a = rng.integers(0, 1 << k, n, dtype=np.uint64)
    b = rng.integers(0, 1 << k, n, dtype=np.uint64)
    q = n // 4
    neg = rng.integers(0, 2, (2, q)).astype(np.uint64) * mask
    a[:q] = rng.integers(0, 1 << (k // 2), q).astype(np.uint64) ^ neg[0]
    b[:q] = rng.integers(0, 1 << (k // 2), q).astype(np.uint64) ^ neg[1]
    return (a & mask).astype(np.uint32), (b & mask).astype(np.uint32)


@pytest.mark.parametrize("k", list(range(1, 33)))
def test_int_circuits(sim, oracle_lib, k):
    """k-bit integer add/sub/mul, wrapping and both saturations, against the
    oracle (all pairs for k <= 6), 32- and 64-bit words identical."""
    a, b = _int_operands(k, 12000, k)
    for op in range(3):
        for kind in range(3):
            want = oracle_lib.int_binop(op, k, kind, a, b)
            for w in (32, 64):
                c = np.empty_like(a)
                assert sim.bfpsim_int_binop(op, k, kind, w, a.ctypes.data, b.ctypes.data, c.ctypes.data, a.size) == 0
                bad = np.flatnonzero(c != want)
                assert bad.size == 0, (op, kind, w, hex(a[bad[0]]), hex(b[bad[0]]), hex(c[bad[0]]), hex(want[bad[0]]))


def test_int_gate_counts():
    """Figure 2's adder costs one sum and one carry per bit: 2k - 1 gates
    with 3-input gates (the listing spends five bitwise operations per bit);
    the wrapping multiplier grows as ~1.5 k^2, the full-width (saturating)
    ones as ~3 k^2."""
    import ctypes as ct
    L = ct.CDLL(build.HOSTSIM)
    L.bfpsim_int_gate_count.restype = ct.c_long
    L.bfpsim_int_gate_count.argtypes = [ct.c_int] * 3
    for k in range(2, 33):
        assert L.bfpsim_int_gate_count(0, k, 0) == 2 * k - 1
    ks = np.arange(4, 33, dtype=float)
    for kind, lo, hi in ((0, 1.2, 1.8), (1, 2.5, 3.5), (2, 2.5, 3.5)):
        g = np.array([L.bfpsim_int_gate_count(2, int(k), kind) for k in ks], dtype=float)
        c = np.linalg.lstsq(np.stack([np.ones_like(ks), ks, ks ** 2], axis=1), g, rcond=None)[0]
        assert lo < c[2] < hi, (kind, c)


WIDE = [(8, 31), (11, 20), (11, 40), (11, 52)]


@pytest.mark.parametrize("e,m", WIDE)
def test_wide_formats(sim, oracle_lib, e, m):
    """The wide formats (patterns up to 64 bits) against the oracle: random
    pairs, subnormal-heavy and near-cancelling pairs, and the edge set."""
    from tests.exact_model import Fmt, edge_patterns
    B = 1 + e + m
    rng = np.random.default_rng(e * 100 + m)
    n = 4000
    a = rng.integers(0, 1 << B, n, dtype=np.uint64)
    b = rng.integers(0, 1 << B, n, dtype=np.uint64)
    low = np.uint64(((1 << (m + 2)) - 1) | (1 << (e + m)))
    a[:800] &= low
    b[800:1600] &= low
    b[1600:2400] = (a[1600:2400] + rng.integers(0, 3, 800).astype(np.uint64)) ^ np.uint64(1 << (e + m))
    pos = edge_patterns(Fmt(e, m))
    pats = pos + [p | (1 << (e + m)) for p in pos]
    a = np.concatenate([a, np.array([x for x in pats for _ in pats], dtype=np.uint64)])
    b = np.concatenate([b, np.array([y for _ in pats for y in pats], dtype=np.uint64)])
    for op in range(4):
        for mode in (0, 1):
            want = oracle_lib.binop(op, e, m, mode, a, b, nthreads=4).astype(np.uint64)
            for w in (32, 64):
                c = np.empty_like(a)
                assert sim.bfpsim_binop64(op, e, m, mode, w, a.ctypes.data, b.ctypes.data, c.ctypes.data, a.size) == 0
                bad = np.flatnonzero(c != want)
                assert bad.size == 0, (op, mode, w, hex(a[bad[0]]), hex(b[bad[0]]), hex(c[bad[0]]), hex(want[bad[0]]))
