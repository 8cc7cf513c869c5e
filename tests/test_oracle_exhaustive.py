"""Pin the oracle against an independent exact model (no GPU).

* Every format of at most 8 bits in the sweep: all 2^B x 2^B operand pairs,
  add/sub/mul/div, both rounding modes (Section 4: round toward zero and round to
  nearest, ties to even), against exact-rational table search.
* Every sweep format: random pairs plus the edge set, checked with the
  neighbour test (the result is correctly rounded iff no adjacent pattern is
  nearer / not above the exact value), which needs no table.
"""
import numpy as np
import pytest

from tests.exact_model import (Fmt, check_correctly_rounded, edge_patterns, sweep_formats,
                               table_round, tables, wide_formats)

SMALL = [(e, m) for (e, m) in sweep_formats() if 1 + e + m <= 8]


@pytest.mark.parametrize("e,m", SMALL)
@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
@pytest.mark.parametrize("mode", [0, 1])
def test_exhaustive_small_formats(oracle_lib, e, m, op, mode):
    f = Fmt(e, m)
    ta, tm = tables(f)
    n = 1 << f.B
    a = np.repeat(np.arange(n, dtype=np.uint32), n)
    b = np.tile(np.arange(n, dtype=np.uint32), n)
    got = oracle_lib.binop(op, e, m, mode, a, b)
    bad = []
    for i in range(a.size):
        want = table_round(f, ta, tm, op, mode, int(a[i]), int(b[i]))
        if int(got[i]) != want:
            bad.append((int(a[i]), int(b[i]), want, int(got[i])))
            if len(bad) > 5:
                break
    assert not bad, bad


def test_exhaustive_5_2_is_config_vector(oracle_lib):
    """The 256x256 pair vector of the (5,2) workload: a_i = i >> 8, b_i = i & 255."""
    e, m = 5, 2
    i = np.arange(65536, dtype=np.uint32)
    a, b = i >> 8, i & 255
    f = Fmt(e, m)
    ta, tm = tables(f)
    got = oracle_lib.binop("add", e, m, 0, a, b)
    for k in range(0, 65536, 7):
        assert int(got[k]) == table_round(f, ta, tm, "add", 0, int(a[k]), int(b[k]))


@pytest.mark.parametrize("e,m", [(3, 5), (4, 5)])
def test_nine_and_ten_bit_formats_sampled_table(oracle_lib, e, m):
    f = Fmt(e, m)
    ta, tm = tables(f)
    rng = np.random.default_rng(17)
    n = 4000
    a = rng.integers(0, 1 << f.B, n, dtype=np.uint32)
    b = rng.integers(0, 1 << f.B, n, dtype=np.uint32)
    for op in ("add", "sub", "mul", "div"):
        for mode in (0, 1):
            got = oracle_lib.binop(op, e, m, mode, a, b)
            for k in range(n):
                want = table_round(f, ta, tm, op, mode, int(a[k]), int(b[k]))
                assert int(got[k]) == want, (op, mode, hex(a[k]), hex(b[k]))


def _neighbour_case(oracle_lib, e, m, a, b):
    f = Fmt(e, m)
    for op in ("add", "sub", "mul", "div"):
        for mode in (0, 1):
            got = oracle_lib.binop(op, e, m, mode, a, b)
            for k in range(a.size):
                err = check_correctly_rounded(f, op, mode, int(a[k]), int(b[k]), int(got[k]))
                assert err is None, (e, m, op, mode, hex(a[k]), hex(b[k]), hex(got[k]), err)


@pytest.mark.parametrize("e,m", sweep_formats() + wide_formats())
def test_neighbour_random(oracle_lib, e, m):
    f = Fmt(e, m)
    rng = np.random.default_rng(1000 + 17 * e + m)
    n = 300
    a = rng.integers(0, 1 << f.B, n, dtype=np.uint64)
    # half the b's near a in magnitude, to exercise cancellation and ties
    b = rng.integers(0, 1 << f.B, n, dtype=np.uint64)
    near = np.array([(int(x) + int(d)) % (1 << f.B) for x, d in zip(a, rng.integers(-3, 4, n))], dtype=np.uint64)
    flip = rng.integers(0, 2, n).astype(np.uint64) << np.uint64(e + m)
    b[: n // 2] = near[: n // 2] ^ flip[: n // 2]
    _neighbour_case(oracle_lib, e, m, a, b)


@pytest.mark.parametrize("e,m", sweep_formats() + wide_formats())
def test_neighbour_edges(oracle_lib, e, m):
    f = Fmt(e, m)
    pos = edge_patterns(f)
    pats = pos + [p | f.sign_bit for p in pos]
    a = np.array([x for x in pats for _ in pats], dtype=np.uint64)
    b = np.array([y for _ in pats for y in pats], dtype=np.uint64)
    _neighbour_case(oracle_lib, e, m, a, b)


def test_pack_definition(oracle_lib):
    """Plane k, word i//32, bit i%32 holds bit k of element i (Section 2);
    checked with numpy bit ops, for each container size and a ragged n."""
    rng = np.random.default_rng(5)
    for (e, m) in [(5, 2), (4, 3), (5, 10), (8, 7), (8, 23), (3, 1), (8, 31), (11, 52)]:
        B = 1 + e + m
        for n in (1, 31, 33, 2048 + 17):
            dt = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}[oracle_lib.container_bytes(e, m)]
            x = rng.integers(0, np.iinfo(dt).max, n, dtype=np.uint64, endpoint=True).astype(dt)
            planes = oracle_lib.pack(e, m, x)
            gpad = planes.shape[1]
            assert gpad % 64 == 0 and gpad * 32 >= n
            bits = ((x.astype(np.uint64)[None, :] >> np.arange(B, dtype=np.uint64)[:, None]) & 1)
            full = np.zeros((B, gpad * 32), dtype=np.uint64)
            full[:, :n] = bits
            words = (full.reshape(B, gpad, 32) << np.arange(32, dtype=np.uint64)).sum(axis=2)
            assert np.array_equal(words.astype(np.uint32), planes)
            back = oracle_lib.unpack(e, m, planes, n)
            assert np.array_equal(back, (x.astype(np.uint64) & ((1 << B) - 1)).astype(dt))
