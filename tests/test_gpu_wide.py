"""Wide formats on the GPU (exponent up to 11 bits, patterns up to 64 bits):
pack/unpack, every op in both modes on both paths against the oracle, bit
for bit, and binary64 against the GPU's own double arithmetic at 2^24
elements."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1602_04716_amd import bfp

pytestmark = pytest.mark.gpu

WIDE = [(8, 31), (11, 20), (11, 40), (11, 52)]
OPS = ["add", "sub", "mul", "div"]
NPAR = 70000 + 13


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bfp.lib()
    oracle.build()
    yield
    torch.cuda.synchronize()


def _np_dtype(e, m):
    return {4: np.uint32, 8: np.uint64}[oracle.container_bytes(e, m)]


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _operands(e, m, n, seed):
    B = 1 + e + m
    dt = _np_dtype(e, m)
    rng = np.random.default_rng(seed)
    hi = 1 << (8 * np.dtype(dt).itemsize)
    a = rng.integers(0, hi, n, dtype=np.uint64)  # garbage above bit B-1 too
    b = rng.integers(0, hi, n, dtype=np.uint64)
    q = n // 4
    mask = np.uint64((1 << B) - 1) if B < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    sign = np.uint64(1 << (e + m))
    b[:q] = ((a[:q] & mask) + rng.integers(0, 3, q).astype(np.uint64)) ^ sign
    low = np.uint64(((1 << (m + 2)) - 1) | (1 << (e + m)))
    a[q:2 * q] &= low
    b[2 * q:3 * q] &= low
    return a.astype(dt), b.astype(dt)


@pytest.mark.parametrize("e,m", WIDE)
def test_wide_pack_unpack(e, m):
    B = 1 + e + m
    f = bfp.fmt(e, m)
    rng = np.random.default_rng(e + m)
    dt = _np_dtype(e, m)
    for n in (1, 31, 33, 2048 + 5, NPAR):
        x = rng.integers(0, np.iinfo(dt).max, n, dtype=np.uint64, endpoint=True).astype(dt)
        bs = bfp.pack(f, _dev(x))
        assert np.array_equal(_host(bs), oracle.pack(e, m, x)), n
        back = _host(bfp.unpack(f, bs, n)).astype(np.uint64)
        mask = (1 << B) - 1
        assert np.array_equal(back, x.astype(np.uint64) & np.uint64(mask)), n


@pytest.mark.parametrize("e,m", WIDE)
def test_wide_ops_both_paths(e, m):
    a, b = _operands(e, m, NPAR, 17 * e + m)
    da, db = _dev(a), _dev(b)
    for mode in (0, 1):
        f = bfp.fmt(e, m, mode)
        pa, pb = bfp.pack(f, da), bfp.pack(f, db)
        for op in OPS:
            want = oracle.binop(op, e, m, mode, a, b, nthreads=8).astype(np.uint64)
            pc = bfp.empty_bitslice(f, NPAR)
            bfp.bfp_binop(op, f, pa, pb, pc, NPAR)
            assert np.array_equal(_host(pc), oracle.pack(e, m, want)), ("bitslice", op, mode)
            dc = torch.empty_like(da)
            bfp.bfp_binop_std(op, f, da, db, dc, NPAR)
            got = _host(dc).astype(np.uint64)
            bad = np.flatnonzero(got != want)
            assert bad.size == 0, ("std", op, mode, hex(a[bad[0]]), hex(b[bad[0]]), hex(got[bad[0]]),
                                   hex(want[bad[0]]))


def test_binary64_against_device_double():
    """(11,52) = binary64: every output of 2^24 elements against torch's float64
    arithmetic on the same GPU (round to nearest even), NaNs compared as NaN."""
    n = 1 << 24
    rng = np.random.default_rng(64)
    a = rng.standard_normal(n) * np.exp2(rng.integers(-60, 60, n))
    b = rng.standard_normal(n) * np.exp2(rng.integers(-60, 60, n))
    b[: n // 8] = -a[: n // 8] * (1 + rng.integers(-4, 5, n // 8) * 2.0 ** -52)
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    f = bfp.fmt(11, 52)
    pa, pb = bfp.pack(f, ta.view(torch.uint64)), bfp.pack(f, tb.view(torch.uint64))
    for op in OPS:
        pc = bfp.empty_bitslice(f, n)
        bfp.bfp_binop(op, f, pa, pb, pc, n)
        got = bfp.unpack(f, pc, n).view(torch.float64)
        ref = {"add": ta + tb, "sub": ta - tb, "mul": ta * tb, "div": ta / tb}[op]
        same = (got.view(torch.int64) == ref.view(torch.int64)) | (torch.isnan(got) & torch.isnan(ref))
        assert bool(same.all()), (op, int((~same).sum()))
        del pc, got, ref
    torch.cuda.synchronize()


def test_wide_formats_rejected_by_batch_and_server():
    f = bfp.fmt(11, 52)
    n = 1000
    x = bfp.empty_bitslice(f, n)
    with pytest.raises(bfp.BfpError):
        bfp.bfp_batch_plan_create([(x, x, x, n, f, "add")])
    with pytest.raises(bfp.BfpError):
        bfp.bfp_autotune("mul", f, 1 << 16, 2, 1)  # two-word kernels are not compiled for f
    best, us = bfp.bfp_autotune("add", f, 1 << 16, 3, 1)
    assert best.words_per_lane == 1 and us > 0
