"""GPU parity: the HIP path (through the C ABI) against the oracle, bit-exact.

Every test calls libbfp through its Python binding; expected values come only
from ``oracle`` (CPU).  Integer/bit work, so the bar is equality of every
bit, including the zero padding of the bitslice layout.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1602_04716_amd import bfp, inputs

pytestmark = pytest.mark.gpu

FORMATS = inputs.sweep_formats()
OPS = ["add", "sub", "mul", "div"]
NPAR = 70000 + 13  # 2188 words per plane: several blocks and a ragged last word


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bfp.lib()
    oracle.build()
    yield
    torch.cuda.synchronize()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _operands(e, m, n, seed):
    """Half format-shaped values, a quarter uniform bit patterns (NaN/Inf,
    upper garbage bits excluded by the container), a quarter near-cancelling."""
    dt = inputs.container_dtype(e, m)
    B = 1 + e + m
    rng = np.random.default_rng(seed)
    a = inputs.sweep_operands(e, m, n, seed).astype(np.uint64)
    b = inputs.sweep_operands(e, m, n, seed + 1).astype(np.uint64)
    q = n // 4
    a[:q] = rng.integers(0, 1 << B, q, dtype=np.uint64)
    b[:q] = rng.integers(0, 1 << B, q, dtype=np.uint64)
    b[q:2 * q] = ((a[q:2 * q] + rng.integers(0, 3, q).astype(np.uint64)) % (1 << B)) ^ (1 << (e + m))
    return a.astype(dt), b.astype(dt)


def _set_wpl(op, f, wpl, unroll=1):
    bfp.bfp_launch_set(op, f, wpl, 256, 0, unroll)


def _shapes(e, m):
    """(words per lane, units per step) pairs compiled for the format."""
    sh = [(1, 1), (2, 1), (1, 2)]
    if 1 + e + m <= 10:
        sh.append((4, 1))
    return sh


@pytest.mark.parametrize("e,m", FORMATS)
def test_pack_unpack(e, m):
    f = bfp.fmt(e, m)
    dt = inputs.container_dtype(e, m)
    rng = np.random.default_rng(e * 100 + m)
    for n in (1, 31, 33, 64 * 32 + 5, NPAR):
        x = rng.integers(0, np.iinfo(dt).max, n, dtype=np.uint64, endpoint=True).astype(dt)
        bs = bfp.pack(f, _dev(x))
        want = oracle.pack(e, m, x)
        assert np.array_equal(_host(bs), want), ("pack", n)
        back = bfp.unpack(f, bs, n)
        mask = (1 << (1 + e + m)) - 1
        assert np.array_equal(_host(back), (x.astype(np.uint64) & mask).astype(dt)), ("unpack", n)


@pytest.mark.parametrize("e,m", FORMATS + [(8, 31)])
def test_pack_unpack_across_lanes(e, m):
    """The cross-lane transposes (BFP_TRANSPOSE_XLANE) against the oracle's
    layout, on ragged lengths, tails and padding tiles included; 8-byte
    containers keep the per-lane method."""
    f = bfp.fmt(e, m)
    dt = inputs.container_dtype(e, m) if 1 + e + m <= 32 else np.uint64
    cb = bfp.bfp_container_bytes(f)
    rng = np.random.default_rng(e * 1000 + m)
    if cb == 8:
        with pytest.raises(bfp.BfpError):
            bfp.bfp_layout_method_set("pack", cb, bfp.BFP_TRANSPOSE_XLANE)
        return
    try:
        bfp.bfp_layout_method_set("pack", cb, bfp.BFP_TRANSPOSE_XLANE)
        bfp.bfp_layout_method_set("unpack", cb, bfp.BFP_TRANSPOSE_XLANE)
        for n in (1, 31, 33, 2047, 2049, 64 * 32 * 5 + 17, NPAR):
            x = rng.integers(0, np.iinfo(dt).max, n, dtype=np.uint64, endpoint=True).astype(dt)
            bs = bfp.pack(f, _dev(x))
            assert np.array_equal(_host(bs), oracle.pack(e, m, x)), ("pack", n)
            back = bfp.unpack(f, bs, n)
            mask = (1 << (1 + e + m)) - 1
            assert np.array_equal(_host(back), (x.astype(np.uint64) & mask).astype(dt)), ("unpack", n)
    finally:
        bfp.bfp_layout_method_set("pack", cb, bfp.BFP_TRANSPOSE_LANE)
        bfp.bfp_layout_method_set("unpack", cb, bfp.BFP_TRANSPOSE_LANE)


@pytest.mark.parametrize("e,m", FORMATS)
def test_binop_bitslice(e, m):
    a, b = _operands(e, m, NPAR, 7 * e + m)
    da, db = _dev(a), _dev(b)
    for mode in (0, 1):
        f = bfp.fmt(e, m, mode)
        pa, pb = bfp.pack(f, da), bfp.pack(f, db)
        for op in OPS:
            want = oracle.binop(op, e, m, mode, a, b, nthreads=8)
            want_planes = oracle.pack(e, m, want)
            for wpl, unroll in _shapes(e, m):
                _set_wpl(op, f, wpl, unroll)
                pc = bfp.empty_bitslice(f, NPAR)
                bfp.bfp_binop(op, f, pa, pb, pc, NPAR)
                got = _host(pc)
                if not np.array_equal(got, want_planes):
                    res = oracle.unpack(e, m, got, NPAR).astype(np.uint32)
                    bad = np.flatnonzero(res != want)
                    k = bad[0] if bad.size else -1
                    pytest.fail("(%d,%d) %s mode %d wpl %d unroll %d: %d bad elements, e.g. a=%#x b=%#x got=%#x "
                                "want=%#x" % (e, m, op, mode, wpl, unroll, bad.size, a[k], b[k], res[k], want[k]))
            _set_wpl(op, f, 1)
            out = bfp.unpack(f, pc, NPAR)
            assert np.array_equal(_host(out).astype(np.uint32), want)


@pytest.mark.parametrize("e,m", FORMATS)
def test_binop_std_fused(e, m):
    a, b = _operands(e, m, NPAR, 11 * e + m)
    da, db = _dev(a), _dev(b)
    for mode in (0, 1):
        f = bfp.fmt(e, m, mode)
        for op in OPS:
            want = oracle.binop(op, e, m, mode, a, b, nthreads=8)
            dc = torch.empty_like(da)
            bfp.bfp_binop_std(op, f, da, db, dc, NPAR)
            got = _host(dc).astype(np.uint32)
            bad = np.flatnonzero(got != want)
            assert bad.size == 0, ((e, m, op, mode), hex(a[bad[0]]), hex(b[bad[0]]), hex(got[bad[0]]),
                                   hex(want[bad[0]]))


SMALL = [(e, m) for (e, m) in FORMATS if 1 + e + m <= 8]


@pytest.mark.parametrize("e,m", SMALL)
def test_exhaustive_small_formats(e, m):
    """All 2^B x 2^B pairs (the 256 x 256 check at B = 8), both paths."""
    B = 1 + e + m
    a, b = inputs.exhaustive_pairs(B)
    a8, b8 = a.astype(np.uint8), b.astype(np.uint8)
    n = a.size
    da, db = _dev(a8), _dev(b8)
    for mode in (0, 1):
        f = bfp.fmt(e, m, mode)
        pa, pb = bfp.pack(f, da), bfp.pack(f, db)
        for op in OPS:
            want = oracle.binop(op, e, m, mode, a, b, nthreads=8)
            dc = torch.empty_like(da)
            bfp.bfp_binop_std(op, f, da, db, dc, n)
            assert np.array_equal(_host(dc).astype(np.uint32), want), ("std", op, mode)
            pc = bfp.empty_bitslice(f, n)
            bfp.bfp_binop(op, f, pa, pb, pc, n)
            assert np.array_equal(_host(bfp.unpack(f, pc, n)).astype(np.uint32), want), ("bs", op, mode)


def test_plain_add_5_2_workload():
    """65,536-element (5,2) add, 32-lane words, pack + add + unpack (fused and
    three-kernel), uniform patterns without NaN/Inf."""
    e, m = 5, 2
    n = 65536
    a = inputs.plain_8bit(n, seed=1)
    b = inputs.plain_8bit(n, seed=101)
    want = oracle.binop("add", e, m, 0, a, b)
    f = bfp.fmt(e, m)
    da, db = _dev(a), _dev(b)
    dc = torch.empty_like(da)
    bfp.bfp_binop_std("add", f, da, db, dc, n)
    assert np.array_equal(_host(dc).astype(np.uint32), want)
    _set_wpl("add", f, 1)
    pa, pb = bfp.pack(f, da), bfp.pack(f, db)
    pc = bfp.empty_bitslice(f, n)
    bfp.bfp_add(f, pa, pb, pc, n)
    assert np.array_equal(_host(bfp.unpack(f, pc, n)).astype(np.uint32), want)


def test_5_2_workload_captured_in_a_graph():
    """The fused call and the pack + add + unpack calls captured in one
    graph (two of each) and replayed three times, with other eager work on
    the operands' buffers between replays: every replay gives the oracle's
    result."""
    e, m = 5, 2
    n = 65536
    a = inputs.plain_8bit(n, seed=1)
    b = inputs.plain_8bit(n, seed=101)
    want = oracle.binop("add", e, m, 0, a, b)
    f = bfp.fmt(e, m)
    _set_wpl("add", f, 1)
    da, db = _dev(a), _dev(b)
    dc, dd = torch.empty_like(da), torch.empty_like(da)
    pa, pb, pc = (bfp.empty_bitslice(f, n) for _ in range(3))
    bfp.bfp_binop_std("add", f, da, db, dc, n)  # eager once, before the capture
    bfp.bfp_add(f, pa, pb, pc, n)
    torch.cuda.synchronize()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cs):
        for _ in range(2):
            bfp.bfp_binop_std("add", f, da, db, dc, n, cs)
            bfp.bfp_pack(f, da, pa, n, cs)
            bfp.bfp_pack(f, db, pb, n, cs)
            bfp.bfp_add(f, pa, pb, pc, n, cs)
            bfp.bfp_unpack(f, pc, dd, n, cs)
    for rep in range(3):
        dc.zero_()
        dd.fill_(0xFF)
        pc.zero_()
        g.replay()
        assert np.array_equal(_host(dc).astype(np.uint32), want), rep
        assert np.array_equal(_host(dd).astype(np.uint32), want), rep
        assert np.array_equal(_host(pc), oracle.pack(e, m, want)), rep
        bfp.bfp_mul(f, pa, pb, pc, n)  # eager work between replays


def test_in_place_and_zero_length():
    e, m = 5, 10
    f = bfp.fmt(e, m)
    a, b = _operands(e, m, 5000, 3)
    want = oracle.binop("mul", e, m, 0, a, b)
    pa, pb = bfp.pack(f, _dev(a)), bfp.pack(f, _dev(b))
    bfp.bfp_mul(f, pa, pb, pa, 5000)  # c == a
    assert np.array_equal(_host(bfp.unpack(f, pa, 5000)).astype(np.uint32), want)
    bfp.bfp_add(f, pa, pb, pa, 0)  # no-op
    pa = bfp.pack(f, _dev(a))
    bfp.bfp_div(f, pa, pb, pb, 5000)  # c == b
    assert np.array_equal(_host(bfp.unpack(f, pb, 5000)).astype(np.uint32), oracle.binop("div", e, m, 0, a, b))
    pb = bfp.pack(f, _dev(b))
    da = _dev(a)
    bfp.bfp_binop_std("sub", f, da, _dev(b), da, 5000)  # c == a, fused path
    assert np.array_equal(_host(da).astype(np.uint32), oracle.binop("sub", e, m, 0, a, b))


@pytest.mark.parametrize("e,m", [(5, 10), (8, 7)])
def test_full_size_2_26(e, m):
    """2^26 elements, 64-element lane words (the benchmark's launch
    configuration); sampled outputs against the oracle, and every output of
    (5,10) against the GPU's native binary16 arithmetic, (8,7) against
    bfloat16 computed in float32 (both correctly rounded to nearest-even)."""
    n = 1 << 26
    a = inputs.scaled_normal(e, m, n, 2)
    b = inputs.scaled_normal(e, m, n, 3)
    f = bfp.fmt(e, m)
    da, db = _dev(a), _dev(b)
    pa, pb = bfp.pack(f, da), bfp.pack(f, db)
    rng = np.random.default_rng(5)
    idx = np.concatenate([np.arange(4096), np.arange(n - 4096, n), rng.integers(0, n, 200000)])
    for op in OPS:
        bfp.bfp_launch_set(op, f, 2, 256, 0)
        pc = bfp.empty_bitslice(f, n)
        bfp.bfp_binop(op, f, pa, pb, pc, n)
        out = bfp.unpack(f, pc, n)
        got = _host(out).astype(np.uint32)
        want = oracle.binop(op, e, m, 0, a[idx], b[idx], nthreads=8)
        assert np.array_equal(got[idx], want), op
        ta, tb = da.view(torch.int16), db.view(torch.int16)
        if (e, m) == (5, 10):
            ha, hb = ta.view(torch.float16), tb.view(torch.float16)
        else:
            ha, hb = ta.view(torch.bfloat16).float(), tb.view(torch.bfloat16).float()
        r = {"add": ha + hb, "sub": ha - hb, "mul": ha * hb, "div": ha / hb}[op]
        if (e, m) == (8, 7):
            r = r.to(torch.bfloat16)
        nat = r.view(torch.int16).cpu().numpy().view(np.uint16).astype(np.uint32)
        E = (nat >> m) & ((1 << e) - 1)
        nat_nan = (E == (1 << e) - 1) & ((nat & ((1 << m) - 1)) != 0)
        mism = (nat != got) & ~nat_nan
        assert not mism.any(), (op, int(mism.sum()))
        del pc, out
    torch.cuda.synchronize()


@pytest.mark.parametrize("e,m", [(5, 10), (8, 7)])
def test_full_size_2_26_toward_zero(e, m):
    """The benchmark's size and launch configuration (64-element lane words)
    in round-toward-zero: every op, the first and last 4096 outputs and
    200,000 sampled ones against the oracle."""
    n = 1 << 26
    a = inputs.scaled_normal(e, m, n, 4)
    b = inputs.scaled_normal(e, m, n, 5)
    f = bfp.fmt(e, m, bfp.BFP_RZ)
    pa, pb = bfp.pack(f, _dev(a)), bfp.pack(f, _dev(b))
    rng = np.random.default_rng(6)
    idx = np.concatenate([np.arange(4096), np.arange(n - 4096, n), rng.integers(0, n, 200000)])
    for op in OPS:
        bfp.bfp_launch_set(op, f, 2, 256, 0)
        pc = bfp.empty_bitslice(f, n)
        bfp.bfp_binop(op, f, pa, pb, pc, n)
        got = _host(bfp.unpack(f, pc, n)).astype(np.uint32)
        want = oracle.binop(op, e, m, 1, a[idx], b[idx], nthreads=8)
        assert np.array_equal(got[idx], want), op
        del pc
    torch.cuda.synchronize()


def test_beyond_32_bit_offsets():
    """n = 2^33 + 77 elements of (5,2) (8 GiB per operand): plane word offsets
    and element offsets exceed 2^32, through pack, add, mul, unpack and the
    fused path; the first and last 4096 outputs and 100,000 sampled ones
    against the oracle, and the two paths against each other on every output."""
    e, m = 5, 2
    n = (1 << 33) + 77
    f = bfp.fmt(e, m)
    g = torch.Generator(device="cuda")
    g.manual_seed(33)
    da = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda", generator=g)
    db = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda", generator=g)
    rng = np.random.default_rng(33)
    idx = np.unique(np.concatenate([np.arange(4096), np.arange(n - 4096, n),
                                    rng.integers(0, n, 100000, dtype=np.int64)]))
    tidx = torch.from_numpy(idx).cuda()
    a = da[tidx].cpu().numpy()
    b = db[tidx].cpu().numpy()
    pa, pb = bfp.pack(f, da), bfp.pack(f, db)
    for op in ("add", "mul"):
        pc = bfp.empty_bitslice(f, n)
        bfp.bfp_binop(op, f, pa, pb, pc, n)
        out = bfp.unpack(f, pc, n)
        del pc
        want = oracle.binop(op, e, m, 0, a, b, nthreads=8)
        assert np.array_equal(out[tidx].cpu().numpy().astype(np.uint32), want), op
        fused = torch.empty_like(da)
        bfp.bfp_binop_std(op, f, da, db, fused, n)
        assert torch.equal(fused, out), op
        del out, fused
    torch.cuda.synchronize()


@pytest.mark.parametrize("e,m", FORMATS + inputs.wide_formats())
def test_small_ragged_lengths_all_formats(e, m):
    """Three random lengths in [1, 3000] per format (a partial last word and
    a partial last tile), every op, both modes, both paths, against the oracle."""
    B = 1 + e + m
    rng = np.random.default_rng(500 + 13 * e + m)
    dt = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}[oracle.container_bytes(e, m)]
    for n in rng.integers(1, 3001, 3):
        n = int(n)
        a = rng.integers(0, 1 << B, n, dtype=np.uint64).astype(dt)
        b = rng.integers(0, 1 << B, n, dtype=np.uint64).astype(dt)
        da, db = _dev(a), _dev(b)
        for mode in (0, 1):
            f = bfp.fmt(e, m, mode)
            pa, pb = bfp.pack(f, da), bfp.pack(f, db)
            for op in OPS:
                want = oracle.binop(op, e, m, mode, a, b).astype(np.uint64)
                pc = bfp.empty_bitslice(f, n)
                bfp.bfp_binop(op, f, pa, pb, pc, n)
                assert np.array_equal(_host(pc), oracle.pack(e, m, want)), (n, op, mode, "bitslice")
                dc = torch.empty_like(da)
                bfp.bfp_binop_std(op, f, da, db, dc, n)
                assert np.array_equal(_host(dc).astype(np.uint64), want), (n, op, mode, "std")


@pytest.mark.parametrize("e,m", [(5, 10), (8, 7)])
def test_all_2_32_pairs_against_device_arithmetic(e, m):
    """Every pair of 16-bit patterns (2^32 pairs) of binary16 and bfloat16,
    add/sub/mul/div to nearest even, on the fused path against the GPU's own
    arithmetic in torch (computed in float32 and rounded once to the 16-bit
    type, which is the correctly rounded result since 24 >= 2p + 2); NaN
    results compared as NaN."""
    f = bfp.fmt(e, m)
    dt = torch.float16 if (e, m) == (5, 10) else torch.bfloat16
    chunk = 1 << 28
    for base in range(0, 1 << 32, chunk):
        i = torch.arange(base, base + chunk, device="cuda", dtype=torch.int64)
        a = (i >> 16).to(torch.int32).to(torch.int16)
        b = (i & 0xFFFF).to(torch.int32).to(torch.int16)
        del i
        fa, fb = a.view(dt).float(), b.view(dt).float()
        for op in OPS:
            ours = torch.empty_like(a)
            bfp.bfp_binop_std(op, f, a, b, ours, chunk)
            r = {"add": fa + fb, "sub": fa - fb, "mul": fa * fb, "div": fa / fb}[op].to(dt)
            same = (ours == r.view(torch.int16)) | (torch.isnan(ours.view(dt)) & torch.isnan(r))
            if not bool(same.all()):
                bad = torch.nonzero(~same)[:5, 0]
                pytest.fail("%s (%d,%d): %d mismatches, e.g. %s" % (
                    op, e, m, int((~same).sum()),
                    [(hex(int(a[k]) & 0xFFFF), hex(int(b[k]) & 0xFFFF), hex(int(ours[k]) & 0xFFFF),
                      hex(int(r.view(torch.int16)[k]) & 0xFFFF)) for k in bad.tolist()]))
            del ours, r, same
        del a, b, fa, fb
    torch.cuda.synchronize()


def test_binary32_against_device_arithmetic():
    """(8,23) = binary32: 2^28 random pairs (uniform bit patterns, and pairs
    near cancellation) on the bitslice path against the GPU's own float32
    add/sub/mul/div (round to nearest even), NaN results compared as NaN."""
    f = bfp.fmt(8, 23)
    n = 1 << 28
    g = torch.Generator(device="cuda")
    g.manual_seed(32)
    a = torch.randint(-(1 << 31), 1 << 31, (n,), dtype=torch.int64, device="cuda", generator=g).to(torch.int32)
    b = torch.randint(-(1 << 31), 1 << 31, (n,), dtype=torch.int64, device="cuda", generator=g).to(torch.int32)
    q = n // 4
    b[:q] = (a[:q] + torch.randint(0, 3, (q,), dtype=torch.int32, device="cuda", generator=g)) ^ (-(1 << 31))
    pa, pb = bfp.pack(f, a), bfp.pack(f, b)
    fa, fb = a.view(torch.float32), b.view(torch.float32)
    for op in OPS:
        pc = bfp.empty_bitslice(f, n)
        bfp.bfp_binop(op, f, pa, pb, pc, n)
        ours = bfp.unpack(f, pc, n).view(torch.int32)
        del pc
        r = {"add": fa + fb, "sub": fa - fb, "mul": fa * fb, "div": fa / fb}[op]
        same = (ours == r.view(torch.int32)) | (torch.isnan(ours.view(torch.float32)) & torch.isnan(r))
        assert bool(same.all()), (op, int((~same).sum()))
        del ours, r, same
    torch.cuda.synchronize()


@pytest.mark.parametrize("e,m", FORMATS)
def test_sweep_format_full_size_2_24(e, m):
    """The format sweep at its full size: 2^24 elements per format, operands
    from the sweep recipe (a 2^20-element pool of log-uniform magnitudes with
    1% subnormals and zeros, drawn at random indices), add and mul in both
    modes with the tuned launch table.  Sampled outputs (first and last 4096,
    and 20,000 random ones) against the oracle; every output checked for
    commutativity (a op b and b op a give the same planes)."""
    n = 1 << 24
    rng = np.random.default_rng(2400 + 13 * e + m)
    pool_a = inputs.sweep_operands(e, m, 1 << 20, 3 + e)
    pool_b = inputs.sweep_operands(e, m, 1 << 20, 4 + m)
    a = pool_a[rng.integers(0, 1 << 20, n)]
    b = pool_b[rng.integers(0, 1 << 20, n)]
    idx = np.concatenate([np.arange(4096), np.arange(n - 4096, n), rng.integers(0, n, 20000)])
    da, db = _dev(a), _dev(b)
    for mode in (0, 1):
        f = bfp.fmt(e, m, mode)
        pa, pb = bfp.pack(f, da), bfp.pack(f, db)
        for op in ("add", "mul"):
            pc = bfp.empty_bitslice(f, n)
            bfp.bfp_binop(op, f, pa, pb, pc, n)
            pd = bfp.empty_bitslice(f, n)
            bfp.bfp_binop(op, f, pb, pa, pd, n)
            assert torch.equal(pc, pd), (op, mode, "commutativity")
            got = _host(bfp.unpack(f, pc, n)).astype(np.uint32)
            want = oracle.binop(op, e, m, mode, a[idx], b[idx], nthreads=8)
            assert np.array_equal(got[idx], want), (op, mode)
            del pc, pd
    torch.cuda.synchronize()
