"""Two-op chains and axpy on the GPU (through the C ABI) against the oracle's
composition of the elementwise ops, bit for bit, and against the same two
ops launched separately (identical planes, padding included)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1602_04716_amd import bfp, inputs

pytestmark = pytest.mark.gpu

FORMATS = inputs.sweep_formats()
OPS = ["add", "sub", "mul"]
NPAR = 70000 + 13


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
    dt = inputs.container_dtype(e, m)
    B = 1 + e + m
    rng = np.random.default_rng(seed)
    xs = [inputs.sweep_operands(e, m, n, seed + k).astype(np.uint64) for k in range(3)]
    q = n // 4
    for x in xs:
        x[:q] = rng.integers(0, 1 << B, q, dtype=np.uint64)
    # near-cancelling c against a*b's neighbourhood is data-dependent; take
    # c close to -a for a quarter of the elements instead
    xs[2][q:2 * q] = ((xs[0][q:2 * q] + rng.integers(0, 3, q).astype(np.uint64)) % (1 << B)) ^ (1 << (e + m))
    return [x.astype(dt) for x in xs]


@pytest.mark.parametrize("e,m", FORMATS)
def test_chain2_all_op_pairs(e, m):
    a, b, c = _operands(e, m, NPAR, 13 * e + m)
    for mode in (0, 1):
        f = bfp.fmt(e, m, mode)
        pa, pb, pc = (bfp.pack(f, _dev(x)) for x in (a, b, c))
        for op1 in OPS:
            for op2 in OPS:
                want = oracle.chain2(op1, op2, e, m, mode, a, b, c, nthreads=8)
                pd = bfp.empty_bitslice(f, NPAR)
                bfp.bfp_chain2(op1, op2, f, pa, pb, pc, pd, NPAR)
                got = _host(pd)
                if not np.array_equal(got, oracle.pack(e, m, want)):
                    res = oracle.unpack(e, m, got, NPAR).astype(np.uint32)
                    bad = np.flatnonzero(res != want)
                    k = bad[0] if bad.size else -1
                    pytest.fail("(%d,%d) %s,%s mode %d: %d bad, e.g. a=%#x b=%#x c=%#x got=%#x want=%#x"
                                % (e, m, op1, op2, mode, bad.size, a[k], b[k], c[k], res[k], want[k]))
                # the same two ops launched separately: identical planes
                t = bfp.empty_bitslice(f, NPAR)
                bfp.bfp_binop(op1, f, pa, pb, t, NPAR)
                two = bfp.empty_bitslice(f, NPAR)
                bfp.bfp_binop(op2, f, t, pc, two, NPAR)
                assert torch.equal(two, pd), (op1, op2, mode)


@pytest.mark.parametrize("e,m", [(5, 10), (8, 7), (3, 1), (8, 23), (4, 3), (6, 15)])
def test_axpy_alphas(e, m):
    x, y, _ = _operands(e, m, NPAR, 31 * e + m)
    B = 1 + e + m
    emax = ((1 << e) - 1) << m
    one = ((1 << (e - 1)) - 1) << m
    alphas = [one, one | (1 << (e + m)), 0, 1 << (e + m), 1, emax, emax | 1, emax - 1, (emax - 1) | (1 << (e + m)),
              one + (1 << (m - 1)), (1 << B) - 1]
    for mode in (0, 1):
        f = bfp.fmt(e, m, mode)
        px, py = bfp.pack(f, _dev(x)), bfp.pack(f, _dev(y))
        for al in alphas:
            want = oracle.axpy(e, m, mode, al, x, y, nthreads=8)
            pd = bfp.empty_bitslice(f, NPAR)
            bfp.bfp_axpy(f, al, px, py, pd, NPAR)
            assert np.array_equal(_host(pd), oracle.pack(e, m, want)), (mode, hex(al))
        # upper pattern bits are ignored
        pd = bfp.empty_bitslice(f, NPAR)
        bfp.bfp_axpy(f, one | (0xFFFFFFFF << B) & 0xFFFFFFFF, px, py, pd, NPAR)
        assert np.array_equal(_host(pd), oracle.pack(e, m, oracle.axpy(e, m, mode, one, x, y, nthreads=8)))


def test_chain_lengths_and_aliasing():
    e, m = 5, 10
    f = bfp.fmt(e, m)
    for n in (1, 31, 32, 33, 2047, 64 * 32 + 5, 2048 * 32 + 7):
        a, b, c = _operands(e, m, n, n)
        want = oracle.chain2("mul", "add", e, m, 0, a, b, c)
        pa, pb, pc = (bfp.pack(f, _dev(v)) for v in (a, b, c))
        pd = bfp.empty_bitslice(f, n)
        bfp.bfp_chain2("mul", "add", f, pa, pb, pc, pd, n)
        assert np.array_equal(_host(pd), oracle.pack(e, m, want)), n
        bfp.bfp_chain2("mul", "add", f, pa, pb, pc, pc, n)  # d == c
        assert np.array_equal(_host(pc), oracle.pack(e, m, want)), ("d == c", n)
        bfp.bfp_chain2("sub", "mul", f, pa, pb, pa, pa, n)  # d == a, a read twice
        assert np.array_equal(_host(pa), oracle.pack(e, m, oracle.chain2("sub", "mul", e, m, 0, a, b, a))), n
    bfp.bfp_chain2("mul", "add", f, pa, pb, pc, pd, 0)  # no-op


def test_full_size_2_26_mul_add():
    """2^26 elements in (5,10) and (8,7): sampled outputs against the oracle,
    every output against the two separate launches."""
    n = 1 << 26
    for (e, m) in [(5, 10), (8, 7)]:
        f = bfp.fmt(e, m)
        a = inputs.scaled_normal(e, m, n, 2)
        b = inputs.scaled_normal(e, m, n, 3)
        c = inputs.scaled_normal(e, m, n, 4)
        pa, pb, pc = (bfp.pack(f, _dev(v)) for v in (a, b, c))
        pd = bfp.empty_bitslice(f, n)
        bfp.bfp_chain2("mul", "add", f, pa, pb, pc, pd, n)
        got = _host(bfp.unpack(f, pd, n)).astype(np.uint32)
        rng = np.random.default_rng(6)
        idx = np.concatenate([np.arange(4096), np.arange(n - 4096, n), rng.integers(0, n, 200000)])
        want = oracle.chain2("mul", "add", e, m, 0, a[idx], b[idx], c[idx], nthreads=8)
        assert np.array_equal(got[idx], want), (e, m)
        t = bfp.empty_bitslice(f, n)
        bfp.bfp_mul(f, pa, pb, t, n)
        bfp.bfp_add(f, t, pc, t, n)
        assert torch.equal(t, pd), (e, m)
        del pa, pb, pc, pd, t
        torch.cuda.synchronize()
