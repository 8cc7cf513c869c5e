"""Autotuner: installs a valid configuration that it measured, and results
stay bit-exact under every configuration it can choose."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1602_04716_amd import bfp, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bfp.lib()
    oracle.build()


@pytest.mark.parametrize("e,m,op", [(5, 10, "add"), (8, 23, "mul"), (3, 1, "sub"), (5, 10, "div")])
def test_autotune_installs_measured_best(e, m, op):
    f = bfp.fmt(e, m)
    old = bfp.bfp_launch_get(op, f)
    best, us = bfp.bfp_autotune(op, f, 1 << 20, 3, 2)
    assert us > 0
    cur = bfp.bfp_launch_get(op, f)
    assert (cur.words_per_lane, cur.block, cur.blocks_per_cu, cur.unroll) == \
        (best.words_per_lane, best.block, best.blocks_per_cu, best.unroll)
    assert best.words_per_lane in (1, 2) and best.block in (64, 128, 256, 512) and best.blocks_per_cu in (0, 4, 8)
    assert best.unroll in (1, 2)
    best1, _ = bfp.bfp_autotune(op, f, 1 << 18, 1, 1)
    assert best1.words_per_lane == 1
    bfp.bfp_launch_set(op, f, old.words_per_lane, old.block, old.blocks_per_cu, max(1, old.unroll))


@pytest.mark.parametrize("e,m", [(6, 7), (4, 3)])
def test_every_candidate_configuration_is_exact(e, m):
    """Every compiled launch variant (words per lane 1, 2 and, at most 10
    bits, 4; units per step 1 and 2; 4 block sizes; 3 grid depths) gives
    identical, oracle-exact results (ragged n)."""
    n = 300000 + 5
    a = inputs.sweep_operands(e, m, n, 1)
    b = inputs.sweep_operands(e, m, n, 2)
    f = bfp.fmt(e, m)
    pa, pb = bfp.pack(f, torch.from_numpy(a).cuda()), bfp.pack(f, torch.from_numpy(b).cuda())
    shapes = [(1, 1), (2, 1), (1, 2)] + ([(4, 1)] if 1 + e + m <= 10 else [])
    for op in ("add", "mul", "div"):
        want = oracle.binop(op, e, m, 0, a, b, nthreads=8)
        old = bfp.bfp_launch_get(op, f)
        for wpl, unroll in shapes:
            for blk in (64, 128, 256, 512):
                for bpc in (0, 4, 8):
                    bfp.bfp_launch_set(op, f, wpl, blk, bpc, unroll)
                    pc = bfp.empty_bitslice(f, n)
                    bfp.bfp_binop(op, f, pa, pb, pc, n)
                    got = bfp.unpack(f, pc, n).cpu().numpy().astype(np.uint32)
                    assert np.array_equal(got, want), (op, wpl, unroll, blk, bpc)
        with pytest.raises(bfp.BfpError):
            bfp.bfp_launch_set(op, f, 2, 256, 0, 2)      # two words and two units: not compiled
        if 1 + e + m > 10:
            with pytest.raises(bfp.BfpError):
                bfp.bfp_launch_set(op, f, 4, 256, 0)     # four words only up to 10 bits
        bfp.bfp_launch_set(op, f, old.words_per_lane, old.block, old.blocks_per_cu, max(1, old.unroll))


def test_autotune_errors():
    f = bfp.fmt(5, 10)
    with pytest.raises(bfp.BfpError):
        bfp.bfp_autotune("add", f, 0, 3, 1)
    with pytest.raises(bfp.BfpError):
        bfp.bfp_autotune("add", f, 1024, 0, 1)
    with pytest.raises(bfp.BfpError):
        bfp.bfp_autotune("add", bfp.fmt(7, 4), 1024, 3, 1)


def test_measure_copy_is_plausible():
    """The copy-bandwidth helper reports a rate between 1 TB/s and the 8 TB/s peak."""
    g = bfp.bfp_measure_copy(256 << 20, 5)
    assert 1000.0 < g < 8000.0, g


def test_measure_hbm_modes_are_plausible():
    """Read, write, copy and two-reads-one-write ceilings over 1 GiB streams:
    between 1 TB/s and the 8 TB/s peak (bytes moved per second, every
    stream counted)."""
    for mode in ("read", "write", "copy", "read2_write1"):
        r = bfp.bfp_measure_hbm(1 << 30, mode, 3)
        assert 1000.0 < r["GB/s"] < 8000.0, (mode, r)
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        assert r["grid"] // cus in (1, 2, 4, 8, 16, 32) and r["grid"] % cus == 0, r
        assert r["block"] in (256, 512, 1024) and r["in_flight"] in (1, 2, 4, 8), r
        assert r["block"] == 256 or r["grid"] // cus <= 2, r
    with pytest.raises(bfp.BfpError):
        bfp.bfp_measure_hbm(1 << 30, "copy", 0)


def test_flush_llc_runs():
    bfp.bfp_flush_llc(1 << 28)
    bfp.bfp_flush_llc(1 << 30)
    torch.cuda.synchronize()
    with pytest.raises(bfp.BfpError):
        bfp.bfp_flush_llc(100)


def test_wave_clock_lasts_longer_with_more_iterations():
    s = torch.cuda.current_stream()
    times = {}
    for iters in (20000, 80000):
        bfp.bfp_wave_clock(iters, s)  # warm
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        bfp.bfp_wave_clock(iters, s)
        e1.record(s)
        torch.cuda.synchronize()
        times[iters] = e0.elapsed_time(e1)
    # a dependent chain: four times the iterations takes clearly longer
    assert times[80000] > 2.5 * times[20000], times
    with pytest.raises(bfp.BfpError):
        bfp.bfp_wave_clock(0)


def test_chain_and_int_autotune_install_and_stay_exact():
    f = bfp.fmt(5, 10)
    old = bfp.bfp_chain_launch_get("mul", "add", f)
    best, us = bfp.bfp_autotune_chain("mul", "add", f, 1 << 20, 2)
    cur = bfp.bfp_chain_launch_get("mul", "add", f)
    assert us > 0 and (cur.block, cur.blocks_per_cu) == (best.block, best.blocks_per_cu)
    n = 100003
    a, b, c = (inputs.sweep_operands(5, 10, n, s) for s in (1, 2, 3))
    pa, pb, pc = (bfp.pack(f, torch.from_numpy(x).cuda()) for x in (a, b, c))
    want = oracle.binop("add", 5, 10, 0, oracle.binop("mul", 5, 10, 0, a, b), c)
    for blk in (64, 512):
        for bpc in (0, 8):
            bfp.bfp_chain_launch_set("mul", "add", f, blk, bpc)
            pd = bfp.empty_bitslice(f, n)
            bfp.bfp_chain2("mul", "add", f, pa, pb, pc, pd, n)
            assert np.array_equal(bfp.unpack(f, pd, n).cpu().numpy().astype(np.uint32), want), (blk, bpc)
    bfp.bfp_chain_launch_set("mul", "add", f, old.block, old.blocks_per_cu)
    k = 13
    oi = bfp.bfp_int_launch_get("mul", k, "sats")
    best, us = bfp.bfp_autotune_int("mul", k, "sats", 1 << 20, 2)
    assert us > 0 and best.words_per_lane == oi.words_per_lane
    rng = np.random.default_rng(5)
    x = rng.integers(0, 1 << k, n).astype(np.uint16)
    y = rng.integers(0, 1 << k, n).astype(np.uint16)
    px, py = bfp.int_pack(k, torch.from_numpy(x).cuda()), bfp.int_pack(k, torch.from_numpy(y).cuda())
    want = oracle.int_binop("mul", k, "sats", x, y)
    for blk in (64, 512):
        for bpc in (0, 8):
            bfp.bfp_int_launch_set("mul", k, "sats", blk, bpc)
            pz = bfp.int_empty_bitslice(k, n)
            bfp.bfp_int_binop("mul", k, "sats", px, py, pz, n)
            assert np.array_equal(bfp.int_unpack(k, pz, n).cpu().numpy().astype(np.uint32), want), (blk, bpc)
    bfp.bfp_int_launch_set("mul", k, "sats", oi.block, oi.blocks_per_cu)
