"""Serving loop on the GPU: every result equals the oracle computed from the
host data that was put, and equals the same request run alone (bit for bit);
ticks overlap on the device; operands freed while in use stay intact until
their requests complete; admission keeps the arena within budget."""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1602_04716_amd import bfp, inputs, serving

pytestmark = pytest.mark.gpu

FMTS = [(5, 10), (8, 7), (5, 2), (3, 1), (8, 23), (4, 3), (6, 15), (3, 23)]
N0 = 50000 + 7


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bfp.lib()
    oracle.build()


def _operands(host, em, idx):
    """Host values of both pool operands of format em at element indices idx."""
    xa, xb = host[em]
    return xa[idx % len(xa)], xb[idx % len(xb)]


def _unpacked(srv, h, f, n):
    out = torch.empty(n, dtype=bfp.container_dtype(f), device="cuda")
    srv.get(h, f, out)
    return out


def _as_u32(t):
    return t.cpu().numpy().astype(np.uint32)


def _whole_planes(srv, h, f):
    """Every element slot of a resident result's planes, padding included:
    unpack of 32 * G_pad elements over the result's own memory (the stride
    of 32 * G_pad elements is G_pad again)."""
    ptr, n = srv.view(h)
    gpad = bfp.bfp_plane_stride_words(n)
    assert bfp.bfp_plane_stride_words(32 * gpad) == gpad
    out = torch.empty(32 * gpad, dtype=bfp.container_dtype(f), device="cuda")
    bfp.bfp_unpack(f, ptr, out, 32 * gpad)
    torch.cuda.synchronize()
    return _as_u32(out), n


def _check_alone(srv, pool, reqs, res, ks):
    """Requests ks run again, each alone in its own tick: identical planes."""
    for k in ks:
        op, (e, m), n = reqs[k]
        f = bfp.fmt(e, m)
        a, b, _n0 = pool[(e, m)]
        rid = srv.submit(op, f, a, b, n)
        srv.wait_idle()
        comp = [c for c in srv.poll() if c.req_id == rid]
        assert len(comp) == 1 and comp[0].status == 0
        alone = _unpacked(srv, comp[0].result, f, n)
        mixed = _unpacked(srv, res["completions"][res["ids"][k]][1], f, n)
        assert torch.equal(alone, mixed), (k, reqs[k])
        srv.free(comp[0].result)


def test_mix_matches_oracle_and_alone():
    srv = serving.Server(2 << 30, 256)
    host = {}
    pool = serving.build_pool(srv, FMTS, N0, seed=5, device="cuda", host_out=host)
    reqs = serving.request_stream(400, FMTS, seed=6, nmin_log2=0, nmax_log2=16, nmax=N0, ops=serving.ALL_OPS)
    res = serving.run(srv, pool, reqs, rate=None, rnd=0, keep_results=True)
    assert res["errors"] == 0
    st = srv.stats()
    assert st["completed"] == 400 and st["high_water"] <= st["budget"]
    for k, rid in enumerate(res["ids"]):
        op, (e, m), n = reqs[k]
        f = bfp.fmt(e, m)
        status, h, *_t = res["completions"][rid]
        a, b = _operands(host, (e, m), np.arange(n))
        want = oracle.binop(op, e, m, 0, a, b)
        planes, n_res = _whole_planes(srv, h, f)
        assert n_res == n
        assert np.array_equal(planes[:n], want), (k, reqs[k])
        assert not planes[n:].any(), ("padding", k, reqs[k])
    _check_alone(srv, pool, reqs, res, range(0, 400, 10))
    srv.close()


def test_overlapping_ticks_bit_exact():
    """Continuous batching on the device: a long tick of (8,23) products is
    running when a second group of mixed requests arrives (native arrival
    schedule, 300 us later); the second group launches on the other stream
    before the first completes.  Every result matches the oracle on sampled
    elements from the host data, and a sample equals the request run alone."""
    n0 = 1 << 22
    fmts = [(8, 23), (5, 10), (8, 7), (4, 3), (3, 1)]
    srv = serving.Server(8 << 30, 1024)
    host = {}
    pool = serving.build_pool(srv, fmts, n0, seed=31, device="cuda", host_out=host)
    group_a = [("mul", (8, 23), n0 - 5 * k) for k in range(96)]
    group_b = serving.request_stream(64, fmts, seed=32, nmin_log2=10, nmax_log2=20, ops=serving.ALL_OPS)
    reqs = group_a + group_b
    sched = []
    for k, (op, (e, m), n) in enumerate(reqs):
        a, b, _n = pool[(e, m)]
        sched.append((op, bfp.fmt(e, m), a, b, n, 0 if k < len(group_a) else 300_000))
    first = srv.replay(sched)
    srv.wait_idle(120000)
    comp = {}
    for c in srv.poll():
        comp[c.req_id] = c
    ids = list(range(first, first + len(reqs)))
    assert sorted(comp) == ids and all(comp[i].status == 0 for i in ids)
    st = srv.stats()
    assert st["max_inflight_ticks"] >= 2, st
    done_a = max(comp[i].t_done_ns for i in ids[:len(group_a)])
    launch_b = min(comp[i].t_launch_ns for i in ids[len(group_a):])
    assert launch_b < done_a, "the second group did not start while the first tick ran"
    rng = np.random.default_rng(33)
    res = {"ids": ids, "completions": {i: (comp[i].status, comp[i].result) for i in ids}}
    for k, i in enumerate(ids):
        op, (e, m), n = reqs[k]
        f = bfp.fmt(e, m)
        got = _as_u32(_unpacked(srv, comp[i].result, f, n))
        idx = np.sort(rng.choice(n, min(n, 1024), replace=False))
        a, b = _operands(host, (e, m), idx)
        assert np.array_equal(got[idx], oracle.binop(op, e, m, 0, a, b)), (k, reqs[k])
    _check_alone(srv, pool, reqs, res, list(range(0, 96, 24)) + list(range(96, 160, 8)))
    srv.close()


def test_prefix_requests_across_the_stride_skew():
    """Requests on a prefix of longer operands where the result's plane
    stride exceeds the operands' (the 8 KiB skew makes the stride rule
    non-monotonic: stride(65000) = 2304 > stride(66000) = 2112 words).  The
    operands sit at the end of a snug arena.  Every element matches the
    oracle and every padding bit of the result is zero."""
    na = 66000
    assert bfp.bfp_plane_stride_words(65000) > bfp.bfp_plane_stride_words(na)
    fmts = [(5, 10), (8, 23), (3, 1), (6, 7)]
    ns = [65000, 64001, 65535, 63489, 1]
    results = sum(bfp.bfp_bitslice_bytes(bfp.fmt(e, m), n) for (e, m) in fmts for n in ns) * 8
    operands = sum(2 * bfp.bfp_bitslice_bytes(bfp.fmt(e, m), na) for (e, m) in fmts)
    n_fill = 32 * (-(-results // 64))                    # (5,10): 64 bytes per plane word
    fill_bytes = bfp.bfp_bitslice_bytes(bfp.fmt(5, 10), n_fill)
    assert fill_bytes >= results
    srv = serving.Server(fill_bytes + operands, 4096)     # operands end exactly at the arena's end
    hfill = srv.put(bfp.fmt(5, 10), torch.zeros(n_fill, dtype=torch.uint16, device="cuda"))
    host = {}
    pool = {}
    for i, (e, m) in enumerate(fmts):
        f = bfp.fmt(e, m)
        xa = inputs.sweep_operands(e, m, na, 40 + 2 * i)
        xb = inputs.sweep_operands(e, m, na, 41 + 2 * i)
        pool[(e, m)] = (srv.put(f, torch.from_numpy(xa).cuda()), srv.put(f, torch.from_numpy(xb).cuda()), na)
        host[(e, m)] = (xa, xb)
    assert srv.stats()["used"] == srv.stats()["budget"]
    srv.free(hfill)                                        # results land below the operands
    reqs = [(op, em, n, rnd) for em in fmts for n in ns for op in serving.ALL_OPS for rnd in (0, 1)]
    ids = []
    for (op, (e, m), n, rnd) in reqs:
        a, b, _n = pool[(e, m)]
        ids.append(srv.submit(op, bfp.fmt(e, m, rnd), a, b, n))
    srv.wait_idle(60000)
    comp = {c.req_id: c for c in srv.poll()}
    for (op, (e, m), n, rnd), rid in zip(reqs, ids):
        c = comp[rid]
        assert c.status == 0
        planes, n_res = _whole_planes(srv, c.result, bfp.fmt(e, m))
        a, b = host[(e, m)]
        want = oracle.binop(op, e, m, rnd, a[:n], b[:n])
        assert n_res == n and np.array_equal(planes[:n], want), (op, e, m, n, rnd)
        assert not planes[n:].any(), ("padding", op, e, m, n, rnd)
        srv.free(c.result)
    srv.close()


def test_free_while_running_keeps_operand_intact():
    """An operand freed right after its requests are submitted: the next put
    must not reuse its memory while they run, so every result still matches
    the oracle on the original data."""
    n0 = 1 << 22
    e, m = 8, 23
    f = bfp.fmt(e, m)
    srv = serving.Server(3 << 30, 256)
    xa = inputs.sweep_operands(e, m, n0, 51)
    xb = inputs.sweep_operands(e, m, n0, 52)
    ha = srv.put(f, torch.from_numpy(xa).cuda())
    hb = srv.put(f, torch.from_numpy(xb).cuda())
    first = srv.replay([("mul", f, ha, hb, n0 - 7 * k, 0) for k in range(96)])
    ids = list(range(first, first + 96))
    srv.free(ha)                                   # retired while its requests queue or run
    with pytest.raises(bfp.BfpError):
        srv.submit("add", f, ha, hb, 10)           # the handle is gone at once
    junk = torch.from_numpy(inputs.sweep_operands(e, m, n0, 53)).cuda()
    hj = srv.put(f, junk)                          # would have landed on a's range
    srv.wait_idle(60000)
    comp = {c.req_id: c for c in srv.poll()}
    rng = np.random.default_rng(54)
    for k, rid in enumerate(ids):
        n = n0 - 7 * k
        assert comp[rid].status == 0
        got = _as_u32(_unpacked(srv, comp[rid].result, f, n))
        idx = np.sort(rng.choice(n, 4096, replace=False))
        assert np.array_equal(got[idx], oracle.binop("mul", e, m, 0, xa[idx], xb[idx])), k
        srv.free(comp[rid].result)
    assert srv.stats()["deferred_frees"] == 1
    srv.free(hj)
    srv.free(hb)
    assert srv.stats()["used"] == 0
    srv.close()


def test_cancel_timeout_and_handle_reuse():
    srv = serving.Server(1 << 30, 1)                # one slot: requests queue behind each other
    f = bfp.fmt(5, 10)
    n = 1 << 20
    x = inputs.sweep_operands(5, 10, n, 61)
    h = srv.put(f, torch.from_numpy(x).cuda())
    ids = [srv.submit("mul", f, h, h, n) for _ in range(6)]
    srv.cancel(ids[5])
    with pytest.raises(bfp.BfpError):
        srv.cancel(ids[5])                          # already withdrawn
    srv.wait_idle(60000)
    comp = {c.req_id: c for c in srv.poll()}
    assert comp[ids[5]].status == bfp.BFP_E_CANCELLED and comp[ids[5]].result == 0
    want = oracle.binop("mul", 5, 10, 0, x, x)
    for rid in ids[:5]:
        assert comp[rid].status == 0
        assert np.array_equal(_as_u32(_unpacked(srv, comp[rid].result, f, n)), want)
        srv.free(comp[rid].result)
    # queue timeout: with one slot and a 1 us limit, most of a burst expires
    srv.set_queue_timeout(1000)
    burst = [srv.submit("add", f, h, h, n) for _ in range(20)]
    srv.wait_idle(60000)
    srv.set_queue_timeout(0)
    comp = {c.req_id: c for c in srv.poll()}
    sts = [comp[r].status for r in burst]
    assert set(sts) <= {0, bfp.BFP_E_TIMEOUT} and sts.count(bfp.BFP_E_TIMEOUT) >= 10
    for r in burst:
        if comp[r].status == 0:
            srv.free(comp[r].result)
    assert srv.stats()["timed_out"] == sts.count(bfp.BFP_E_TIMEOUT)
    # handles: a freed handle stays invalid after its slot is reused (free
    # slots are reused oldest first, so cycle through all of them)
    h2 = srv.put(f, torch.from_numpy(x[:1000]).cuda())
    srv.free(h2)
    reused = []
    for _ in range(200):
        hx = srv.put(f, torch.from_numpy(x[:1000]).cuda())
        if (hx & 0xFFFFFFFF) == (h2 & 0xFFFFFFFF):
            reused.append(hx)
            with pytest.raises(bfp.BfpError):
                srv.submit("add", f, h2, hx, 10)     # the old handle, same slot
            srv.submit("add", f, hx, hx, 10)          # the new one works
        srv.free(hx)
    assert reused and all(hx != h2 for hx in reused)
    srv.wait_idle(60000)
    for c in srv.poll():
        assert c.status == 0
        srv.free(c.result)
    slots = srv.stats()["table_slots"]
    for _ in range(300):                           # steady state: the table does not grow
        srv.free(srv.put(f, torch.from_numpy(x[:1000]).cuda()))
    st = srv.stats()
    assert st["table_slots"] == slots and st["live_vectors"] == 1, st
    srv.close()


def test_budget_defers_and_never_exceeds():
    f_list = [(5, 10), (8, 7)]
    probe = serving.Server(1 << 30, 8)
    pool = serving.build_pool(probe, f_list, N0, seed=7, device="cuda")
    pool_bytes = probe.stats()["used"]
    probe.close()
    biggest = max(bfp.bfp_bitslice_bytes(bfp.fmt(e, m), N0) for (e, m) in f_list)
    budget = pool_bytes + 3 * biggest + 4096
    srv = serving.Server(budget, 64)
    pool = serving.build_pool(srv, f_list, N0, seed=7, device="cuda")
    reqs = [(op, fm, N0 - 3 * k) for k, (op, fm) in enumerate([(o, f) for o in serving.ALL_OPS for f in f_list] * 10)]
    res = serving.run(srv, pool, reqs, rate=None)
    st = srv.stats()
    assert res["errors"] == 0 and st["completed"] == len(reqs)
    assert st["high_water"] <= st["budget"] and st["deferred_budget"] > 0
    srv.close()


def test_server_errors():
    srv = serving.Server(64 << 20, 4)
    f = bfp.fmt(5, 10)
    x = torch.from_numpy(inputs.sweep_operands(5, 10, 1000, 1)).cuda()
    h = srv.put(f, x)
    with pytest.raises(bfp.BfpError):
        srv.submit("add", f, h, 9999, 10)            # unknown handle
    with pytest.raises(bfp.BfpError):
        srv.submit("add", bfp.fmt(8, 7), h, h, 10)   # format mismatch
    with pytest.raises(bfp.BfpError):
        srv.submit("add", f, h, h, 1001)             # longer than the operand
    with pytest.raises(bfp.BfpError):
        srv.submit(7, f, h, h, 10)
    big = torch.zeros(1 << 26, dtype=torch.uint16, device="cuda")
    with pytest.raises(bfp.BfpError):
        srv.put(f, big)                              # 128 MiB > 64 MiB budget
    srv.free(h)
    with pytest.raises(bfp.BfpError):
        srv.free(h)
    srv.close()


def test_native_replay_poisson_autofree():
    srv = serving.Server(1 << 30, 128)
    pool = serving.build_pool(srv, FMTS, N0, seed=9, device="cuda")
    pool_bytes = srv.stats()["used"]
    reqs = serving.request_stream(2000, FMTS, seed=10, nmin_log2=5, nmax_log2=15.5, nmax=N0)
    sat = serving.run_native(srv, pool, reqs)
    assert sat["errors"] == 0 and sat["requests"] == 2000
    r = serving.run_native(srv, pool, reqs, rate=0.5 * sat["requests_per_s"], seed=3, skip=100)
    assert r["errors"] == 0 and r["requests"] == 1900 and r["p99_us"] >= r["p50_us"] > 0
    srv.wait_idle()
    st = srv.stats()
    assert st["used"] == pool_bytes  # every result went back to the arena
    assert st["max_inflight_ticks"] >= 1 and st["high_water"] <= st["budget"]
    with pytest.raises(bfp.BfpError):  # arrivals out of order are rejected before submission
        srv.replay([("add", bfp.fmt(5, 10), pool[(5, 10)][0], pool[(5, 10)][1], 10, 1000),
                    ("add", bfp.fmt(5, 10), pool[(5, 10)][0], pool[(5, 10)][1], 10, 0)])
    assert srv.stats()["submitted"] == st["submitted"]
    srv.close()


def test_full_size_mix_all_sweep_formats():
    """The serving workload at its full shape: every sweep format resident at
    2^22 elements, 600 requests of length log-uniform in 2^10..2^22 over
    add/sub/mul/div, all submitted at once under the budget.  Each result
    matches the oracle, computed from the host data put, on 2048 sampled
    elements; every 15th request, run alone, gives the same result planes."""
    fmts = inputs.sweep_formats()
    n0 = 1 << 22
    srv = serving.Server(8 << 30, 256)
    host = {}
    pool = serving.build_pool(srv, fmts, n0, seed=21, device="cuda", host_out=host)
    reqs = serving.request_stream(600, fmts, seed=22, nmin_log2=10, nmax_log2=22, nmax=n0, ops=serving.ALL_OPS)
    res = serving.run(srv, pool, reqs, rate=None, rnd=0, keep_results=True)
    assert res["errors"] == 0
    st = srv.stats()
    assert st["completed"] == 600 and st["high_water"] <= st["budget"]
    rng = np.random.default_rng(23)
    for k, rid in enumerate(res["ids"]):
        op, (e, m), n = reqs[k]
        f = bfp.fmt(e, m)
        status, h, *_t = res["completions"][rid]
        assert status == 0
        got = _as_u32(_unpacked(srv, h, f, n))
        idx = np.sort(rng.choice(n, min(n, 2048), replace=False))
        a, b = _operands(host, (e, m), idx)
        assert np.array_equal(got[idx], oracle.binop(op, e, m, 0, a, b)), (k, reqs[k])
    _check_alone(srv, pool, reqs, res, range(0, 600, 15))
    srv.close()
