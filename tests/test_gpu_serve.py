"""Serving loop on the GPU: every result equals the oracle and equals the same
request run alone (bit for bit); admission keeps the arena within budget."""
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


def _pool_host(srv, pool, f_list):
    host = {}
    for (e, m) in f_list:
        a, b, n = pool[(e, m)]
        f = bfp.fmt(e, m)
        out = []
        for h in (a, b):
            t = torch.empty(n, dtype=bfp.container_dtype(f), device="cuda")
            srv.get(h, f, t)
            out.append(t.cpu().numpy())
        host[(e, m)] = out
    return host


def _result(srv, h, f, n):
    out = torch.empty(n, dtype=bfp.container_dtype(f), device="cuda")
    srv.get(h, f, out)
    return out.view(torch.int16 if out.element_size() == 2 else (torch.int32 if out.element_size() == 4
                                                                  else torch.uint8))


def test_mix_matches_oracle_and_alone():
    srv = serving.Server(2 << 30, 256)
    pool = serving.build_pool(srv, FMTS, N0, seed=5, device="cuda")
    host = _pool_host(srv, pool, FMTS)
    reqs = serving.request_stream(400, FMTS, seed=6, nmin_log2=0, nmax_log2=16, nmax=N0, ops=serving.ALL_OPS)
    res = serving.run(srv, pool, reqs, rate=None, rnd=0, keep_results=True)
    assert res["errors"] == 0
    st = srv.stats()
    assert st["completed"] == 400 and st["high_water"] <= st["budget"]
    for k, rid in enumerate(res["ids"]):
        op, (e, m), n = reqs[k]
        f = bfp.fmt(e, m)
        status, h, *_t = res["completions"][rid]
        out = torch.empty(n, dtype=bfp.container_dtype(f), device="cuda")
        srv.get(h, f, out)
        a, b = host[(e, m)]
        want = oracle.binop(op, e, m, 0, a[:n], b[:n])
        assert np.array_equal(out.cpu().numpy().astype(np.uint32), want), (k, reqs[k])
    # the same requests alone: identical result planes
    for k in range(0, 400, 10):
        op, (e, m), n = reqs[k]
        f = bfp.fmt(e, m)
        a, b, _n0 = pool[(e, m)]
        rid = srv.submit(op, f, a, b, n)
        srv.wait_idle()
        comp = [c for c in srv.poll() if c.req_id == rid]
        assert len(comp) == 1 and comp[0].status == 0
        alone = _result(srv, comp[0].result, f, n)
        mixed = _result(srv, res["completions"][res["ids"][k]][1], f, n)
        assert torch.equal(alone, mixed), (k, reqs[k])
        srv.free(comp[0].result)
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
    matches the oracle on 2048 sampled elements; every 15th request, run
    alone, gives the same result planes."""
    fmts = inputs.sweep_formats()
    n0 = 1 << 22
    srv = serving.Server(8 << 30, 256)
    pool = serving.build_pool(srv, fmts, n0, seed=21, device="cuda")
    host = _pool_host(srv, pool, fmts)
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
        out = torch.empty(n, dtype=bfp.container_dtype(f), device="cuda")
        srv.get(h, f, out)
        idx = np.sort(rng.choice(n, min(n, 2048), replace=False))
        got = out.cpu().numpy()[idx].astype(np.uint32)
        a, b = host[(e, m)]
        want = oracle.binop(op, e, m, 0, a[idx], b[idx])
        assert np.array_equal(got, want), (k, reqs[k])
    for k in range(0, 600, 15):
        op, (e, m), n = reqs[k]
        f = bfp.fmt(e, m)
        a, b, _n0 = pool[(e, m)]
        rid = srv.submit(op, f, a, b, n)
        srv.wait_idle()
        comp = [c for c in srv.poll() if c.req_id == rid]
        assert len(comp) == 1 and comp[0].status == 0
        assert torch.equal(_result(srv, comp[0].result, f, n),
                           _result(srv, res["completions"][res["ids"][k]][1], f, n)), (k, reqs[k])
        srv.free(comp[0].result)
    srv.close()
