"""Batched persistent launch: every vector of a mixed batch equals its
single-launch result and the oracle, bit for bit, on every graph replay."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1602_04716_amd import bfp, inputs, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bfp.lib()
    oracle.build()
    yield
    torch.cuda.synchronize()


def _mixed_specs(count, seed):
    rng = np.random.default_rng(seed)
    fmts = inputs.sweep_formats()
    edge_n = [1, 2, 31, 32, 33, 63, 64, 65, 2047, 2048, 2049, 64 * 32, 64 * 32 + 1, 1024 * 32, 1024 * 32 + 1,
              2048 * 32 + 7, 100000]
    specs = []
    for i in range(count):
        n = edge_n[i] if i < len(edge_n) else int(np.exp(rng.uniform(0, np.log(120000))))
        e, m = fmts[int(rng.integers(0, len(fmts)))] if i >= len(edge_n) else fmts[i % len(fmts)]
        op = workloads.ALL_OPS[int(rng.integers(0, len(workloads.ALL_OPS)))]
        specs.append((max(1, n), e, m, op, int(rng.integers(0, 2))))
    # every format x op x mode at least once
    for k, (e, m) in enumerate(fmts):
        for op in workloads.ALL_OPS:
            for r in (0, 1):
                specs.append((1000 + 37 * k, e, m, op, r))
    return specs


def _scrub(bt):
    for (a, b, c, n, f, op) in bt.tasks:
        c.view(torch.int32).fill_(0x25A5A5A5)


def _outputs(bt):
    torch.cuda.synchronize()
    return [c.view(torch.int32).clone() for (a, b, c, n, f, op) in bt.tasks]


def test_batch_mixed_all_variants():
    bt = workloads.build_batch(_mixed_specs(200, 11), seed=11, device="cuda", pool_log2=17)
    plan = bfp.BatchPlan(bt.tasks)
    info = plan.info()
    assert info["chunks"] >= len(bt.tasks) and info["grid"] > 0
    # per-vector launches first
    _scrub(bt)
    plan.run_per_vector()
    ref = _outputs(bt)
    # oracle on every element of every task
    for i, (n, e, m, op, rnd) in enumerate(bt.specs):
        a, b = bt.operands(i)
        want = oracle.binop(op, e, m, rnd, a, b)
        got = bfp.unpack(bt.tasks[i][4], ref[i].view(torch.uint32), n).cpu().numpy().astype(np.uint32)
        assert np.array_equal(got, want), (i, bt.specs[i])
    # graph replays, with eager work and scrubbing between them, and an eager run
    for rep in range(3):
        _scrub(bt)
        x = torch.arange(1 << 20, device="cuda").sum()  # unrelated eager work
        plan.run()
        out = _outputs(bt)
        assert int(x) == (1 << 20) * ((1 << 20) - 1) // 2
        for i in range(len(bt.tasks)):
            assert torch.equal(out[i], ref[i]), ("replay", rep, i, bt.specs[i])
    _scrub(bt)
    plan.run_eager()
    out = _outputs(bt)
    for i in range(len(bt.tasks)):
        assert torch.equal(out[i], ref[i]), ("eager", i)
    # launches that follow each other on one stream with no host step between
    # them: each starts from the counters the previous one left at zero
    _scrub(bt)
    plan.run()
    plan.run_eager()
    plan.run()
    plan.run_eager()
    out = _outputs(bt)
    for i in range(len(bt.tasks)):
        assert torch.equal(out[i], ref[i]), ("back to back", i)
    # the per-vector launches replayed from their captured graph
    for rep in range(2):
        _scrub(bt)
        plan.run_per_vector_graph()
        out = _outputs(bt)
        for i in range(len(bt.tasks)):
            assert torch.equal(out[i], ref[i]), ("per-vector graph", rep, i)
    plan.close()


def test_batch_4096_log_uniform():
    """4096 vectors, n log-uniform in [1024, 2^20], random sweep format and op:
    batched == per-vector on every word, oracle on a sample."""
    specs = inputs.batch_tasks(4096, seed=4)
    bt = workloads.build_batch(specs, seed=4, device="cuda", pool_log2=20)
    plan = bfp.BatchPlan(bt.tasks)
    _scrub(bt)
    plan.run_per_vector()
    ref = _outputs(bt)
    _scrub(bt)
    plan.run()
    out = _outputs(bt)
    for i in range(len(bt.tasks)):
        assert torch.equal(out[i], ref[i]), (i, bt.specs[i])
    rng = np.random.default_rng(44)
    for i in rng.choice(len(bt.tasks), 128, replace=False):
        n, e, m, op, rnd = bt.specs[i]
        a, b = bt.operands(i)
        want = oracle.binop(op, e, m, rnd, a, b, nthreads=8)
        got = bfp.unpack(bt.tasks[i][4], out[i].view(torch.uint32), n).cpu().numpy().astype(np.uint32)
        assert np.array_equal(got, want), (i, bt.specs[i])
    plan.close()


def test_batch_errors():
    f = bfp.fmt(5, 10)
    a = bfp.empty_bitslice(f, 100)
    with pytest.raises(bfp.BfpError):
        bfp.bfp_batch_plan_create([(a, a, a, 100, bfp.fmt(7, 3), "add")])
    with pytest.raises(bfp.BfpError):
        bfp.bfp_batch_plan_create([(a, a, a, 0, f, "add")])
    with pytest.raises(bfp.BfpError):
        bfp.bfp_batch_plan_create([(a, a, a, 100, f, 9)])
    with pytest.raises(bfp.BfpError):
        bfp.bfp_batch_plan_create([])
