"""The allocation-free batched launch (bfp_batch_run_noalloc) against the
batch plan path (bfp_batch_plan_create + bfp_batch_run): identical result
planes, bit for bit, on two calls in a row (the second smaller), plus its
error reporting.  Calls go through the C ABI."""
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


def _specs(count, seed, nmax):
    rng = np.random.default_rng(seed)
    fmts = inputs.sweep_formats()
    specs = []
    for i in range(count):
        n = int(np.exp(rng.uniform(0, np.log(nmax))))
        e, m = fmts[int(rng.integers(0, len(fmts)))]
        op = workloads.ALL_OPS[int(rng.integers(0, len(workloads.ALL_OPS)))]
        specs.append((max(1, n), e, m, op, int(rng.integers(0, 2))))
    for k, (e, m) in enumerate(fmts):          # every class kernel gets work
        for op in workloads.ALL_OPS:
            specs.append((700 + 37 * k, e, m, op, k % 2))
    return specs


def _scrub(bt):
    for (a, b, c, n, f, op) in bt.tasks:
        c.view(torch.int32).fill_(0x25A5A5A5)


def _outputs(bt):
    torch.cuda.synchronize()
    return [c.view(torch.int32).clone() for (a, b, c, n, f, op) in bt.tasks]


def _plan_outputs(bt):
    plan = bfp.BatchPlan(bt.tasks)
    _scrub(bt)
    plan.run()
    out = _outputs(bt)
    plan.close()
    return out


def _noalloc_outputs(bt):
    table = bfp.task_table(bt.tasks)
    status = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    _scrub(bt)
    bfp.bfp_batch_run_noalloc(table, len(bt.tasks), status)
    out = _outputs(bt)
    assert int(status.item()) == bfp.BFP_OK
    return out


def test_noalloc_matches_plan_two_calls():
    big = workloads.build_batch(_specs(600, 71, 300000), seed=71, device="cuda", pool_log2=19)
    small = workloads.build_batch(_specs(90, 72, 5000), seed=72, device="cuda", pool_log2=13)
    for bt in (big, small):
        want = _plan_outputs(bt)
        got = _noalloc_outputs(bt)
        for i in range(len(bt.tasks)):
            assert torch.equal(got[i], want[i]), (i, bt.specs[i])
        rng = np.random.default_rng(73)
        for i in rng.choice(len(bt.tasks), 40, replace=False):
            n, e, m, op, rnd = bt.specs[i]
            a, b = bt.operands(i)
            res = bfp.unpack(bt.tasks[i][4], got[i].view(torch.uint32), n).cpu().numpy().astype(np.uint32)
            assert np.array_equal(res, oracle.binop(op, e, m, rnd, a, b)), (i, bt.specs[i])


def test_noalloc_errors():
    f = bfp.fmt(5, 10)
    a = bfp.empty_bitslice(f, 100)
    c = bfp.empty_bitslice(f, 100)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    good = (a, a, c, 100, f, "add")
    # an invalid task anywhere: its error is reported and nothing is computed
    for bad, code in (((a, a, c, 100, bfp.fmt(7, 3), "add"), bfp.BFP_E_FORMAT),
                      ((a, a, c, 100, bfp.fmt(11, 52), "add"), bfp.BFP_E_FORMAT),
                      ((a, a, c, 0, f, "add"), bfp.BFP_E_ARG),
                      ((a, a, c, 100, f, 9), bfp.BFP_E_OP),
                      ((a, 0, c, 100, f, "add"), bfp.BFP_E_NULL)):
        c.view(torch.int32).fill_(0x5A5A5A5A)
        table = bfp.task_table([good, bad, good])
        bfp.bfp_batch_run_noalloc(table, 3, status)
        torch.cuda.synchronize()
        assert int(status.item()) == code, (bad, int(status.item()))
        assert bool((c.view(torch.int32) == 0x5A5A5A5A).all())
    table = bfp.task_table([good])
    with pytest.raises(bfp.BfpError):
        bfp.bfp_batch_run_noalloc(table, 0, status)
    with pytest.raises(bfp.BfpError):
        bfp.bfp_batch_run_noalloc(table, 16385, status)
    with pytest.raises(bfp.BfpError):
        bfp.bfp_batch_run_noalloc(0, 1, status)
    # a valid table after the failures runs normally
    bfp.bfp_batch_run_noalloc(table, 1, status)
    torch.cuda.synchronize()
    assert int(status.item()) == bfp.BFP_OK
