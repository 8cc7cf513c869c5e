"""Device-resident workloads built from the seeded input recipes.

``build_batch`` turns a list of (n, e, m, op[, round]) task specs into
bitslice operands on the device: for every format it draws a pool of
standard-layout operands with ``inputs.sweep_operands`` and packs, for each
task, its own copy of a random slice of the pool (so every task reads
distinct memory).  It returns the task tuples that ``bfp.BatchPlan`` takes and
the host-side pools and offsets that a checker needs.
"""
from __future__ import annotations

import numpy as np

from . import bfp, inputs

OPS = ("add", "sub", "mul")           # the op mix of the batched measurement
ALL_OPS = ("add", "sub", "mul", "div")


class Batch:
    def __init__(self):
        self.tasks = []        # (a, b, c, n, fmt, op) for BatchPlan
        self.specs = []        # (n, e, m, op, round)
        self.offsets = []      # (off_a, off_b) into the format's pools
        self.pools = {}        # (e, m) -> (pool_a, pool_b) host arrays

    def operands(self, i):
        """Host standard-layout operands of task i."""
        n, e, m, op, rnd = self.specs[i]
        pa, pb = self.pools[(e, m)]
        oa, ob = self.offsets[i]
        return pa[oa:oa + n], pb[ob:ob + n]

    def bytes_moved(self):
        """Algorithmic bytes of one pass: 2 operands in, 1 result out."""
        return sum(3 * (1 + e + m) / 8 * n for (n, e, m, op, rnd) in self.specs)

    def elements(self):
        return sum(s[0] for s in self.specs)


def build_batch(specs, seed: int, device, pool_log2: int = 20) -> Batch:
    import torch
    rng = np.random.default_rng(seed)
    pool_n = 1 << pool_log2
    bt = Batch()
    dev_pools = {}
    fmts = sorted({(s[1], s[2]) for s in specs})
    for i, (e, m) in enumerate(fmts):
        pa = inputs.sweep_operands(e, m, pool_n, seed * 1000 + 2 * i)
        pb = inputs.sweep_operands(e, m, pool_n, seed * 1000 + 2 * i + 1)
        bt.pools[(e, m)] = (pa, pb)
        dev_pools[(e, m)] = (torch.from_numpy(pa).to(device), torch.from_numpy(pb).to(device))
    for s in specs:
        n, e, m, op = s[:4]
        rnd = s[4] if len(s) > 4 else bfp.BFP_RNE
        if n > pool_n:
            raise ValueError("task longer than the operand pool")
        f = bfp.fmt(e, m, rnd)
        da, db = dev_pools[(e, m)]
        oa = int(rng.integers(0, (pool_n - n) // 16 + 1)) * 16
        ob = int(rng.integers(0, (pool_n - n) // 16 + 1)) * 16
        a = bfp.empty_bitslice(f, n, device)
        b = bfp.empty_bitslice(f, n, device)
        c = bfp.empty_bitslice(f, n, device)
        bfp.bfp_pack(f, da[oa:oa + n], a, n)
        bfp.bfp_pack(f, db[ob:ob + n], b, n)
        bt.tasks.append((a, b, c, n, f, op))
        bt.specs.append((n, e, m, op, rnd))
        bt.offsets.append((oa, ob))
    return bt
