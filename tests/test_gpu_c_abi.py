"""The library called from a plain C99 program (tests/abi_consumer.c: only
include/bfp.h and the HIP runtime's C API, linked against libbfp.so): pack,
a bitslice op and unpack, and the fused standard op, on ragged lengths;
every output against the oracle, and the two paths against each other (the
program exits non-zero if they differ)."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1602_04716_amd import inputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CONSUMER = os.path.join(ROOT, "tests", "abi_consumer")


@pytest.mark.parametrize("e,m,op,n", [(5, 10, "add", 100003), (8, 7, "mul", 65536 + 31), (4, 3, "div", 4097),
                                      (5, 2, "sub", 1), (11, 52, "mul", 20011)])
def test_c_program_matches_oracle(tmp_path, e, m, op, n):
    assert os.path.exists(CONSUMER), "tests/abi_consumer is built by paper_1602_04716_amd.build"
    a = inputs.sweep_operands(e, m, n, 71) if (e, m) != (11, 52) else None
    if a is None:
        rng = np.random.default_rng(71)  # uniform 64-bit patterns: both signs, NaN and Inf included
        a = np.frombuffer(rng.bytes(8 * n), dtype=np.uint64).copy()
        b = np.frombuffer(rng.bytes(8 * n), dtype=np.uint64).copy()
    else:
        b = inputs.sweep_operands(e, m, n, 72)
    dt = a.dtype
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as fp:
        fp.write(a.tobytes())
        fp.write(b.astype(dt).tobytes())
    print("abi_consumer", e, m, op, n, flush=True)
    r = subprocess.run([CONSUMER, "run", str(e), str(m), op, str(n), str(inp), str(out)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stderr)
    got = np.fromfile(out, dtype=dt)
    assert got.shape == (n,)
    want = oracle.binop(op, e, m, 0, a, b.astype(dt))
    assert np.array_equal(got.astype(np.uint64), np.asarray(want).astype(np.uint64)), (e, m, op, n)
