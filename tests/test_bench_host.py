"""Host-side checks of bench.py's contract, no GPU: it measures one GPU and
refuses more, its labels name the device kernels the counter summaries are
keyed by, and the committed counter traffic of the dominant kernel belongs
to the current library sources (otherwise the bench line would report it
as null)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, capture_output=True,
                          text=True, timeout=300, env=env, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_a_distributed_launch_is_refused():
    r = _run([], env=dict(os.environ, WORLD_SIZE="2", RANK="0", LOCAL_RANK="0"))
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_labels_name_the_device_kernels():
    assert bench.device_kernel("pack(5,10)") == "bfp::k_pack<2>"
    assert bench.device_kernel("unpack(8,7)") == "bfp::k_unpack<2>"
    assert bench.device_kernel("add(5,10)") == "bfp::k_binop<5, 10, false, 0, 2, 1>"
    assert bench.device_kernel("sub(8,7)") == "bfp::k_binop<8, 7, false, 0, 2, 1>"
    assert bench.device_kernel("mul(5,10)") == "bfp::k_binop<5, 10, false, 1, 2, 1>"


def test_committed_traffic_is_current():
    """The stored calibrated bytes per launch of k_unpack<2> (2^26 elements,
    2-byte containers, 16 planes: 2^26 x (2 + 2) bytes algorithmic) and of the
    batch kernel were taken with the library sources as they are now."""
    t = bench.committed_traffic("bfp::k_unpack<2>")
    assert t is not None, "profiles/*.traffic.txt were taken with other kernel sources"
    alg = (1 << 26) * 4
    assert abs(t - alg) / alg < 0.01
    assert bench.committed_traffic("bfp::k_batch<0>") is not None
