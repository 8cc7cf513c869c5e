"""CPU builds under sanitizers: the oracle and the host build of the circuits
and scheduler with AddressSanitizer + UndefinedBehaviorSanitizer (drivers in
tests/sanitize/), and the serving scheduler's worker loop raced by submitter
and poller threads under ThreadSanitizer.  Host code only: no GPU code is
built here."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1602_04716_amd", "csrc")
INC = os.path.join(ROOT, "include")
SAN = os.path.join(ROOT, "tests", "sanitize")


def _run(cmd, **kw):
    return subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)


def _supported(flag, tmp_path):
    src = tmp_path / "probe.cpp"
    src.write_text("int main() { return 0; }\n")
    r = _run(["g++", flag, str(src), "-o", str(tmp_path / "probe")])
    return r.returncode == 0 and _run([str(tmp_path / "probe")]).returncode == 0


def test_asan_ubsan_oracle_and_host_circuits(tmp_path):
    flags = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
    if not _supported(flags[0], tmp_path):
        pytest.skip("address/undefined sanitizer runtime not available")
    o_obj = tmp_path / "oracle.o"
    r = _run(["gcc", "-std=c11", "-c", os.path.join(ROOT, "oracle", "bfp_oracle.c"), "-o", str(o_obj)] + flags)
    assert r.returncode == 0, r.stdout
    exe = tmp_path / "host_check"
    # a representative subset of the circuits keeps the instrumented build to
    # about a minute: 8-bit, 16-bit and 32-bit formats, every op class, the
    # widest format, and integer widths around byte and word boundaries
    subset = ["-DBFP_SIM_FORMATS(X)=X(3,1) X(5,2) X(4,3) X(5,10) X(8,7) X(6,15) X(8,23)",
              "-DBFP_SIM_WIDE_FORMATS(X)=X(11,52)",
              "-DBFP_SIM_INT_K(X)=X(1) X(5) X(8) X(9) X(16) X(17) X(31) X(32)"]
    r = _run(["g++", "-std=c++17", "-I" + INC, "-I" + CSRC, os.path.join(SAN, "host_check.cpp"),
              os.path.join(CSRC, "bfp_host_sim.cpp"), str(o_obj), "-o", str(exe), "-pthread"] + subset + flags)
    assert r.returncode == 0, r.stdout
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = _run([str(exe)], env=env, timeout=600)
    assert r.returncode == 0 and "host_check ok" in r.stdout, r.stdout[-4000:]
    # 7 formats x 4 ops x 2 modes x 2 word widths, binary64 x 4 x 2, 8 widths x 9 integer ops
    assert "host_check ok: 120 format/op/mode/word cases, 72 integer cases" in r.stdout, r.stdout


def test_tsan_scheduler_worker_loop(tmp_path):
    flags = ["-fsanitize=thread", "-g", "-O1"]
    if not _supported(flags[0], tmp_path):
        pytest.skip("thread sanitizer runtime not available")
    exe = tmp_path / "sched_tsan"
    r = _run(["g++", "-std=c++17", "-I" + INC, "-I" + CSRC, os.path.join(SAN, "sched_tsan.cpp"), "-o", str(exe),
              "-pthread"] + flags)
    assert r.returncode == 0, r.stdout
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")
    r = _run([str(exe)], env=env, timeout=600)
    assert r.returncode == 0 and "sched_tsan ok" in r.stdout, r.stdout[-4000:]
