"""Build libbfp.so (HIP kernels for gfx950 + C ABI), the host-side circuit
simulator used by the CPU tests, and the plain C program the tests use to
call the library from C.

    python -m paper_1602_04716_amd.build [--force] [-j N]

Every ``csrc/*.hip`` file is compiled with hipcc for gfx950 and every
``csrc/*.cpp`` that belongs to the library with the host compiler; the objects
are linked into ``paper_1602_04716_amd/libbfp.so``.  ``bfp_host_sim.cpp`` is
built separately into ``paper_1602_04716_amd/libbfp_hostsim.so`` (test-only:
the GPU library never loads it), and ``tests/abi_consumer.c``, a C99 program
that includes only ``include/bfp.h`` and the HIP runtime's C API, into
``tests/abi_consumer`` (linked against libbfp.so).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libbfp.so")
HOSTSIM = os.path.join(PKG, "libbfp_hostsim.so")
CONSUMER_SRC = os.path.join(ROOT, "tests", "abi_consumer.c")
CONSUMER = os.path.join(ROOT, "tests", "abi_consumer")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC,
             # packed fp32 instructions are kept out of every code object
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
CXX_FLAGS = ["-O1", "-std=c++17", "-fPIC", "-Wall", "-Wno-unknown-pragmas", "-I" + INCLUDE, "-I" + CSRC]
HEADERS = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")] + \
    [os.path.join(INCLUDE, "bfp.h")]


def _stale(out: str, srcs) -> bool:
    if not os.path.exists(out):
        return True
    t = os.path.getmtime(out)
    return any(os.path.getmtime(s) > t for s in srcs)


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n%s\n%s" % (" ".join(cmd), r.stdout))
    return r.stdout


def build(force: bool = False, jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    hips = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    cpps = ["bfp_cost.cpp"]
    tasks = []
    objs = []
    for f in hips:
        src = os.path.join(CSRC, f)
        obj = os.path.join(OBJDIR, f[:-4] + ".o")
        objs.append(obj)
        if force or _stale(obj, [src] + HEADERS):
            tasks.append([HIPCC] + HIP_FLAGS + ["-c", src, "-o", obj])
    for f in cpps:
        src = os.path.join(CSRC, f)
        obj = os.path.join(OBJDIR, f[:-4] + ".cpp.o")
        objs.append(obj)
        if force or _stale(obj, [src] + HEADERS):
            tasks.append(["g++"] + CXX_FLAGS + ["-c", src, "-o", obj])
    hs_src = os.path.join(CSRC, "bfp_host_sim.cpp")
    if force or _stale(HOSTSIM, [hs_src] + HEADERS):
        tasks.append(["g++"] + CXX_FLAGS + ["-shared", hs_src, "-o", HOSTSIM + ".tmp"])
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for cmd, out in zip(tasks, ex.map(_run, tasks)):
            if verbose:
                print(" ".join(cmd[-3:]), flush=True)
    if os.path.exists(HOSTSIM + ".tmp"):
        os.replace(HOSTSIM + ".tmp", HOSTSIM)
    if force or _stale(LIB, objs):
        tmp = LIB + ".tmp%d" % os.getpid()
        _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
        os.replace(tmp, LIB)
    if force or _stale(CONSUMER, [CONSUMER_SRC, LIB, os.path.join(INCLUDE, "bfp.h")]):
        tmp = CONSUMER + ".tmp%d" % os.getpid()
        _run(["gcc", "-std=c99", "-O1", "-Wall", "-Wextra", "-pedantic", "-D__HIP_PLATFORM_AMD__",
              "-I" + INCLUDE, "-I" + os.path.join(ROCM, "include"), CONSUMER_SRC, "-o", tmp,
              "-L" + PKG, "-lbfp", "-Wl,-rpath,$ORIGIN/../paper_1602_04716_amd",
              "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
        os.replace(tmp, CONSUMER)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--force", action="store_true")
    ap.add_argument("-j", type=int, default=None)
    a = ap.parse_args(argv)
    print(build(force=a.force, jobs=a.j, verbose=True))


if __name__ == "__main__":
    sys.exit(main())
