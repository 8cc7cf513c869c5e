"""Code generation checks on the library's own kernels (CPU: hipcc emits
gfx950 assembly without a GPU).

The elementwise kernels read their block and grid sizes in the kernel and
pass them to the inlined bodies.  Read inside an inlined body, the compiler
fetched the block size with a 16-bit vector load from the dispatch's hidden
arguments and waited for it (``s_waitcnt vmcnt(0)``) before the first
operand load of every wave; this checks that no kernel starts that way."""
import os
import re
import subprocess

import pytest

from paper_1602_04716_amd import build

INSTANCES = r"""
#include "bfp_kernels.hpp"
template __global__ void bfp::k_binop<5, 10, false, 1, 2, 1>(const uint32_t*, const uint32_t*, uint32_t*, uint64_t,
                                                            uint64_t, uint32_t);
template __global__ void bfp::k_binop<8, 7, false, 0, 1, 2>(const uint32_t*, const uint32_t*, uint32_t*, uint64_t,
                                                           uint64_t, uint32_t);
template __global__ void bfp::k_binop_std<5, 2, false, 0>(const uint8_t*, const uint8_t*, uint8_t*, uint64_t,
                                                          uint32_t);
template __global__ void bfp::k_binop_std_w<11, 52, false, 1>(const uint8_t*, const uint8_t*, uint8_t*, uint64_t,
                                                              uint32_t);
"""


def _kernels(asm: str):
    """(name, instructions) of every kernel in an assembly listing."""
    parts = re.split(r"\n(_Z\w+):\s+; @", asm)
    for k in range(1, len(parts), 2):
        body = parts[k + 1][:parts[k + 1].find("s_endpgm")]
        yield parts[k], [ln.strip() for ln in body.splitlines()
                         if ln.startswith("\t") and not ln.strip().startswith((";", "."))]


def test_no_vector_load_of_launch_dimensions(tmp_path):
    if not os.path.exists(build.HIPCC):
        pytest.skip("hipcc not installed")
    src = tmp_path / "inst.hip"
    src.write_text(INSTANCES)
    out = tmp_path / "inst.s"
    subprocess.run([build.HIPCC] + build.HIP_FLAGS + ["--cuda-device-only", "-S", str(src), "-o", str(out)],
                   check=True, capture_output=True, timeout=600)
    kernels = dict(_kernels(out.read_text()))
    assert len(kernels) == 4, sorted(kernels)
    for name, ins in kernels.items():
        # the first vector memory access is an operand load of 32-bit words
        # or wider, not the 16-bit read of the block size
        first_vm = next(ln for ln in ins if ln.startswith(("global_load", "buffer_load", "flat_load")))
        assert first_vm.startswith("global_load_dword"), (name, first_vm)
