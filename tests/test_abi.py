"""The C ABI without a GPU: the library loads, exports every function that
include/bfp.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1602_04716_amd import bfp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def declared():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(bfp_\w+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_functions():
    assert "bfp_pack" in declared() and "bfp_binop" in declared()


def test_every_declared_symbol_is_exported():
    out = subprocess.check_output(["nm", "-D", "--defined-only", bfp.LIB_PATH], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_binding_covers_header():
    missing = [n for n in declared() if not hasattr(bfp, n)]
    assert not missing, missing


def test_sizing():
    f = bfp.fmt(5, 10)
    assert bfp.bfp_container_bytes(f) == 2
    assert bfp.bfp_container_bytes(bfp.fmt(5, 2)) == 1
    assert bfp.bfp_container_bytes(bfp.fmt(8, 23)) == 4
    assert bfp.bfp_plane_stride_words(1) == 64
    assert bfp.bfp_plane_stride_words(64 * 32) == 64
    assert bfp.bfp_plane_stride_words(64 * 32 + 1) == 128
    assert bfp.bfp_plane_stride_words(2048 * 32) == 2048 + 256      # 8 KiB-multiple strides are skewed
    assert bfp.bfp_plane_stride_words(1 << 26) == (1 << 21) + 256
    assert bfp.bfp_plane_stride_words(2048 * 32 + 1) == 2048 + 64
    for n in (1, 1000, 65536, 70013, 1 << 20, (1 << 24) + 3):
        g = bfp.bfp_plane_stride_words(n)
        assert g % 64 == 0 and g * 32 >= n and g % 2048 != 0
    assert bfp.bfp_bitslice_bytes(f, 1 << 26) == 16 * ((1 << 21) + 256) * 4
    assert bfp.bfp_bitslice_bytes(bfp.fmt(7, 3), 10) == 0  # not compiled


def test_oracle_layout_follows_the_library_stride():
    """The oracle lays planes out at the library's documented stride, so the
    two sides are compared word for word: every n up to 2^17 + 2048, the
    non-monotonic window around a skewed stride (65,000 elements take 2,304
    words, 66,000 take 2,112), and large powers of two with their
    neighbours."""
    import oracle
    ns = list(range(0, (1 << 17) + 2048, 7)) + [65000, 66000, 65536, 65535, 65537]
    ns += [(1 << k) + d for k in range(17, 34) for d in (-1, 0, 1, 4096)]
    for n in ns:
        n = max(n, 1)
        assert oracle.plane_stride_words(n) == bfp.bfp_plane_stride_words(n), n
    assert oracle.plane_stride_words(65000) == 2304 and oracle.plane_stride_words(66000) == 2112


def test_wide_formats_sizing_and_table():
    for (e, m), C in (((8, 31), 8), ((11, 20), 4), ((11, 40), 8), ((11, 52), 8)):
        f = bfp.fmt(e, m)
        assert bfp.bfp_format_supported(f)
        assert bfp.bfp_container_bytes(f) == C
        assert bfp.bfp_bitslice_bytes(f, 1000) == (1 + e + m) * 64 * 4
        for op in ("add", "mul", "div"):
            assert bfp.bfp_launch_get(op, f).words_per_lane == 1
            assert bfp.bfp_gate_count(op, f) > 0
    w = bfp.fmt(11, 52)
    old = bfp.bfp_launch_get("mul", w)
    with pytest.raises(bfp.BfpError):
        bfp.bfp_launch_set("mul", w, 2, 256, 0)  # one-word kernels only
    bfp.bfp_launch_set("mul", w, 1, 128, 4)
    bfp.bfp_launch_set("mul", w, old.words_per_lane, old.block, old.blocks_per_cu, max(1, old.unroll))
    assert not bfp.bfp_format_supported(bfp.fmt(11, 53))
    assert not bfp.bfp_format_supported(bfp.fmt(12, 40))


def test_supported_formats():
    from paper_1602_04716_amd import inputs
    for (e, m) in inputs.sweep_formats():
        for r in (0, 1):
            assert bfp.bfp_format_supported(bfp.fmt(e, m, r))
    assert not bfp.bfp_format_supported(bfp.fmt(5, 2, 2))
    assert not bfp.bfp_format_supported(bfp.bfp_format(5, 2, 0, 1))
    assert not bfp.bfp_format_supported(bfp.fmt(9, 2))


def test_argument_errors_before_any_device_work():
    L = bfp.lib()
    f = bfp.fmt(5, 10)
    assert L.bfp_pack(bfp.fmt(7, 4), 16, 4096, 10, None) == -1          # format
    assert L.bfp_pack(f, 0, 4096, 10, None) == -2                        # null
    assert L.bfp_pack(f, 17, 4096, 10, None) == -3                       # alignment
    assert L.bfp_pack(f, 4096, 4096, 10, None) == -7                     # overlap
    assert L.bfp_pack(f, 0, 0, 0, None) == 0                             # n == 0
    assert L.bfp_binop(4, f, 16, 32, 48, 1, None) == -4                  # op
    assert L.bfp_binop(-1, f, 16, 32, 48, 1, None) == -4
    assert L.bfp_binop(0, f, 16, 32, 0, 1, None) == -2
    assert L.bfp_binop(0, f, 4096, 1 << 20, 4096 + 16, 100, None) == -7  # partial overlap
    assert L.bfp_binop(0, f, 4096, 1 << 20, 0, 0, None) == 0
    assert L.bfp_binop_std(2, bfp.fmt(5, 10, 3), 16, 32, 48, 1, None) == -1
    assert L.bfp_unpack(f, 16, 32, 1 << 40, None) == -6                  # too long
    assert L.bfp_chain2(3, 0, f, 16, 32, 48, 64, 1, None) == -4           # division is not chained
    assert L.bfp_chain2(0, 4, f, 16, 32, 48, 64, 1, None) == -4
    assert L.bfp_chain2(2, 0, f, 0, 32, 48, 64, 1, None) == -2
    assert L.bfp_chain2(2, 0, f, 16, 32, 48, 72, 1, None) == -3
    assert L.bfp_chain2(2, 0, f, 4096, 1 << 20, 1 << 21, 4096 + 16, 100, None) == -7
    assert L.bfp_chain2(2, 0, f, 0, 0, 0, 0, 0, None) == 0
    assert L.bfp_axpy(f, 0x3C00, 0, 32, 48, 1, None) == -2
    assert L.bfp_axpy(bfp.fmt(7, 4), 0x3C00, 16, 32, 48, 1, None) == -1
    assert L.bfp_int_binop(3, 8, 0, 16, 32, 48, 1, None) == -4             # no integer division
    assert L.bfp_int_binop(0, 0, 0, 16, 32, 48, 1, None) == -1             # k
    assert L.bfp_int_binop(0, 33, 0, 16, 32, 48, 1, None) == -1
    assert L.bfp_int_binop(0, 8, 3, 16, 32, 48, 1, None) == -1             # kind
    assert L.bfp_int_binop(0, 8, 1, 16, 0, 48, 1, None) == -2
    assert L.bfp_int_binop(0, 8, 1, 16, 40, 48, 1, None) == -3
    assert L.bfp_int_binop(2, 8, 2, 4096, 1 << 20, 4096 + 16, 100, None) == -7
    assert L.bfp_int_binop(2, 8, 2, 0, 0, 0, 0, None) == 0
    assert L.bfp_int_pack(33, 16, 4096, 10, None) == -1
    assert L.bfp_int_unpack(5, 16, 32, 1 << 40, None) == -6
    assert bfp.bfp_int_container_bytes(9) == 2 and bfp.bfp_int_container_bytes(0) == 0
    assert bfp.bfp_int_bitslice_bytes(13, 70000) == 13 * bfp.bfp_plane_stride_words(70000) * 4
    # wide formats: elementwise ops only (no chains, no batch or serving kernels)
    w = bfp.fmt(11, 52)
    assert L.bfp_chain2(2, 0, w, 16, 32, 48, 64, 1, None) == -1
    assert L.bfp_axpy(w, 0, 16, 32, 48, 1, None) == -1
    assert bfp.bfp_status_string(-5).startswith("HIP")
    g = ctypes.c_double()
    assert L.bfp_measure_copy(1 << 10, 10, None, ctypes.byref(g)) == -6   # too small
    assert L.bfp_measure_copy((1 << 20) + 8, 10, None, ctypes.byref(g)) == -6
    assert L.bfp_measure_copy(1 << 20, 0, None, ctypes.byref(g)) == -6
    assert L.bfp_measure_copy(1 << 20, 10, None, None) == -2
    assert L.bfp_wave_clock(0, None) == -6 and L.bfp_wave_clock((1 << 26) + 1, None) == -6
    assert L.bfp_measure_hbm(1 << 20, 4, 1, None, ctypes.byref(g), None, None, None) == -6    # no mode 4
    assert L.bfp_measure_hbm(1 << 20, -1, 1, None, ctypes.byref(g), None, None, None) == -6


def test_launch_table_roundtrip(tmp_path):
    f = bfp.fmt(6, 7, 1)
    old = bfp.bfp_launch_get("mul", f)
    bfp.bfp_launch_set("mul", f, 2, 128, 4)
    c = bfp.bfp_launch_get("mul", f)
    assert (c.words_per_lane, c.block, c.blocks_per_cu) == (2, 128, 4)
    assert bfp.bfp_launch_get("mul", f).block == 128
    p = str(tmp_path / "t.txt")
    bfp.bfp_launch_save(p)
    bfp.bfp_launch_set("mul", f, old.words_per_lane, old.block, old.blocks_per_cu, max(1, old.unroll))
    bfp.bfp_launch_load(p)
    assert bfp.bfp_launch_get("mul", f).block == 128
    bfp.bfp_launch_set("mul", f, old.words_per_lane, old.block, old.blocks_per_cu, max(1, old.unroll))
    # division has a table entry of its own
    old_d = bfp.bfp_launch_get("div", f)
    bfp.bfp_launch_set("div", f, 1, 512, 8)
    bfp.bfp_launch_save(p)
    bfp.bfp_launch_set("div", f, old_d.words_per_lane, old_d.block, old_d.blocks_per_cu, max(1, old_d.unroll))
    cm = bfp.bfp_launch_get("mul", f)
    assert (cm.words_per_lane, cm.block, cm.blocks_per_cu) == (old.words_per_lane, old.block, old.blocks_per_cu)
    bfp.bfp_launch_load(p)
    c = bfp.bfp_launch_get("div", f)
    assert (c.words_per_lane, c.block, c.blocks_per_cu) == (1, 512, 8)
    bfp.bfp_launch_set("div", f, old_d.words_per_lane, old_d.block, old_d.blocks_per_cu, max(1, old_d.unroll))
    bfp.bfp_launch_set("mul", f, old.words_per_lane, old.block, old.blocks_per_cu, max(1, old.unroll))
    with pytest.raises(bfp.BfpError):
        bfp.bfp_launch_set("add", f, 3, 256, 0)
    with pytest.raises(bfp.BfpError):
        bfp.bfp_launch_set("add", f, 1, 100, 0)


def test_gate_counts_positive():
    for op in ("add", "sub", "mul", "div"):
        assert bfp.bfp_gate_count(op, bfp.fmt(5, 10)) > 100
    assert bfp.bfp_gate_count(4, bfp.fmt(5, 10)) == -1
    assert bfp.bfp_gate_count("add", bfp.fmt(5, 10)) == bfp.bfp_gate_count("sub", bfp.fmt(5, 10))
    assert bfp.bfp_gate_count("add", bfp.fmt(7, 3)) == -1


def test_one_hip_runtime_per_process():
    """Loading the binding first and torch afterwards leaves one HIP runtime in
    the process (the binding binds torch's before libbfp.so loads)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1602_04716_amd import bfp\n"
            "bfp.lib()\n"
            "import torch\n"
            "print(sorted(set(l.split()[-1] for l in open('/proc/self/maps') if 'amdhip64' in l)))\n"
            % os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    import ast
    runtimes = ast.literal_eval(out.stdout.strip().splitlines()[-1])
    assert len(runtimes) == 1, runtimes


def test_chain_and_int_launch_tables_round_trip(tmp_path):
    """Chain and integer launch entries: validation, and save/load of the
    table with their lines (host only)."""
    f = bfp.fmt(5, 10)
    old_c = bfp.bfp_chain_launch_get("mul", "sub", f)
    old_i = bfp.bfp_int_launch_get("add", 9, "wrap")
    bfp.bfp_chain_launch_set("mul", "sub", f, 128, 4)
    bfp.bfp_int_launch_set("add", 9, "wrap", 512, 8)
    c = bfp.bfp_chain_launch_get("mul", "add", f)          # sub shares add's entry
    assert (c.block, c.blocks_per_cu, c.words_per_lane) == (128, 4, 1)
    i = bfp.bfp_int_launch_get("add", 9, "wrap")
    assert (i.block, i.blocks_per_cu) == (512, 8) and i.words_per_lane == old_i.words_per_lane
    with pytest.raises(bfp.BfpError):
        bfp.bfp_chain_launch_set("div", "add", f, 128, 0)  # division is not chained
    with pytest.raises(bfp.BfpError):
        bfp.bfp_chain_launch_set("mul", "add", f, 100, 0)
    with pytest.raises(bfp.BfpError):
        bfp.bfp_int_launch_set("add", 33, "wrap", 256, 0)
    path = str(tmp_path / "table.txt")
    bfp.bfp_launch_save(path)
    text = open(path).read()
    assert "chain 2 0 5 10 0 128 4" in text and "int 0 9 0 512 8" in text
    bfp.bfp_chain_launch_set("mul", "sub", f, old_c.block, old_c.blocks_per_cu)
    bfp.bfp_int_launch_set("add", 9, "wrap", old_i.block, old_i.blocks_per_cu)
    bfp.bfp_launch_load(path)
    assert bfp.bfp_chain_launch_get("mul", "add", f).block == 128
    assert bfp.bfp_int_launch_get("add", 9, "wrap").blocks_per_cu == 8
    bfp.bfp_chain_launch_set("mul", "sub", f, old_c.block, old_c.blocks_per_cu)
    bfp.bfp_int_launch_set("add", 9, "wrap", old_i.block, old_i.blocks_per_cu)


def test_layout_method_table(tmp_path):
    for d in ("pack", "unpack"):
        for cb in (1, 2, 4, 8):
            assert bfp.bfp_layout_method_get(d, cb) == bfp.BFP_TRANSPOSE_LANE
    bfp.bfp_layout_method_set("unpack", 2, bfp.BFP_TRANSPOSE_XLANE)
    assert bfp.bfp_layout_method_get("unpack", 2) == bfp.BFP_TRANSPOSE_XLANE
    path = str(tmp_path / "t.txt")
    bfp.bfp_launch_save(path)
    assert "layout 1 2 1" in open(path).read()
    bfp.bfp_layout_method_set("unpack", 2, bfp.BFP_TRANSPOSE_LANE)
    bfp.bfp_launch_load(path)
    assert bfp.bfp_layout_method_get("unpack", 2) == bfp.BFP_TRANSPOSE_XLANE
    bfp.bfp_layout_method_set("unpack", 2, bfp.BFP_TRANSPOSE_LANE)
    with pytest.raises(bfp.BfpError):
        bfp.bfp_layout_method_set("pack", 8, bfp.BFP_TRANSPOSE_XLANE)  # 8-byte containers: per lane only
    with pytest.raises(bfp.BfpError):
        bfp.bfp_layout_method_set("pack", 3, 0)
    with pytest.raises(bfp.BfpError):
        bfp.bfp_layout_method_set(2, 1, 0)


CONSUMER = os.path.join(ROOT, "tests", "abi_consumer")


def test_c_consumer_host_mode():
    """A C99 program that includes only include/bfp.h (and the HIP runtime's
    C API) and links libbfp.so: its host-side calls agree with the binding's."""
    assert os.path.exists(CONSUMER), "tests/abi_consumer is built by paper_1602_04716_amd.build"
    out = subprocess.run([CONSUMER, "host"], check=True, capture_output=True, text=True, timeout=60).stdout
    kv = dict(line.split(" ", 1) for line in out.strip().splitlines())
    f = bfp.fmt(5, 10)
    assert kv["version"] == bfp.bfp_version()
    assert int(kv["container_bytes_5_10"]) == bfp.bfp_container_bytes(f)
    for n in (1, 2048, 65000, 66000):
        assert int(kv["stride_%d" % n]) == bfp.bfp_plane_stride_words(n)
    assert int(kv["bitslice_bytes_5_10_65000"]) == bfp.bfp_bitslice_bytes(f, 65000)
    assert int(kv["gates_add_5_10"]) == bfp.bfp_gate_count("add", f)
    assert int(kv["gates_mul_5_10"]) == bfp.bfp_gate_count("mul", f)
    assert kv["format_7_4_supported"] == "0" and kv["pack_bad_format"] == str(bfp.BFP_E_FORMAT)
    assert kv["status_null"] == bfp.bfp_status_string(bfp.BFP_E_NULL)


def test_header_compiles_as_c99_and_cxx():
    src = '#include "bfp.h"\nint main(void) { bfp_format f = {5, 10, BFP_RNE, 0}; return (int)bfp_container_bytes(f); }\n'
    inc = os.path.join(ROOT, "include")
    for cc, std, ext in (("gcc", "-std=c99", "c"), ("g++", "-std=c++17", "cpp")):
        r = subprocess.run([cc, std, "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only", "-I" + inc,
                            "-x", "c" if ext == "c" else "c++", "-"], input=src, capture_output=True, text=True)
        assert r.returncode == 0, (cc, r.stderr)
