"""Oracle for bitslice custom-precision floating point.

TEST INFRASTRUCTURE ONLY: this package is used by ``tests/``, by the smoke
check in ``__graft_entry__`` and by the CPU-baseline leg of ``bench.py``.  The
GPU library and its Python binding never import it.

The arithmetic lives in ``bfp_oracle.c`` (plain C, exact integers): decode to
(sign, integer significand, exponent), compute the exact sum, product or
quotient, round once to nearest-even or toward zero (Section 4 of the paper
fixes the two modes; Table 1 the operations).  k-bit integer vectors
(Section 3, Figure 2) take the exact result modulo 2^k or clamped to the
unsigned / signed range.  This module only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bfp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ADD, SUB, MUL, DIV = 0, 1, 2, 3
RNE, RZ = 0, 1
OPS = {"add": ADD, "sub": SUB, "mul": MUL, "div": DIV}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread",
             _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        u32, i32, u64 = ctypes.c_uint32, ctypes.c_int, ctypes.c_uint64
        vp = ctypes.c_void_p
        L.oracle_op1.restype = u32
        L.oracle_op1.argtypes = [i32, i32, i32, i32, u32, u32]
        L.oracle_op1_64.restype = u64
        L.oracle_op1_64.argtypes = [i32, i32, i32, i32, u64, u64]
        L.oracle_from_double.restype = u64
        L.oracle_from_double.argtypes = [i32, i32, i32, ctypes.c_double]
        L.oracle_binop64.restype = i32
        L.oracle_binop64.argtypes = [i32, i32, i32, i32, vp, vp, vp, u64, i32]
        L.oracle_pack.restype = i32
        L.oracle_pack.argtypes = [i32, i32, vp, vp, u64, u64]
        L.oracle_unpack.restype = i32
        L.oracle_unpack.argtypes = [i32, i32, vp, vp, u64, u64]
        L.oracle_int_binop.restype = i32
        L.oracle_int_binop.argtypes = [i32, i32, i32, vp, vp, vp, u64]
        _lib = L
    return _lib


def _op(op) -> int:
    return OPS[op] if isinstance(op, str) else int(op)


def op1(op, e: int, m: int, mode: int, a: int, b: int) -> int:
    """One element: pattern of a op b."""
    r = lib().oracle_op1_64(_op(op), e, m, mode, a, b)
    if r == 0xFFFFFFFFFFFFFFFF:
        raise ValueError("invalid oracle arguments")
    return int(r)


def binop(op, e: int, m: int, mode: int, a, b, nthreads: int = 1) -> np.ndarray:
    """Elementwise a op b over arrays of patterns (any unsigned container).
    Returns uint32 patterns for formats of at most 32 bits, else uint64."""
    a64 = np.ascontiguousarray(np.asarray(a).astype(np.uint64))
    b64 = np.ascontiguousarray(np.asarray(b).astype(np.uint64))
    if a64.shape != b64.shape:
        raise ValueError("shape mismatch")
    c = np.empty_like(a64)
    rc = lib().oracle_binop64(_op(op), e, m, mode, a64.ctypes.data, b64.ctypes.data,
                              c.ctypes.data, a64.size, nthreads)
    if rc != 0:
        raise ValueError("invalid oracle arguments")
    return c.astype(np.uint32) if 1 + e + m <= 32 else c


def chain2(op1, op2, e: int, m: int, mode: int, a, b, c, nthreads: int = 1) -> np.ndarray:
    """(a op1 b) op2 c, each op rounded on its own: the definition of a
    two-op chain is the composition of the two elementwise ops."""
    t = binop(op1, e, m, mode, a, b, nthreads)
    return binop(op2, e, m, mode, t, c, nthreads)


def axpy(e: int, m: int, mode: int, alpha: int, x, y, nthreads: int = 1) -> np.ndarray:
    """alpha * x + y with the pattern alpha broadcast (bits above 1+e+m ignored)."""
    xs = np.asarray(x)
    al = np.full(xs.shape, int(alpha) & ((1 << (1 + e + m)) - 1), dtype=np.uint64)
    return chain2("mul", "add", e, m, mode, al, xs, y, nthreads)


INT_WRAP, INT_SAT_U, INT_SAT_S = 0, 1, 2
INT_KINDS = {"wrap": INT_WRAP, "satu": INT_SAT_U, "sats": INT_SAT_S}


def int_binop(op, k: int, kind, a, b) -> np.ndarray:
    """Elementwise a op b on k-bit integer patterns (1 <= k <= 32): wrap
    modulo 2^k, or saturate as unsigned / signed (see bfp_oracle.c)."""
    a32 = np.ascontiguousarray(np.asarray(a).astype(np.uint32))
    b32 = np.ascontiguousarray(np.asarray(b).astype(np.uint32))
    if a32.shape != b32.shape:
        raise ValueError("shape mismatch")
    kd = INT_KINDS[kind] if isinstance(kind, str) else int(kind)
    c = np.empty_like(a32)
    if lib().oracle_int_binop(_op(op), k, kd, a32.ctypes.data, b32.ctypes.data, c.ctypes.data, a32.size) != 0:
        raise ValueError("invalid oracle arguments")
    return c


def int_container_bytes(k: int) -> int:
    return 1 if k <= 8 else (2 if k <= 16 else 4)


def from_double(e: int, m: int, mode: int, v: float) -> int:
    return int(lib().oracle_from_double(e, m, mode, float(v)))


def container_bytes(e: int, m: int) -> int:
    B = 1 + e + m
    return 1 if B <= 8 else (2 if B <= 16 else (4 if B <= 32 else 8))


def plane_stride_words(n: int) -> int:
    """32-bit words per plane: ceil(n/32) rounded up to a multiple of 64, plus
    256 when that is a multiple of 2048 (the library's documented layout)."""
    g = (n + 31) // 32
    gp = (g + 63) // 64 * 64
    return gp + 256 if gp % 2048 == 0 else gp


def pack(e: int, m: int, x, gpad: int | None = None) -> np.ndarray:
    """Standard containers -> bitslice planes, shape (B, gpad) uint32."""
    B = 1 + e + m
    c = container_bytes(e, m)
    dt = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}[c]
    xs = np.ascontiguousarray(np.asarray(x).astype(dt))
    n = xs.size
    gpad = plane_stride_words(n) if gpad is None else gpad
    planes = np.empty((B, gpad), dtype=np.uint32)
    if lib().oracle_pack(B, c, xs.ctypes.data, planes.ctypes.data, n, gpad) != 0:
        raise ValueError("invalid pack arguments")
    return planes


def unpack(e: int, m: int, planes, n: int) -> np.ndarray:
    """Bitslice planes (B, gpad) -> standard containers (uint8/16/32)."""
    B = 1 + e + m
    c = container_bytes(e, m)
    dt = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}[c]
    p = np.ascontiguousarray(np.asarray(planes, dtype=np.uint32))
    if p.shape[0] != B:
        raise ValueError("plane count mismatch")
    out = np.empty(n, dtype=dt)
    if lib().oracle_unpack(B, c, p.ctypes.data, out.ctypes.data, n, p.shape[1]) != 0:
        raise ValueError("invalid unpack arguments")
    return out
