"""Seeded synthetic operands for custom-precision FP vectors.

This module only draws input bit patterns; it holds none of the arithmetic
that is being tested (no add, sub, mul or rounding of results).  Tests, the
benchmark and the smoke check all take their operands from here.

Patterns use the standard layout of a (1, e, m) value in the low 1+e+m bits
of an unsigned container: mantissa in bits [0, m), exponent in [m, m+e),
sign in bit m+e.  Real-valued draws are mapped onto the format by truncation
of the binary64 value (an input recipe only; the choice does not matter for
the distribution the workloads describe).

Workload recipes (the paper measures synthetic FP8/FP16/FP32 vectors,
Section 5.2; there is no dataset):

* ``plain_8bit``: uniform random (5,2) patterns, NaN/Inf patterns redrawn.
* ``scaled_normal``: N(0,1) * 2^U(-8,8), mapped to the format.
* ``sweep_operands``: magnitude log-uniform over the normal range, random sign,
  plus 0.5% random subnormals and 0.5% signed zeros.
* ``batch_tasks``: lengths log-uniform in [1024, 1048576], format uniform over
  the 40-format sweep, op uniform over add/sub/mul.
"""
from __future__ import annotations

import numpy as np

SWEEP_E = (3, 4, 5, 6, 8)
SWEEP_M = (1, 2, 3, 5, 7, 10, 15, 23)


def sweep_formats():
    return [(e, m) for e in SWEEP_E for m in SWEEP_M]


def wide_formats():
    """The compiled formats beyond the sweep (8-byte containers above 32 bits)."""
    return [(8, 31), (11, 20), (11, 40), (11, 52)]


def container_dtype(e: int, m: int):
    B = 1 + e + m
    return np.uint8 if B <= 8 else (np.uint16 if B <= 16 else np.uint32)


def _exp_field_max(e):
    return (1 << e) - 1


def plain_8bit(n: int = 65536, seed: int = 1, e: int = 5, m: int = 2) -> np.ndarray:
    """Uniform random patterns of a format with B <= 8, excluding NaN/Inf."""
    rng = np.random.default_rng(seed)
    out = rng.integers(0, 1 << (1 + e + m), n, dtype=np.uint32)
    while True:
        bad = ((out >> m) & _exp_field_max(e)) == _exp_field_max(e)
        k = int(bad.sum())
        if k == 0:
            break
        out[bad] = rng.integers(0, 1 << (1 + e + m), k, dtype=np.uint32)
    return out.astype(container_dtype(e, m))


def exhaustive_pairs(B: int):
    """All 2^B x 2^B operand pairs as two vectors: a_i = i >> B, b_i = i & (2^B - 1)."""
    i = np.arange(1 << (2 * B), dtype=np.uint32)
    return i >> B, i & ((1 << B) - 1)


def from_real_truncate(x: np.ndarray, e: int, m: int) -> np.ndarray:
    """Map binary64 values to (1,e,m) patterns by truncation; values beyond the
    largest finite magnitude map to it."""
    x = np.asarray(x, dtype=np.float64)
    bias = (1 << (e - 1)) - 1
    s = np.signbit(x).astype(np.uint64)
    ax = np.abs(x)
    mant, ex = np.frexp(ax)  # ax = mant * 2^ex, mant in [0.5, 1)
    E = ex.astype(np.int64) - 1 + bias
    Mn = np.floor((2.0 * mant - 1.0) * (1 << m)).astype(np.int64)
    Emax = _exp_field_max(e) - 1
    sub = E <= 0
    over = E > Emax
    Ms = np.floor(np.ldexp(np.where(sub, ax, 0.0), bias - 1 + m)).astype(np.int64)  # subnormal grid
    Ef = np.where(sub, 0, np.where(over, Emax, E))
    Mf = np.where(sub, np.minimum(Ms, (1 << m) - 1), np.where(over, (1 << m) - 1, Mn))
    Ef = np.where(ax == 0, 0, Ef)
    Mf = np.where(ax == 0, 0, Mf)
    pat = (s << (e + m)) | (Ef.astype(np.uint64) << m) | Mf.astype(np.uint64)
    return pat.astype(container_dtype(e, m))


def scaled_normal(e: int, m: int, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n) * np.exp2(rng.uniform(-8.0, 8.0, n))
    return from_real_truncate(x, e, m)


def sweep_operands(e: int, m: int, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    bias = (1 << (e - 1)) - 1
    mag = np.exp2(rng.uniform(1 - bias, bias + 1, n))
    sign = rng.integers(0, 2, n) * 2 - 1
    pat = from_real_truncate(mag * sign, e, m).astype(np.uint64)
    u = rng.random(n)
    sub = u < 0.005
    zero = (u >= 0.005) & (u < 0.01)
    ns, nz = int(sub.sum()), int(zero.sum())
    sgn = rng.integers(0, 2, n).astype(np.uint64) << (e + m)
    pat[sub] = sgn[sub] | rng.integers(1, 1 << m, ns, dtype=np.uint64, endpoint=False)
    pat[zero] = sgn[zero]
    return pat.astype(container_dtype(e, m))


def batch_tasks(count: int = 4096, seed: int = 4, nmin: int = 1024, nmax: int = 1048576):
    """List of (n, e, m, op) with op in {'add','sub','mul'}."""
    rng = np.random.default_rng(seed)
    fmts = sweep_formats()
    ns = np.floor(np.exp(rng.uniform(np.log(nmin), np.log(nmax + 1), count))).astype(np.int64)
    ns = np.clip(ns, nmin, nmax)
    fi = rng.integers(0, len(fmts), count)
    ops = rng.integers(0, 3, count)
    names = ("add", "sub", "mul")
    return [(int(ns[i]), fmts[fi[i]][0], fmts[fi[i]][1], names[ops[i]]) for i in range(count)]
