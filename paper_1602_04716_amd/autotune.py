"""Autotune bfp_binop for every compiled format and record the format sweep.

    python -m paper_1602_04716_amd.autotune [--n-log2 26] [--reps 7] [--out tuning/gfx950.txt]

For each format of the sweep (e in {3,4,5,6,8} x m in {1,2,3,5,7,10,15,23})
and the four wide formats (one-word kernels only),
each op class (add, mul, div) and each rounding mode, ``bfp_autotune`` times the
launch variants (words per lane, units per step, block, grid depth) on a
2^26-element probe with the last-level cache swept clean (at 2^24 elements a
single launch of a light format is a few microseconds, close to the dispatch
time, and the candidates differ by less than the noise)
before every run and installs the fastest; the table is saved for
``bfp.lib()`` to load.  The printed JSON lines are the format-sweep
measurement: elements/s, achieved HBM GB/s (3B/8 bytes per element) and
bitwise VALU rate (gate count / 32 per element) of the tuned kernel, and the
fraction of each peak.  The two-op chain kernels (``bfp_autotune_chain``) and
the k-bit integer kernels (``bfp_autotune_int``) are tuned after them over
block size and grid depth, and saved in the same table.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

from . import bfp, inputs

HBM_PEAK = 8.0e12
VALU_PEAK = 256 * 4 * 16 * 2.4e9


def tune(formats, ops=("add", "mul", "div"), modes=(0, 1), n=1 << 26, reps=7, mask=7, log=print):
    out = []
    for (e, m) in formats:
        for op in ops:
            for r in modes:
                f = bfp.fmt(e, m, r)
                best, us = bfp.bfp_autotune(op, f, n, mask, reps)
                B = 1 + e + m
                G = bfp.bfp_gate_count(op, f)
                gbs = 3 * B / 8 * n / (us * 1e-6)
                ops_s = G * n / 32 / (us * 1e-6)
                rec = {"op": op, "e": e, "m": m, "round": "RZ" if r else "RNE", "n": n,
                       "words_per_lane": best.words_per_lane, "block": best.block,
                       "blocks_per_cu": best.blocks_per_cu, "unroll": max(1, best.unroll), "us": us, "elements_per_s": n / (us * 1e-6),
                       "GB/s": gbs / 1e9, "hbm_frac": gbs / HBM_PEAK, "Tops/s": ops_s / 1e12,
                       "valu_frac": ops_s / VALU_PEAK, "gates": G,
                       "bound": "alu" if ops_s / VALU_PEAK > gbs / HBM_PEAK else "hbm"}
                out.append(rec)
                log(json.dumps(rec))
    return out


def tune_chains(formats, modes=(0, 1), n=1 << 24, reps=5, log=print):
    """Block and grid depth of the two-op chain kernels, per format, op-class
    pair and mode (sub shares add's entries)."""
    for (e, m) in formats:
        for o1 in ("add", "mul"):
            for o2 in ("add", "mul"):
                for r in modes:
                    best, us = bfp.bfp_autotune_chain(o1, o2, bfp.fmt(e, m, r), n, reps)
                    log(json.dumps({"kind": "chain", "op1": o1, "op2": o2, "e": e, "m": m, "round": r,
                                    "block": best.block, "blocks_per_cu": best.blocks_per_cu, "us": us}))


def tune_ints(ks=range(1, 33), n=1 << 24, reps=5, log=print):
    """Block and grid depth of the k-bit integer kernels, per k, op and kind."""
    for k in ks:
        for op in ("add", "sub", "mul"):
            for kind in ("wrap", "satu", "sats"):
                best, us = bfp.bfp_autotune_int(op, k, kind, n, reps)
                log(json.dumps({"kind": "int", "op": op, "k": k, "int_kind": kind, "block": best.block,
                                "blocks_per_cu": best.blocks_per_cu, "words_per_lane": best.words_per_lane,
                                "us": us}))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-log2", type=int, default=26)
    ap.add_argument("--reps", type=int, default=7)
    ap.add_argument("--out", default=bfp.TUNE_TABLE)
    ap.add_argument("--formats", default="", help="comma list like 5:10,8:7; default all 44")
    ap.add_argument("--ops", default="add,mul,div", help="op classes to tune (sub shares add's entry)")
    ap.add_argument("--no-chains", action="store_true")
    ap.add_argument("--no-ints", action="store_true")
    a = ap.parse_args(argv)
    import torch
    assert torch.cuda.is_available()
    os.environ["BFP_TUNE_FILE"] = ""  # start from the built-in defaults
    bfp.lib()
    fmts = inputs.sweep_formats() + inputs.wide_formats()
    if a.formats:
        fmts = [tuple(int(x) for x in s.split(":")) for s in a.formats.split(",")]
    log = lambda s: print(s, flush=True)
    tune(fmts, ops=tuple(a.ops.split(",")), n=1 << a.n_log2, reps=a.reps, log=log)
    if not a.no_chains:
        tune_chains([f for f in fmts if f in inputs.sweep_formats()], n=1 << a.n_log2, log=log)
    if not a.no_ints:
        tune_ints(n=1 << a.n_log2, log=log)
    if a.out:
        os.makedirs(os.path.dirname(a.out), exist_ok=True)
        bfp.bfp_launch_save(a.out)
        print("saved", a.out, flush=True)


if __name__ == "__main__":
    sys.exit(main())
