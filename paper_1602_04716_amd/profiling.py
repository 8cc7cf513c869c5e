"""Summaries of rocprofv3 databases (kernel trace and byte counters).

    python -m paper_1602_04716_amd.profiling --trace T.db --fetch F.db --write W.db \
        --kernel k_unpack<2> --out profiles/NAME --command-trace "..." --command-fetch "..." \
        --command-write "..."

writes ``NAME.md`` (per-kernel durations and calibrated HBM bytes, with the
commands that produced the databases) and ``NAME.traffic.txt`` (the chosen
kernel's HBM bytes per launch and the hash of the kernel sources the counters
were taken with).  The byte counters are scaled by what the same counter reads
for the run's calibration kernel, a plain int32 -> float32 conversion of 2^26
elements (256 MiB read, 256 MiB written).
"""
from __future__ import annotations

import argparse
import collections
import hashlib
import os
import re
import sqlite3

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["bfp_word.hpp", "bfp_circuits.hpp", "bfp_transpose.hpp", "bfp_kernels.hpp",
                  "bfp_ops.hpp", "bfp_runtime.hip", "bfp_batch.hip"]
CALIB_BYTES = 256 * 1024 * 1024  # read and written by the calibration kernel
CALIB_PATTERN = "direct_copy_kernel"


def source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(PKG, "csrc", f), "rb") as fp:
            h.update(fp.read())
    return h.hexdigest()[:16]


def short_name(n: str) -> str:
    return re.sub(r"\(.*", "", n.replace("void ", "")).strip()


def trace_stats(db: str):
    c = sqlite3.connect(db).cursor()
    return [(short_name(r[0]), r[1], r[3], r[2], r[4])
            for r in c.execute("select name, total_calls, total_duration, average, percentage from top_kernels")]


def counter_per_dispatch(db: str):
    """(kernel short name) -> list of per-dispatch values (KiB)."""
    c = sqlite3.connect(db).cursor()
    d = collections.defaultdict(list)
    for name, val in c.execute("select kernel_name, value from counters_collection"):
        d[name].append(val)
    return d


def _calib(d):
    for name, vals in d.items():
        if CALIB_PATTERN in name:
            return vals[0]
    raise RuntimeError("calibration kernel not found in counter database")


def summarize(trace_db, fetch_db, write_db, kernel, out, commands):
    stats = trace_stats(trace_db)
    fetch = counter_per_dispatch(fetch_db)
    write = counter_per_dispatch(write_db)
    f_fac = (CALIB_BYTES / 1024) / _calib(fetch)
    w_fac = (CALIB_BYTES / 1024) / _calib(write)
    lines = ["# rocprofv3 summary: %s" % os.path.basename(out), "",
             "Kernel sources hash: `%s`" % source_hash(), "",
             "Commands (run from the repository root on one MI355X):", ""]
    for k, v in commands.items():
        lines.append("- %s: `%s`" % (k, v))
    lines += ["", "## Kernel trace (--kernel-trace --stats)", "",
              "| kernel | calls | avg us | total us | % |", "|---|---|---|---|---|"]
    for (n, calls, avg, tot, pct) in stats:
        lines.append("| `%s` | %d | %.2f | %.1f | %.1f |" % (n, calls, avg, tot, pct))
    lines += ["", "## HBM bytes per dispatch (FETCH_SIZE, WRITE_SIZE)", "",
              "Calibration: the int32->float32 copy of 2^26 elements reads and writes 262144 KiB; its "
              "FETCH_SIZE reads %.1f KiB and WRITE_SIZE %.1f KiB, so the factors are %.4f (fetch) and "
              "%.4f (write)." % (_calib(fetch), _calib(write), f_fac, w_fac), "",
              "| kernel | dispatches | FETCH KiB (raw) | WRITE KiB (raw) | HBM MB (scaled) |",
              "|---|---|---|---|---|"]
    chosen = None
    for name in fetch:
        fv = sum(fetch[name]) / len(fetch[name])
        wv = sum(write.get(name, [0.0])) / max(1, len(write.get(name, [])))
        mb = (fv * f_fac + wv * w_fac) * 1024 / 1e6
        lines.append("| `%s` | %d | %.1f | %.1f | %.1f |" % (short_name(name)[:70], len(fetch[name]), fv, wv, mb))
        if short_name(name).endswith(kernel) or short_name(name) == kernel or kernel in short_name(name):
            chosen = (short_name(name), fv * f_fac * 1024, wv * w_fac * 1024)
    with open(out + ".md", "w") as fp:
        fp.write("\n".join(lines) + "\n")
    if chosen:
        with open(out + ".traffic.txt", "w") as fp:
            fp.write("kernel %s\nsource_hash %s\nfetch_bytes_per_launch %.0f\nwrite_bytes_per_launch %.0f\n"
                     "traffic_bytes_per_launch %.0f\n" % (chosen[0], source_hash(), chosen[1], chosen[2],
                                                         chosen[1] + chosen[2]))
    return chosen


def read_traffic(path: str):
    """Traffic per launch from a .traffic.txt file, or None if the kernel
    sources changed since the counters were taken."""
    if not os.path.exists(path):
        return None
    d = {}
    for line in open(path):
        k, _, v = line.strip().partition(" ")
        d[k] = v
    if d.get("source_hash") != source_hash():
        return None
    return {"kernel": d.get("kernel"), "bytes": float(d["traffic_bytes_per_launch"])}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--command-trace", default="")
    ap.add_argument("--command-fetch", default="")
    ap.add_argument("--command-write", default="")
    a = ap.parse_args(argv)
    print(summarize(a.trace, a.fetch, a.write, a.kernel, a.out,
                    {"trace": a.command_trace, "FETCH_SIZE": a.command_fetch, "WRITE_SIZE": a.command_write}))


if __name__ == "__main__":
    main()
