"""Summaries of rocprofv3 databases (kernel trace, byte and VALU counters).

    python -m paper_1602_04716_amd.profiling --trace T.db --fetch F.db --write W.db \
        --kernel k_unpack<2> --out profiles/NAME --command-trace "..." --command-fetch "..." \
        --command-write "..."

writes ``NAME.md`` (per-kernel durations and calibrated HBM bytes, with the
commands that produced the databases) and ``NAME.traffic.txt`` (the chosen
kernel's HBM bytes per launch and the hash of the kernel sources the counters
were taken with).  The byte counters are scaled by what the same counter reads
for the run's calibration kernel, a plain int32 -> float32 conversion of 2^26
elements (256 MiB read, 256 MiB written).

    python -m paper_1602_04716_amd.profiling valu --trace T.db --pmc P.db --out profiles/NAME ...

writes ``NAME.md`` with the circuit kernels' measured VALU instructions
(SQ_INSTS_VALU) per 32 elements beside their gate counts.
"""
from __future__ import annotations

import argparse
import collections
import hashlib
import os
import re
import sqlite3

PKG = os.path.dirname(os.path.abspath(__file__))
FLUSH_KERNEL = "k_sweep_read"  # the cache flush that precedes each cold group in bench.py
CALIB_BYTES = 256 * 1024 * 1024  # read and written by the calibration kernel
CALIB_PATTERN = "direct_copy_kernel"


def source_hash() -> str:
    """Hash of every library source (csrc/ and include/) and of the build
    flags: a committed counter figure is current only for the code it was
    taken with."""
    from . import build
    h = hashlib.sha256()
    srcs = sorted(os.listdir(os.path.join(PKG, "csrc")))
    for f in srcs:
        with open(os.path.join(PKG, "csrc", f), "rb") as fp:
            h.update(f.encode() + b"\0" + fp.read())
    for f in sorted(os.listdir(build.INCLUDE)):
        with open(os.path.join(build.INCLUDE, f), "rb") as fp:
            h.update(f.encode() + b"\0" + fp.read())
    h.update(" ".join(build.HIP_FLAGS + build.CXX_FLAGS).replace(build.ROOT, "").encode())
    return h.hexdigest()[:16]


def short_name(n: str) -> str:
    n = n.replace("void ", "").replace("(anonymous namespace)::", "")
    return re.sub(r"\(.*", "", n).strip()


def trace_stats(db: str):
    c = sqlite3.connect(db).cursor()
    return [(short_name(r[0]), r[1], r[3], r[2], r[4])
            for r in c.execute("select name, total_calls, total_duration, average, percentage from top_kernels")]


def dispatches(db: str):
    """Every kernel dispatch in start order: (short name, duration us, grid size)."""
    c = sqlite3.connect(db).cursor()
    return [(short_name(r[0]), (r[2] - r[1]) / 1e3, r[3])
            for r in c.execute("select name, start, end, grid_x from kernels order by start")]


def cold_average(db: str, kernel: str):
    """Durations (us) of `kernel`'s dispatches that run right after the
    cache flush: each run of back-to-back dispatches of the kernel after a
    flush is one cold run (bench.py's cold groups, and its back-to-back
    measurement of the dominant kernel, the longest run).  Only dispatches at
    the grid size most cold ones have (the bench's main workload) count."""
    import collections as _c
    runs, other = [], []
    prev = None  # last dispatch that was not `kernel`
    cur = None
    for name, us, grid in dispatches(db):
        if name.endswith(kernel) or name == kernel:
            if prev is not None and FLUSH_KERNEL in prev:
                if cur is None:
                    cur = []
                    runs.append(cur)
                cur.append((us, grid))
            else:
                other.append(us)
        else:
            prev = name
            cur = None
    cold = [x for r in runs for x in r]
    grid = _c.Counter(g for _u, g in cold).most_common(1)[0][0] if cold else None
    runs = [[u for u, g in r if g == grid] for r in runs]
    runs = [r for r in runs if r]
    avg = lambda v: sum(v) / len(v) if v else float("nan")
    longest = max(runs, key=len) if runs else []
    return {"cold_grid": grid, "cold_dispatches": sum(len(r) for r in runs),
            "cold_avg_us": avg([u for r in runs for u in r]),
            "longest_run": len(longest), "longest_run_avg_us": avg(longest),
            "other_dispatches": len(other), "other_avg_us": avg(other)}


def counter_per_dispatch(db: str, main_grid_only: bool = False):
    """(kernel name) -> list of per-dispatch values (KiB); with
    `main_grid_only`, only each kernel's dispatches at its largest grid."""
    if main_grid_only:
        d = collections.defaultdict(list)
        for name, _cn, val in _main_grid_rows(db, short=False):
            d[name].append(val)
        return d
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
    # The calibration copy is the first dispatch of its kernel, whatever its
    # grid; every other kernel counts its dispatches at its largest grid.
    f_fac = (CALIB_BYTES / 1024) / _calib(counter_per_dispatch(fetch_db))
    w_fac = (CALIB_BYTES / 1024) / _calib(counter_per_dispatch(write_db))
    fetch = counter_per_dispatch(fetch_db, main_grid_only=True)
    write = counter_per_dispatch(write_db, main_grid_only=True)
    lines = ["# rocprofv3 summary: %s" % os.path.basename(out), "",
             "Kernel sources hash: `%s`" % source_hash(), "",
             "Commands (run from the repository root on one MI355X):", ""]
    for k, v in commands.items():
        lines.append("- %s: `%s`" % (k, v))
    lines += ["", "## Kernel trace (--kernel-trace --stats)", "",
              "| kernel | calls | avg us | total us | % |", "|---|---|---|---|---|"]
    for (n, calls, avg, tot, pct) in stats:
        lines.append("| `%s` | %d | %.2f | %.1f | %.1f |" % (n, calls, avg, tot, pct))
    ca = cold_average(trace_db, kernel)
    lines += ["", "## `%s`: dispatches after the bench's cache flush, and the others" % kernel, "",
              "| dispatches | count | avg us |", "|---|---|---|",
              "| longest back-to-back run after a flush (the bench's roofline measurement) | %d | %.2f |"
              % (ca["longest_run"], ca["longest_run_avg_us"]),
              "| every run after a flush (cold groups and the run above) | %d | %.2f |"
              % (ca["cold_dispatches"], ca["cold_avg_us"]),
              "| in the pipeline and elsewhere | %d | %.2f |" % (ca["other_dispatches"], ca["other_avg_us"])]
    lines += ["", "## HBM bytes per dispatch (FETCH_SIZE, WRITE_SIZE)", "",
              "Calibration: the int32->float32 copy of 2^26 elements reads and writes 262144 KiB; its "
              "FETCH_SIZE reads %.1f KiB and WRITE_SIZE %.1f KiB, so the factors are %.4f (fetch) and "
              "%.4f (write)." % ((CALIB_BYTES / 1024) / f_fac, (CALIB_BYTES / 1024) / w_fac, f_fac, w_fac), "",
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
                     "traffic_bytes_per_launch %.0f\nback_to_back_avg_us %.3f\n" % (
                         chosen[0], source_hash(), chosen[1], chosen[2], chosen[1] + chosen[2],
                         ca["longest_run_avg_us"]))
    return chosen, ca


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


VALU_PEAK = 256 * 4 * 16 * 2.4e9  # 32-bit lane-ops/s: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz


def main_grids(db: str):
    """(kernel short name) -> its largest grid size in a kernel trace."""
    top = {}
    for name, _us, grid in dispatches(db):
        top[name] = max(top.get(name, 0), grid or 0)
    return top


def main_grid_durations(db: str):
    """(kernel short name) -> average duration (us) of its dispatches at its
    largest grid."""
    by = collections.defaultdict(list)
    for name, us, grid in dispatches(db):
        by[name].append((grid, us))
    out = {}
    for name, v in by.items():
        g = max(x for x, _u in v)
        sel = [u for x, u in v if x == g]
        out[name] = sum(sel) / len(sel)
    return out


def counter_grids(db: str):
    """(kernel short name) -> its largest grid size among counter records
    (empty if this rocprofv3 version does not record grid sizes)."""
    c = sqlite3.connect(db).cursor()
    cols = [r[1] for r in c.execute("pragma table_info(counters_collection)")]
    if "grid_size" not in cols:
        return {}
    top = {}
    for name, g in c.execute("select kernel_name, grid_size from counters_collection"):
        k = short_name(name)
        top[k] = max(top.get(k, 0), g or 0)
    return top


def _main_grid_rows(db: str, short: bool = True):
    """(kernel short name, counter name, value) of every counter record of
    each kernel's dispatches at that kernel's largest grid (the bench's main
    workload; the batch's per-vector launches and the sweep run the same
    kernels on smaller grids).  `short=False` keeps the full kernel names."""
    c = sqlite3.connect(db).cursor()
    cols = [r[1] for r in c.execute("pragma table_info(counters_collection)")]
    if "grid_size" in cols:
        rows = list(c.execute("select kernel_name, counter_name, value, grid_size from counters_collection"))
    else:
        rows = [(a, b, v, 0) for (a, b, v) in c.execute("select kernel_name, counter_name, value "
                                                          "from counters_collection")]
    top = collections.defaultdict(int)
    for name, _cn, _v, g in rows:
        top[short_name(name)] = max(top[short_name(name)], g or 0)
    return [(short_name(n) if short else n, cn, v) for (n, cn, v, g) in rows
            if (g or 0) == top[short_name(n)]]


def counter_by_name(db: str, counter: str):
    """(kernel short name) -> list of per-dispatch values of one counter, at
    each kernel's largest grid."""
    d = collections.defaultdict(list)
    for name, cname, val in _main_grid_rows(db):
        if cname == counter:
            d[name].append(val)
    return d


def _gates(kernel: str):
    """Gate count per 32 elements of a bench circuit kernel, from its template
    arguments: k_binop<E, M, RZ, OPC, R> or k_chain2<E, M, RZ, O1, O2, R>."""
    from . import bfp
    m = re.match(r"bfp::k_(binop|chain2)<(.*)>$", kernel)
    if not m:
        return None
    args = [x.strip() for x in m.group(2).split(",")]
    e, mm, rz = int(args[0]), int(args[1]), 1 if args[2] == "true" else 0
    op_of = {0: "add", 1: "mul", 2: "div"}
    f = bfp.fmt(e, mm, rz)
    if m.group(1) == "binop":
        return bfp.bfp_gate_count(op_of[int(args[3])], f)
    return bfp.bfp_gate_count(op_of[int(args[3])], f) + bfp.bfp_gate_count(op_of[int(args[4])], f)


def valu_summary(trace_db, pmc_db, n, out, commands):
    """Measured VALU instructions (SQ_INSTS_VALU) of the circuit kernels next
    to their gate counts: instructions issued per 32 elements against gates
    per 32 elements, and the VALU utilisation the instruction count implies
    at the kernel-trace duration."""
    stats = main_grid_durations(trace_db)
    insts = counter_by_name(pmc_db, "SQ_INSTS_VALU")
    # Only kernels whose counted launches ran the n-element workload: a
    # kernel that the counter pass launched on a smaller grid than the trace
    # (the format sweep is skipped there) would be divided by the wrong n.
    tgrid, cgrid = main_grids(trace_db), counter_grids(pmc_db)
    lines = ["# rocprofv3 VALU summary: %s" % os.path.basename(out), "",
             "Kernel sources hash: `%s`" % source_hash(), "",
             "Commands (run from the repository root on one MI355X):", ""]
    for k, v in commands.items():
        lines.append("- %s: `%s`" % (k, v))
    lines += ["", "n = %d elements per launch; a wave64 VALU instruction is 64 lane-ops; peak %.3g lane-ops/s."
              % (n, VALU_PEAK), "",
              "| kernel | dispatches | VALU instr / dispatch | lane-instr / 32 elem | gates / 32 elem | "
              "instr / gate | trace avg us | VALU utilisation (instr) | gate rate / peak |",
              "|---|---|---|---|---|---|---|---|---|"]
    groups = n / 32
    for name in sorted(insts):
        g = _gates(name)
        if g is None or name not in stats:
            continue
        if cgrid and cgrid.get(name) != tgrid.get(name):
            continue
        vi = sum(insts[name]) / len(insts[name])
        per32 = vi * 64 / groups
        us = stats[name]
        util = vi * 64 / (us * 1e-6) / VALU_PEAK
        gfrac = g * groups / (us * 1e-6) / VALU_PEAK
        lines.append("| `%s` | %d | %.4g | %.0f | %d | %.2f | %.1f | %.2f | %.2f |"
                     % (name, len(insts[name]), vi, per32, g, per32 / g, us, util, gfrac))
    with open(out + ".md", "w") as fp:
        fp.write("\n".join(lines) + "\n")


CLOCK_KERNEL = "k_wave_clock"  # one-wave calibration kernel (bfp_wave_clock)


def wave_cycle_unit(trace_db, pmc_db, clock_hz=2.4e9):
    """Shader cycles per count of SQ_WAVE_CYCLES, from the one-wave
    calibration kernel: its traced duration at `clock_hz` over its counter
    value.  Returns (unit, measured ratio, dispatches) or None when either
    database lacks the kernel.  The unit is the ratio rounded to the nearest
    power of two when within 5% of it (the counter counts whole cycles or
    groups of cycles), else the ratio itself."""
    us = [u for name, u, _g in dispatches(trace_db) if CLOCK_KERNEL in name]
    wc = [v for name, cn, v in _main_grid_rows(pmc_db) if CLOCK_KERNEL in name and cn == "SQ_WAVE_CYCLES"]
    if not us or not wc:
        return None
    ratio = (sum(us) / len(us)) * 1e-6 * clock_hz / (sum(wc) / len(wc))
    unit = ratio
    for p2 in (1, 2, 4, 8, 16):
        if abs(ratio / p2 - 1) < 0.05:
            unit = float(p2)
    return unit, ratio, len(wc)


def sq_summary(trace_db, pmc_db, kernels, out, commands, cycle_unit=None, clock_hz=2.4e9, cus=256):
    """Per-dispatch averages of the SQ counters of one --pmc pass for the
    chosen kernels, with derived figures: each wave-state counter
    (SQ_WAIT_ANY, SQ_WAIT_INST_ANY, SQ_ACTIVE_INST_ANY) as a fraction of
    SQ_WAVE_CYCLES, and, when `cycle_unit` (shader cycles per count of those
    counters) is given, the mean lifetime of one wave and the mean number of
    waves resident per CU over the kernel's traced duration at `clock_hz`."""
    stats = main_grid_durations(trace_db)
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for name, cname, val in _main_grid_rows(pmc_db):
        vals[name][cname].append(val)
    calib = None
    if cycle_unit is None:
        calib = wave_cycle_unit(trace_db, pmc_db, clock_hz)
        if calib:
            cycle_unit = calib[0]
    lines = ["# rocprofv3 SQ counters: %s" % os.path.basename(out), "",
             "Kernel sources hash: `%s`" % source_hash(), "",
             "Commands (run from the repository root on one MI355X):", ""]
    for k, v in commands.items():
        lines.append("- %s: `%s`" % (k, v))
    names = sorted({cn for k in kernels for cn in vals.get(k, {})})
    fracs = [c for c in ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY") if c in names]
    derived = ["%s / WAVE_CYCLES" % c[3:] for c in fracs]
    if cycle_unit:
        derived += ["wave life us", "waves per CU"]
    lines += ["", "Per-dispatch averages at each kernel's largest grid (counters summed over the device):", ""]
    if calib:
        lines += ["Counter unit: the one-wave `%s` kernel (%d counted dispatches) lasts %.3f x its "
                  "SQ_WAVE_CYCLES count in %.2f GHz cycles, so one count is %g shader cycles."
                  % (CLOCK_KERNEL, calib[2], calib[1], clock_hz / 1e9, calib[0]), ""]
    if cycle_unit:
        lines += ["SQ_WAVE_CYCLES and the wave-state counters count units of %g shader cycles. Wave life = "
                  "SQ_WAVE_CYCLES / SQ_WAVES x %g / %.2f GHz; waves per CU = SQ_WAVE_CYCLES x %g / (trace avg "
                  "x %.2f GHz) / %d CUs." % (cycle_unit, cycle_unit, clock_hz / 1e9, cycle_unit, clock_hz / 1e9,
                                             cus), ""]
    lines += ["| kernel | dispatches | " + " | ".join(names) + " | " + " | ".join(derived) + " | trace avg us |",
              "|---|---|" + "---|" * len(names) + "---|" * len(derived) + "---|"]
    for k in kernels:
        if k not in vals:
            continue
        d = vals[k]
        avg = {cn: sum(v) / len(v) for cn, v in d.items()}
        nd = max(len(v) for v in d.values())
        wc = avg.get("SQ_WAVE_CYCLES")
        us = stats.get(k, float("nan"))
        row = ["%.2f" % (avg[c] / wc) if wc else "nan" for c in fracs]
        if cycle_unit:
            row.append("%.2f" % (wc / avg["SQ_WAVES"] * cycle_unit / clock_hz * 1e6)
                       if wc and avg.get("SQ_WAVES") else "nan")
            row.append("%.1f" % (wc * cycle_unit / (us * 1e-6 * clock_hz) / cus) if wc and us == us else "nan")
        lines.append("| `%s` | %d | " % (k, nd) + " | ".join("%.4g" % avg.get(cn, float("nan")) for cn in names)
                     + " | " + " | ".join(row) + " | %.2f |" % us)
    with open(out + ".md", "w") as fp:
        fp.write("\n".join(lines) + "\n")


def tick_bursts(trace_db, kernel="k_batch", gap_ns=20e6):
    """Dispatches of `kernel` in a kernel trace, split into bursts wherever
    no such dispatch runs for `gap_ns` (the serving bench's separate runs).
    Per burst: dispatches, window (first start to last end), the share of
    the window in which at least one dispatch ran, and dispatch durations."""
    rows = []
    c = sqlite3.connect(trace_db).cursor()
    for name, start, end in c.execute("select name, start, end from kernels order by start"):
        if kernel in name:
            rows.append((start, end))
    bursts, cur = [], []
    for s_, e_ in rows:
        if cur and s_ - max(e for _s, e in cur) > gap_ns:
            bursts.append(cur)
            cur = []
        cur.append((s_, e_))
    if cur:
        bursts.append(cur)
    out = []
    for bu in bursts:
        t0, t1 = bu[0][0], max(e for _s, e in bu)
        busy, last = 0, t0
        for s_, e_ in sorted(bu):
            if e_ <= last:
                continue
            busy += e_ - max(s_, last)
            last = e_
        durs = sorted((e_ - s_) / 1e3 for s_, e_ in bu)
        out.append({"dispatches": len(bu), "window_ms": (t1 - t0) / 1e6,
                    "busy_frac": busy / (t1 - t0) if t1 > t0 else float("nan"),
                    "median_us": durs[len(durs) // 2], "p90_us": durs[int(len(durs) * 0.9)]})
    return out


def ticks_summary(trace_db, out, commands, labels=()):
    lines = ["# rocprofv3 serving ticks: %s" % os.path.basename(out), "",
             "Kernel sources hash: `%s`" % source_hash(), "",
             "Commands (run from the repository root on one MI355X):", ""]
    for k, v in commands.items():
        lines.append("- %s: `%s`" % (k, v))
    lines += ["", "Persistent batch kernels of the serving bench, one burst per run (runs are separated by more "
              "than 20 ms without a batch kernel); busy = share of the burst's window in which a batch kernel "
              "ran on the device.", "",
              "| run | ticks | window ms | device busy | tick median us | tick p90 us |", "|---|---|---|---|---|---|"]
    for i, b in enumerate(tick_bursts(trace_db)):
        name = labels[i] if i < len(labels) else "run %d" % i
        lines.append("| %s | %d | %.2f | %.1f%% | %.1f | %.1f |" % (name, b["dispatches"], b["window_ms"],
                                                                 100 * b["busy_frac"], b["median_us"], b["p90_us"]))
    with open(out + ".md", "w") as fp:
        fp.write("\n".join(lines) + "\n")


def main(argv=None):
    import sys
    if argv is None:
        argv = sys.argv[1:]
    if argv and argv[0] == "ticks":
        ap = argparse.ArgumentParser()
        ap.add_argument("--trace", required=True)
        ap.add_argument("--out", required=True)
        ap.add_argument("--command-trace", default="")
        ap.add_argument("--label", action="append", default=[])
        a = ap.parse_args(argv[1:])
        ticks_summary(a.trace, a.out, {"trace": a.command_trace}, a.label)
        return 0
    if argv and argv[0] == "sq":
        ap = argparse.ArgumentParser()
        ap.add_argument("--trace", required=True)
        ap.add_argument("--pmc", required=True)
        ap.add_argument("--kernel", action="append", required=True)
        ap.add_argument("--out", required=True)
        ap.add_argument("--command-trace", default="")
        ap.add_argument("--command-pmc", default="")
        ap.add_argument("--cycle-unit", type=float, default=None,
                        help="shader cycles per SQ_WAVE_CYCLES count; by default measured from the one-wave "
                             "k_wave_clock kernel when both databases hold it (bench.py --calibrate-cycles)")
        a = ap.parse_args(argv[1:])
        sq_summary(a.trace, a.pmc, a.kernel, a.out, {"trace": a.command_trace, "SQ counters": a.command_pmc},
                   cycle_unit=a.cycle_unit)
        return
    if argv and argv[0] == "valu":
        ap = argparse.ArgumentParser()
        ap.add_argument("--trace", required=True)
        ap.add_argument("--pmc", required=True)
        ap.add_argument("--n", type=int, default=1 << 26)
        ap.add_argument("--out", required=True)
        ap.add_argument("--command-trace", default="")
        ap.add_argument("--command-pmc", default="")
        a = ap.parse_args(argv[1:])
        valu_summary(a.trace, a.pmc, a.n, a.out, {"trace": a.command_trace, "SQ_INSTS_VALU": a.command_pmc})
        return
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
