"""Benchmark: bitslice custom-precision FP on one MI355X.

Workload (default): 2^26-element vectors in (5,10) and (8,7), operands
N(0,1) * 2^U(-8,8) mapped to the format, 64-element lane words,
round-to-nearest-even.  One step is the whole hot path for both formats:
pack both operands (standard -> bitslice), add, sub and mul on the resident
bitslice vectors, unpack the three results.  ``value`` counts elementwise
operations (2 formats x 3 ops x 2^26 elements per step) per second with the
inputs already in HBM.

The headline workload fixes 64-element lane words (two 32-bit words per
lane) for its add/sub/mul launches, as the workload prescribes, instead of
the tuned table's choice; every other section uses the tuned table.

Also printed in the same JSON line:
  roofline      the dominant kernel (largest share of the step) against
                MI355X's peak (HBM 8 TB/s, or the bitwise VALU rate), and
                against the box's own measured ceiling (best read, write and
                copy sweeps over 1 GiB); its duration comes from a cold pass:
                the same steps with a 1 GiB read sweep (outside the events)
                before each group of launches of one kernel, and HIP events
                around the group on the kernels' stream;
  kernels       every kernel's mean duration and rates, cold as above, and
                cache-assisted (``*_cache_assisted``: the same steps with
                events around each group but no sweep, so a kernel may read
                what the previous one left in the 256 MB last-level cache);
  sweep         the 40-format sweep: add and mul on 2^24 elements per format,
                tuned launches, each launch timed cold (median of 5);
  layout_methods pack and unpack with each transpose method (per lane,
                across lanes) for 1-, 2- and 4-byte containers, cold;
  batched       4096 mixed vectors: one persistent launch vs one launch per
                vector, the per-vector launches also replayed from a captured
                graph (skipped with --no-batched);
  serving       the serving loop at saturation (lowest of three runs) and at
                Poisson loads of 0.5 and 0.9 of it and of a fixed 5e5
                requests/s (skipped with --no-serving);
  div           division (Table 1, Div) on resident bitslice vectors of the
                same size and formats, the launch table's configuration:
                elements/s and its bitwise VALU rate against peak;
  wide          binary64 (11,52) add, mul and div on resident bitslice
                vectors of the same size (tuned one-word kernels);
  int           k-bit integer vectors (k = 5, 9, 13), 2^26 elements: wrapping
                add and mul, signed-saturating mul;
  chain         d = a*b + c on the same vectors: one two-op chain kernel
                (intermediate in registers, 4 vectors through HBM) against
                the two separate launches (6 vectors);
  small         the 65,536-element (5,2) workload (launch-latency bound): the
                fused standard-in/standard-out add, and pack + add + unpack
                as four launches, microseconds per call;
  cpu_baseline  the oracle timed on this host on a bounded sample (threads
                and one thread), with the CPU model.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12                      # bytes/s
VALU_PEAK = 256 * 4 * 16 * 2.4e9       # 32-bit lane-ops/s: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz
FORMATS = [(5, 10), (8, 7)]
OPS = ["add", "sub", "mul"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--settle-ms", type=float, default=100.0,
                    help="untimed device time of steps run before the warmup steps")
    ap.add_argument("--n-log2", type=int, default=26)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one int32->float32 conversion of 2^26 elements (256 MiB read, 256 MiB "
                         "written) so hardware byte counters can be scaled against a kernel of known traffic")
    ap.add_argument("--calibrate-cycles", action="store_true",
                    help="also run the one-wave bfp_wave_clock kernel (400,000 dependent FMAs) so per-wave "
                         "cycle counters can be set against its traced duration")
    ap.add_argument("--batched-reps", type=int, default=10)
    ap.add_argument("--batched-no-graph", action="store_true",
                    help="time the batch's kernels launched directly only (no graph replays), e.g. under counters")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-div", action="store_true")
    ap.add_argument("--no-chain", action="store_true")
    ap.add_argument("--no-int", action="store_true")
    ap.add_argument("--no-wide", action="store_true")
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-layout-methods", action="store_true")
    ap.add_argument("--sweep-n-log2", type=int, default=24)
    ap.add_argument("--div-reps", type=int, default=10)
    ap.add_argument("--serving-requests", type=int, default=20000)
    return ap.parse_args()


def settle(torch, fn, stream, ms=50.0):
    """Run fn back to back, untimed, until `ms` of device time have passed:
    the measurement that follows then sees the clocks the GPU sustains under
    that work, not its ramp from the idle stretches in which the host
    generates inputs."""
    done = 0.0
    for _ in range(100000):  # bounded, in case fn does no device work
        if done >= ms:
            break
        ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ea.record(stream)
        for _ in range(4):
            fn()
        eb.record(stream)
        torch.cuda.synchronize()
        done += ea.elapsed_time(eb)


def bench_batched(torch, bfp, dev, reps, graphs=True):
    """4096 vectors, lengths log-uniform in [1024, 2^20], random format of the
    40-format sweep and random op: one graph launch of the persistent kernel
    vs one launch per vector (both timed with events on one stream, after an
    untimed warm-up, each the lower of two measurements taken in turn)."""
    import numpy as np

    from paper_1602_04716_amd import inputs, workloads
    specs = inputs.batch_tasks(4096, seed=4)
    bt = workloads.build_batch(specs, seed=4, device=dev)
    plan = bfp.BatchPlan(bt.tasks)
    stream = torch.cuda.current_stream()
    ops_alg = 0.0
    for (n, e, m, op, rnd) in bt.specs:
        ops_alg += bfp.bfp_gate_count(op, bfp.fmt(e, m, rnd)) * ((n + 31) // 32)

    def timed(fn):
        # the persistent kernel's own runs bring the device to its working
        # clocks first: a measurement started after a light or idle stretch
        # (the per-vector launches, host work) ran up to 4% slower
        for _ in range(reps):
            plan.run_eager(stream)
        fn()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(reps):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    def cold(fn, k=5):
        """Median of k launches, each after a 1 GiB read sweep outside the events."""
        fn()
        ts = []
        for _ in range(k):
            bfp.bfp_flush_llc(1 << 30, stream)
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            fn()
            ev1.record(stream)
            torch.cuda.synchronize()
            ts.append(ev0.elapsed_time(ev1))
        return float(np.median(ts))

    # each path timed twice in turn, after a warm-up, reported by its lower time
    paths = {"eager": lambda: plan.run_eager(stream), "per_vector": lambda: plan.run_per_vector(stream)}
    if graphs:
        paths["graph"] = lambda: plan.run(stream)
        paths["per_vector_graph"] = lambda: plan.run_per_vector_graph(stream)
    best = {}
    for _round in range(2):
        for name, fn in paths.items():
            best[name] = min(best.get(name, float("inf")), timed(fn))
    e_ms, v_ms = best["eager"], best["per_vector"]
    if graphs:
        g_ms, vg_ms = best["graph"], best["per_vector_graph"]
        g_cold = cold(lambda: plan.run(stream))
        vg_cold = cold(lambda: plan.run_per_vector_graph(stream))
    else:  # the same kernels launched directly stand in for the graph figures
        g_ms = e_ms
        vg_ms = v_ms
        g_cold = cold(lambda: plan.run_eager(stream))
        vg_cold = cold(lambda: plan.run_per_vector(stream), k=1)
    info = plan.info()
    plan.close()
    nbytes = bt.bytes_moved()
    elems = bt.elements()
    return {"tasks": len(bt.specs), "elements": elems, "bytes": nbytes, "chunks": info["chunks"],
            "grid": info["grid"], "graph_ms": g_ms, "eager_persistent_ms": e_ms, "per_vector_ms": v_ms,
            "per_vector_graph_ms": vg_ms, "graph_ms_cold": g_cold, "per_vector_graph_ms_cold": vg_cold,
            "speedup_vs_per_vector": v_ms / g_ms, "speedup_vs_per_vector_graph": vg_ms / g_ms,
            "elements_per_s": elems / (g_ms * 1e-3),
            "per_vector_elements_per_s": elems / (v_ms * 1e-3),
            "per_vector_graph_elements_per_s": elems / (vg_ms * 1e-3),
            "hbm_frac": nbytes / (g_ms * 1e-3) / HBM_PEAK, "valu_frac": ops_alg / (g_ms * 1e-3) / VALU_PEAK,
            "hbm_frac_cold": nbytes / (g_cold * 1e-3) / HBM_PEAK,
            "per_vector_graph_hbm_frac": nbytes / (vg_ms * 1e-3) / HBM_PEAK}


def bench_serving(torch, bfp, dev, n_req):
    """Serving loop: resident pool of two 2^22-element vectors per format of
    the 40-format sweep, requests with n = 2^U(10,22), random format and op,
    64 GB budget.  After 2000 warm-up requests, saturation throughput from
    three runs with all requests submitted at once; mu is the lowest of the
    three (a rate the server sustained every time, so that 0.9 mu stays below
    saturation on every run).  Then Poisson arrivals at 0.5 mu and 0.9 mu,
    and at a fixed 5e5 requests/s for comparison across machines (1000
    warm-up requests not counted), p50/p99 of completion minus submission.
    Arrivals are submitted from native code (bfp_server_replay); results are
    freed by the server as they complete."""
    from paper_1602_04716_amd import inputs, serving
    fmts = inputs.sweep_formats()
    srv = serving.Server(64 << 30, 4096)
    pool = serving.build_pool(srv, fmts, 1 << 22, seed=5, device=dev)
    serving.run_native(srv, pool, serving.request_stream(2000, fmts, seed=49))
    sats = [serving.run_native(srv, pool, serving.request_stream(n_req, fmts, seed=50 + i)) for i in range(3)]
    mus = [r["requests_per_s"] for r in sats]
    mu = min(mus)
    med = sorted(sats, key=lambda r: r["requests_per_s"])[1]
    out = {"budget_bytes": 64 << 30, "slots": 4096, "pool_bytes": srv.stats()["used"], "mu": mu,
           "saturation": dict({k: med[k] for k in ("requests", "requests_per_s", "elements_per_s", "p50_us",
                                                   "p99_us")}, runs_requests_per_s=mus)}
    keys = ("rate", "requests", "requests_per_s", "elements_per_s", "p50_us", "p99_us", "mean_us", "errors",
            "queue_p50_us", "queue_p99_us", "device_p50_us", "device_p99_us", "slowest1pct_queue_us",
            "slowest1pct_device_us")
    for name, rate, seed in (("lambda_0.5_mu", 0.5 * mu, 65), ("lambda_0.9_mu", 0.9 * mu, 69),
                             ("rate_5e5", 5e5, 75)):
        r = serving.run_native(srv, pool, serving.request_stream(n_req + 1000, fmts, seed=seed),
                               rate=rate, seed=7, skip=1000)
        out[name] = {k: r[k] for k in keys}
    st = srv.stats()
    out["high_water_bytes"] = st["high_water"]
    out["ticks"] = st["ticks"]
    out["max_tick_requests"] = st["max_tick_requests"]
    out["max_inflight_ticks"] = st["max_inflight_ticks"]
    srv.close()
    return out


def bench_div(torch, bfp, dev, n, reps):
    """Division on resident bitslice vectors of n elements per bench format,
    round to nearest even, launch configuration from the tuned table; the
    event pair brackets `reps` back-to-back launches on the launch stream."""
    from paper_1602_04716_amd import inputs
    s = torch.cuda.current_stream()
    out = {}
    for (e, m) in FORMATS:
        f = bfp.fmt(e, m)
        B = 1 + e + m
        a = torch.from_numpy(inputs.scaled_normal(e, m, n, 2)).to(dev)
        b = torch.from_numpy(inputs.scaled_normal(e, m, n, 3)).to(dev)
        pa, pb = bfp.pack(f, a), bfp.pack(f, b)
        pc = bfp.empty_bitslice(f, n, dev)
        del a, b
        settle(torch, lambda: bfp.bfp_div(f, pa, pb, pc, n, s), s)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(s)
        for _ in range(reps):
            bfp.bfp_div(f, pa, pb, pc, n, s)
        ev1.record(s)
        torch.cuda.synchronize()
        us = ev0.elapsed_time(ev1) * 1e3 / reps
        G = bfp.bfp_gate_count("div", f)
        cfg = bfp.bfp_launch_get("div", f)
        ops_s = G * n / 32 / (us * 1e-6)
        bytes_s = 3 * B / 8 * n / (us * 1e-6)
        out["(%d,%d)" % (e, m)] = {
            "us": us, "elements_per_s": n / (us * 1e-6), "gates": G, "Tops/s": ops_s / 1e12,
            "valu_frac": ops_s / VALU_PEAK, "GB/s": bytes_s / 1e9, "hbm_frac": bytes_s / HBM_PEAK,
            "device_kernel": "bfp::k_binop<%d, %d, false, 2, %d, %d>" % (e, m, cfg.words_per_lane, max(1, cfg.unroll)),
            "block": cfg.block, "blocks_per_cu": cfg.blocks_per_cu}
        del pa, pb, pc
    out["timing"] = "back to back on the same buffers, warm: inputs partly cache-resident (working set near the 256 MB last-level cache), so rates are cache-assisted; the cold figures are in kernels, sweep and roofline"
    return out


def bench_chain(torch, bfp, dev, n, reps):
    """d = a*b + c per bench format, nearest-even: the fused chain kernel vs
    bfp_mul + bfp_add into a temporary, each timed over `reps` back-to-back
    repetitions between two events on the launch stream."""
    from paper_1602_04716_amd import inputs
    s = torch.cuda.current_stream()
    out = {}
    for (e, m) in FORMATS:
        f = bfp.fmt(e, m)
        B = 1 + e + m
        pa, pb, pc = (bfp.pack(f, torch.from_numpy(inputs.scaled_normal(e, m, n, k)).to(dev)) for k in (2, 3, 4))
        pd, pt = bfp.empty_bitslice(f, n, dev), bfp.empty_bitslice(f, n, dev)

        def fused():
            bfp.bfp_chain2("mul", "add", f, pa, pb, pc, pd, n, s)

        def separate():
            bfp.bfp_mul(f, pa, pb, pt, n, s)
            bfp.bfp_add(f, pt, pc, pd, n, s)

        res = {}
        for name, fn in (("fused", fused), ("separate", separate)):
            settle(torch, fn, s)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(s)
            for _ in range(reps):
                fn()
            ev1.record(s)
            torch.cuda.synchronize()
            res[name] = ev0.elapsed_time(ev1) * 1e3 / reps
        G = bfp.bfp_gate_count("mul", f) + bfp.bfp_gate_count("add", f)
        us = res["fused"]
        out["(%d,%d)" % (e, m)] = {
            "fused_us": us, "separate_us": res["separate"], "speedup": res["separate"] / us,
            "elements_per_s": n / (us * 1e-6), "GB/s": 4 * B / 8 * n / (us * 1e-6) / 1e9,
            "hbm_frac": 4 * B / 8 * n / (us * 1e-6) / HBM_PEAK,
            "valu_frac": G * n / 32 / (us * 1e-6) / VALU_PEAK,
            "device_kernel": "bfp::k_chain2<%d, %d, false, 1, 0, 1>" % (e, m)}
        del pa, pb, pc, pd, pt
    out["timing"] = "back to back on the same buffers, warm: inputs partly cache-resident (working set near the 256 MB last-level cache), so rates are cache-assisted; the cold figures are in kernels, sweep and roofline"
    return out


def bench_small(torch, bfp, dev, reps=200):
    """65,536 uniform (5,2) patterns without NaN/Inf, add to nearest even:
    the fused kernel and the three-kernel path, `reps` back-to-back calls
    between two events, each path measured twice in turn and reported by its
    lower time.  The calls are made from Python (each pays the binding's
    argument marshalling on the host) and, separately, captured once in a
    graph of `reps` calls and replayed, which leaves only the device's own
    time per call; every replay's result is compared with the eager one."""
    from paper_1602_04716_amd import inputs
    s = torch.cuda.current_stream()
    n = 65536
    f = bfp.fmt(5, 2)
    a = torch.from_numpy(inputs.plain_8bit(n, seed=1)).to(dev)
    b = torch.from_numpy(inputs.plain_8bit(n, seed=101)).to(dev)
    c = torch.empty_like(a)
    pa, pb, pc = (bfp.empty_bitslice(f, n, dev) for _ in range(3))

    def fused(st):
        bfp.bfp_binop_std("add", f, a, b, c, n, st)

    def three(st):
        bfp.bfp_pack(f, a, pa, n, st)
        bfp.bfp_pack(f, b, pb, n, st)
        bfp.bfp_add(f, pa, pb, pc, n, st)
        bfp.bfp_unpack(f, pc, c, n, st)

    paths = (("fused", fused), ("pack_add_unpack", three))
    graphs, want, graph_error = {}, {}, None
    for name, fn in paths:
        fn(s)
        torch.cuda.synchronize()
        want[name] = c.clone()
        try:
            cs = torch.cuda.Stream()
            cs.wait_stream(s)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=cs):
                for _ in range(reps):
                    fn(cs)
            torch.cuda.synchronize()
            graphs[name] = g
        except RuntimeError as exc:  # the eager figures stand without the graph ones
            graph_error = "capture of the %s path failed: %s" % (name, exc)
            graphs.clear()
            break

    def timed(run):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(s)
        run()
        ev1.record(s)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) * 1e3 / reps

    out = {"n": n, "format": "(5,2)"}
    best = {}
    for _round in range(2):
        for name, fn in paths:
            settle(torch, lambda: fn(s), s, ms=20.0)
            us = timed(lambda: [fn(s) for _ in range(reps)])
            best[name] = min(best.get(name, us), us)
            if name not in graphs:
                continue
            c.zero_()
            us = timed(graphs[name].replay)
            if not torch.equal(c, want[name]):
                graph_error = "graph replay of the %s path differs from its eager result" % name
                graphs.clear()
                continue
            best[name + "_graph"] = min(best.get(name + "_graph", us), us)
    for name in ("fused", "pack_add_unpack"):
        out[name + "_us"] = best[name]
        out[name + "_elements_per_s"] = n / (best[name] * 1e-6)
        if graph_error is None:
            out[name + "_graph_us"] = best[name + "_graph"]
            out[name + "_graph_elements_per_s"] = n / (best[name + "_graph"] * 1e-6)
    if graph_error is not None:
        out["graph_error"] = graph_error
    return out


def bench_wide(torch, bfp, dev, n, reps):
    """binary64 elementwise ops on resident bitslice vectors of n elements,
    RNE, the launch table's configuration, `reps` launches between events."""
    import numpy as np
    s = torch.cuda.current_stream()
    e, m = 11, 52
    f = bfp.fmt(e, m)
    rng = np.random.default_rng(11)
    pa, pb = (bfp.pack(f, torch.from_numpy(rng.standard_normal(n)).to(dev).view(torch.uint64)) for _ in range(2))
    pc = bfp.empty_bitslice(f, n, dev)
    out = {}
    for op in ("add", "mul", "div"):
        settle(torch, lambda: bfp.bfp_binop(op, f, pa, pb, pc, n, s), s)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(s)
        for _ in range(reps):
            bfp.bfp_binop(op, f, pa, pb, pc, n, s)
        ev1.record(s)
        torch.cuda.synchronize()
        us = ev0.elapsed_time(ev1) * 1e3 / reps
        G = bfp.bfp_gate_count(op, f)
        cfg = bfp.bfp_launch_get(op, f)
        ops_s = G * n / 32 / (us * 1e-6)
        bytes_s = 3 * 64 / 8 * n / (us * 1e-6)
        out["%s(11,52)" % op] = {"us": us, "elements_per_s": n / (us * 1e-6), "gates": G,
                                 "valu_frac": ops_s / VALU_PEAK, "hbm_frac": bytes_s / HBM_PEAK,
                                 "block": cfg.block, "blocks_per_cu": cfg.blocks_per_cu}
    del pa, pb, pc
    out["timing"] = "back to back on the same buffers, warm: inputs partly cache-resident (working set near the 256 MB last-level cache), so rates are cache-assisted; the cold figures are in kernels, sweep and roofline"
    return out


def bench_int(torch, bfp, dev, n, reps):
    """k-bit integer ops on resident bitslice vectors of n elements, timed
    over `reps` back-to-back launches between two events."""
    import numpy as np
    s = torch.cuda.current_stream()
    out = {}
    for k in (5, 9, 13):
        rng = np.random.default_rng(k)
        dt = np.uint8 if k <= 8 else np.uint16
        pa, pb = (bfp.int_pack(k, torch.from_numpy(rng.integers(0, 1 << k, n, dtype=np.uint64).astype(dt)).to(dev))
                  for _ in range(2))
        pc = bfp.int_empty_bitslice(k, n, dev)
        for op, kind in (("add", "wrap"), ("mul", "wrap"), ("mul", "sats")):
            settle(torch, lambda: bfp.bfp_int_binop(op, k, kind, pa, pb, pc, n, s), s)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(s)
            for _ in range(reps):
                bfp.bfp_int_binop(op, k, kind, pa, pb, pc, n, s)
            ev1.record(s)
            torch.cuda.synchronize()
            us = ev0.elapsed_time(ev1) * 1e3 / reps
            nbytes = 3 * k / 8 * n
            out["%s_%s_k%d" % (op, kind, k)] = {
                "us": us, "elements_per_s": n / (us * 1e-6), "GB/s": nbytes / (us * 1e-6) / 1e9,
                "hbm_frac": nbytes / (us * 1e-6) / HBM_PEAK}
        del pa, pb, pc
    out["timing"] = "back to back on the same buffers, warm: inputs partly cache-resident (working set near the 256 MB last-level cache), so rates are cache-assisted; the cold figures are in kernels, sweep and roofline"
    return out


def bench_sweep(torch, bfp, dev, n_log2, reps=5):
    """The 40-format sweep: add and mul (nearest-even) on 2^n_log2 elements
    per format, operands log-uniform over the normal range plus 1% subnormals
    and zeros, the tuned launch table's configuration; each launch is timed
    between events after a 1 GiB read sweep (the 6B MiB working set would
    otherwise sit in the 256 MB last-level cache), median of `reps`, after
    20 ms of untimed launches of the same kernel."""
    import numpy as np

    from paper_1602_04716_amd import inputs
    s = torch.cuda.current_stream()
    n = 1 << n_log2
    out = {"n": n, "formats": {}}
    tot_el, tot_t = 0.0, 0.0
    for (e, m) in inputs.sweep_formats():
        f = bfp.fmt(e, m)
        B = 1 + e + m
        # a 2^20-element draw repeated to n (the circuits' time does not depend on the values)
        k = min(n, 1 << 20)
        xa = torch.from_numpy(inputs.sweep_operands(e, m, k, 100 + e * 32 + m)).to(dev).repeat((n + k - 1) // k)
        xb = torch.from_numpy(inputs.sweep_operands(e, m, k, 200 + e * 32 + m)).to(dev).repeat((n + k - 1) // k)
        pa = bfp.pack(f, xa[:n].contiguous())
        pb = bfp.pack(f, xb[:n].contiguous())
        del xa, xb
        pc = bfp.empty_bitslice(f, n, dev)
        row = {}
        for op in ("add", "mul"):
            settle(torch, lambda: bfp.bfp_binop(op, f, pa, pb, pc, n, s), s, ms=20.0)
            ts = []
            for _ in range(reps):
                bfp.bfp_flush_llc(1 << 30, s)
                ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                ev0.record(s)
                bfp.bfp_binop(op, f, pa, pb, pc, n, s)
                ev1.record(s)
                torch.cuda.synchronize()
                ts.append(ev0.elapsed_time(ev1) * 1e3)
            us = float(np.median(ts))
            G = bfp.bfp_gate_count(op, f)
            cfg = bfp.bfp_launch_get(op, f)
            row[op] = {"us": us, "elements_per_s": n / (us * 1e-6),
                       "hbm_frac": 3 * B / 8 * n / (us * 1e-6) / HBM_PEAK,
                       "valu_frac": G * n / 32 / (us * 1e-6) / VALU_PEAK,
                       "words_per_lane": cfg.words_per_lane, "block": cfg.block}
            tot_el += n
            tot_t += us
        out["formats"]["(%d,%d)" % (e, m)] = row
        del pa, pb, pc
    out["elements_per_s_all"] = tot_el / (tot_t * 1e-6)
    fr = [r[op]["hbm_frac"] for r in out["formats"].values() for op in r]
    vf = [r[op]["valu_frac"] for r in out["formats"].values() for op in r]
    out["bound_frac_median"] = float(np.median([max(a, b) for a, b in zip(fr, vf)]))
    out["bound_frac_min"] = float(min(max(a, b) for a, b in zip(fr, vf)))
    return out


def bench_layout_methods(torch, bfp, dev, n, reps=5):
    """Pack and unpack with each transpose method (per lane, across lanes)
    for 1-, 2- and 4-byte containers ((4,3), (5,10), (8,23)) on n elements,
    each launch timed cold (1 GiB read sweep first), median of `reps`."""
    import numpy as np
    s = torch.cuda.current_stream()
    out = {}
    for (e, m) in ((4, 3), (5, 10), (8, 23)):
        f = bfp.fmt(e, m)
        cb = bfp.bfp_container_bytes(f)
        B = 1 + e + m
        x = torch.randint(0, 1 << min(B, 31), (n,), dtype=torch.int64, device=dev).to(bfp.container_dtype(f))
        bs = bfp.empty_bitslice(f, n, dev)
        y = torch.empty_like(x)
        row = {}
        for meth, name in ((bfp.BFP_TRANSPOSE_LANE, "lane"), (bfp.BFP_TRANSPOSE_XLANE, "xlane")):
            for d, fn in (("pack", lambda: bfp.bfp_pack(f, x, bs, n, s)), ("unpack", lambda: bfp.bfp_unpack(f, bs, y, n, s))):
                bfp.bfp_layout_method_set(d, cb, meth)
                fn()
                ts = []
                for _ in range(reps):
                    bfp.bfp_flush_llc(1 << 30, s)
                    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    ev0.record(s)
                    fn()
                    ev1.record(s)
                    torch.cuda.synchronize()
                    ts.append(ev0.elapsed_time(ev1) * 1e3)
                us = float(np.median(ts))
                nbytes = n * (cb + B / 8)
                row["%s_%s_us" % (d, name)] = us
                row["%s_%s_hbm_frac" % (d, name)] = nbytes / (us * 1e-6) / HBM_PEAK
        for d in ("pack", "unpack"):
            bfp.bfp_layout_method_set(d, cb, bfp.BFP_TRANSPOSE_LANE)
        out["(%d,%d)" % (e, m)] = row
        del x, y, bs
    return out


def device_kernel(label):
    """Device kernel that a bench label ("unpack(8,7)", "mul(5,10)") launches
    with the bench's configuration (64-element lane words, nearest-even)."""
    kind, _, fm = label.partition("(")
    e, m = (int(x) for x in fm.rstrip(")").split(","))
    B = 1 + e + m
    C = 1 if B <= 8 else (2 if B <= 16 else 4)
    if kind == "pack":
        return "bfp::k_pack<%d>" % C
    if kind == "unpack":
        return "bfp::k_unpack<%d>" % C
    return "bfp::k_binop<%d, %d, false, %d, 2, 1>" % (e, m, {"add": 0, "sub": 0, "mul": 1, "div": 2}[kind])


def committed_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summaries (profiles/*.traffic.txt), or None if there is none for the
    current kernel sources."""
    import glob

    from paper_1602_04716_amd import profiling
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.traffic.txt"))):
        t = profiling.read_traffic(path)
        if t and t["kernel"] == kernel:
            return t["bytes"]
    return None


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sample_log2=24, single_log2=22):
    """The oracle on a bounded sample of the same workload: 2^24 elements per
    (format, op), all 6 combinations, on this host's cores; and 2^22 per
    combination on one thread."""
    import numpy as np

    import oracle
    from paper_1602_04716_amd import inputs
    oracle.build()
    threads = max(1, min(os.cpu_count() or 1, 64))

    def timed(n, nthreads):
        total, elapsed = 0, 0.0
        for (e, m) in FORMATS:
            a = inputs.scaled_normal(e, m, n, 2)
            b = inputs.scaled_normal(e, m, n, 3)
            for op in OPS:
                t0 = time.perf_counter()
                oracle.binop(op, e, m, 0, a, b, nthreads=nthreads)
                elapsed += time.perf_counter() - t0
                total += n
        return total / elapsed, elapsed

    v, el = timed(1 << sample_log2, threads)
    v1, el1 = timed(1 << single_log2, 1)
    return {"value": v, "unit": "elements/s", "cores": threads, "kind": "oracle",
            "sample": "2^%d elements x {(5,10),(8,7)} x {add,sub,mul}, RNE, %.1f s wall on %d threads; "
                      "2^%d per combination on 1 thread, %.1f s" % (sample_log2, el, threads, single_log2, el1),
            "single_thread_value": v1, "cpu_model": _cpu_model()}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the path has no cross-GPU step "
              "(each shard is independent); run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1602_04716_amd import bfp, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    n = 1 << args.n_log2

    data = {}
    for (e, m) in FORMATS:
        f = bfp.fmt(e, m)
        for op in OPS:
            bfp.bfp_launch_set(op, f, 2, 256, 0)  # 64-element lane words
        a = torch.from_numpy(inputs.scaled_normal(e, m, n, 2)).to(dev)
        b = torch.from_numpy(inputs.scaled_normal(e, m, n, 3)).to(dev)
        pa, pb = bfp.empty_bitslice(f, n, dev), bfp.empty_bitslice(f, n, dev)
        pc = {op: bfp.empty_bitslice(f, n, dev) for op in OPS}
        out = {op: torch.empty(n, dtype=a.dtype, device=dev) for op in OPS}
        data[(e, m)] = (f, a, b, pa, pb, pc, out)
    torch.cuda.synchronize()

    if args.calibrate_copy:
        src = torch.zeros(1 << 26, dtype=torch.int32, device=dev)
        dst = torch.empty(1 << 26, dtype=torch.float32, device=dev)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.calibrate_cycles:
        bfp.bfp_wave_clock(400000, stream)
        torch.cuda.synchronize()

    # one step = for each format: pack a, pack b, add, sub, mul, unpack x3.
    # Launches of one kernel that follow each other form a group bracketed by
    # two events on the stream the kernels run on, so per-kernel durations come
    # from the timed steps themselves (group time / launches in the group).
    groups = []  # (name, [launch fns], algorithmic bytes per launch, gate ops per launch, bytes read per launch)
    for (e, m) in FORMATS:
        f, a, b, pa, pb, pc, out = data[(e, m)]
        B = 1 + e + m
        C = bfp.bfp_container_bytes(f)
        tag = "(%d,%d)" % (e, m)
        io = n * (C + B / 8)
        groups.append(("pack" + tag, [lambda f=f, a=a, pa=pa: bfp.bfp_pack(f, a, pa, n, stream),
                                      lambda f=f, b=b, pb=pb: bfp.bfp_pack(f, b, pb, n, stream)], io, 0, n * C))
        for op in OPS:
            G = bfp.bfp_gate_count(op, f)
            groups.append((op + tag, [lambda f=f, pa=pa, pb=pb, pc=pc, op=op:
                                      bfp.bfp_binop(op, f, pa, pb, pc[op], n, stream)], n * 3 * B / 8, G * n / 32,
                           n * 2 * B / 8))
        groups.append(("unpack" + tag, [lambda f=f, pc=pc, out=out, op=op: bfp.bfp_unpack(f, pc[op], out[op], n, stream)
                                        for op in OPS], io, 0, n * B / 8))

    def step(evs=None):
        for i, (name, fns, *_r) in enumerate(groups):
            if evs is not None:
                evs[i][0].record(stream)
            for fn in fns:
                fn()
            if evs is not None:
                evs[i][1].record(stream)

    # Settle: the step runs untimed for at least --settle-ms of device time
    # before the W warmup steps, so the timed steps see the GPU at the clocks
    # it sustains under this load (after the host's input generation the
    # device has idled; with 3 warmup steps and no settle period the timed
    # steps measured 3% slower than after 50).
    settle_ms = 0.0
    for _ in range(100000):  # bounded: each pass is 10 steps of device work
        if settle_ms >= args.settle_ms:
            break
        sa = torch.cuda.Event(enable_timing=True)
        sb = torch.cuda.Event(enable_timing=True)
        sa.record(stream)
        for _ in range(10):
            step()
        sb.record(stream)
        torch.cuda.synchronize()
        settle_ms += sa.elapsed_time(sb)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region 1: K plain steps between two events -> value
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record(stream)
    for _ in range(args.steps):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = t0.elapsed_time(t1) / args.steps
    elems_per_step = len(FORMATS) * len(OPS) * n
    value = elems_per_step / (ms_step / 1e3)
    # pass 2 (cache-assisted): the same K steps with events around each
    # kernel group -> per-kernel durations in the pipeline, where a kernel may
    # read what the previous one left in the last-level cache (the event
    # packets add a little time between groups, so this pass is not used for
    # the step time)
    def instrumented(flush):
        evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                for _ in groups] for _ in range(args.steps)]
        for k in range(args.steps):
            for i, (name, fns, *_r) in enumerate(groups):
                if flush:
                    bfp.bfp_flush_llc(1 << 30, stream)
                evs[k][i][0].record(stream)
                for fn in fns:
                    fn()
                evs[k][i][1].record(stream)
        torch.cuda.synchronize()
        return evs

    evs_warm = instrumented(False)
    ms_step_instrumented = evs_warm[0][0][0].elapsed_time(evs_warm[-1][-1][1]) / args.steps
    # pass 3 (cold): a 1 GiB read sweep before each group, outside its events
    evs_cold = instrumented(True)

    kernels = {}
    for i, (name, fns, nbytes, nops, rbytes) in enumerate(groups):
        k = kernels.setdefault(name, {"launches": 0, "us_total": 0.0, "us_total_warm": 0.0, "bytes": nbytes,
                                      "ops": nops, "read_bytes": rbytes})
        for st in range(args.steps):
            k["us_total"] += evs_cold[st][i][0].elapsed_time(evs_cold[st][i][1]) * 1e3
            k["us_total_warm"] += evs_warm[st][i][0].elapsed_time(evs_warm[st][i][1]) * 1e3
            k["launches"] += len(fns)
    for name, k in kernels.items():
        for sfx, tot in (("", k["us_total"]), ("_cache_assisted", k["us_total_warm"])):
            us = tot / k["launches"]
            k["us" + sfx] = us
            k["GB/s" + sfx] = k["bytes"] / (us * 1e-6) / 1e9
            k["hbm_frac" + sfx] = k["bytes"] / (us * 1e-6) / HBM_PEAK
            if k["ops"]:
                k["Tops/s" + sfx] = k["ops"] / (us * 1e-6) / 1e12
                k["valu_frac" + sfx] = k["ops"] / (us * 1e-6) / VALU_PEAK
    # the dominant kernel: largest total (cold) time per step
    dom = max(kernels, key=lambda nm: kernels[nm]["us_total"])
    dk = kernels[dom]
    if dk.get("valu_frac", 0) > dk["hbm_frac"]:
        roof = {"kernel": dom, "bound": "alu", "achieved": dk["Tops/s"], "peak": VALU_PEAK / 1e12,
                "unit": "Tops/s", "frac": dk["valu_frac"], "traffic": None}
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": dk["GB/s"], "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": dk["hbm_frac"], "traffic": None}
    # practical ceilings on this machine: best read, write and copy sweeps over
    # 1 GiB, and a sweep that reads two 1 GiB streams and writes a third (an
    # elementwise binary op's traffic), over launch shapes from one block per
    # CU to 32 and 1 to 8 accesses in flight per lane, events on the same stream
    ceil = {mode: bfp.bfp_measure_hbm(1 << 30, mode, 5, stream)
            for mode in ("read", "write", "copy", "read2_write1")}
    roof["ceiling_GBps"] = {mode: c["GB/s"] for mode, c in ceil.items()}
    roof["ceiling_shapes"] = {mode: {"grid": c["grid"], "block": c["block"], "in_flight": c["in_flight"]}
                              for mode, c in ceil.items()}
    roof["copy_GBps"] = ceil["copy"]["GB/s"]
    if roof["unit"] == "GB/s":
        roof["frac_of_copy"] = roof["achieved"] / roof["copy_GBps"]
        # the kernel's own read/write mix at the measured read and write
        # ceilings: reading r bytes and writing w bytes takes at least
        # r / read + w / write seconds
        rd, wr = dk["read_bytes"], dk["bytes"] - dk["read_bytes"]
        mix = dk["bytes"] / (rd / (ceil["read"]["GB/s"] * 1e9) + wr / (ceil["write"]["GB/s"] * 1e9)) / 1e9
        roof["mix_ceiling_GBps"] = mix
        roof["frac_of_mix_ceiling"] = roof["achieved"] / mix
    for k in kernels.values():
        rd, wr = k["read_bytes"], k["bytes"] - k["read_bytes"]
        k["mix_ceiling_GBps"] = k["bytes"] / (rd / (ceil["read"]["GB/s"] * 1e9) + wr / (ceil["write"]["GB/s"] * 1e9)) / 1e9
        k["frac_of_mix_ceiling"] = k["GB/s"] / k["mix_ceiling_GBps"]
        # kernels with the same traffic shape as a probe, against that probe
        if abs(rd - 2 * wr) <= 1e-9 * rd:
            k["frac_of_probe"] = k["GB/s"] / ceil["read2_write1"]["GB/s"]
        elif abs(rd - wr) <= 1e-9 * rd:
            k["frac_of_probe"] = k["GB/s"] / ceil["copy"]["GB/s"]
    # the dominant kernel alone: after one 1 GiB sweep, its launches of every
    # format back to back, twice over (each launch's input was last touched
    # several launches, and more than the cache holds, earlier), so the event
    # gap spreads over many launches
    dom_kernel = device_kernel(dom)
    dom_fns = [fn for (name, fns, *_r) in groups if device_kernel(name) == dom_kernel for fn in fns]
    bfp.bfp_flush_llc(1 << 30, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(2):
        for fn in dom_fns:
            fn()
    e1.record(stream)
    torch.cuda.synchronize()
    us_dom = e0.elapsed_time(e1) * 1e3 / (2 * len(dom_fns))
    roof["achieved"] = (dk["ops"] / (us_dom * 1e-6) / 1e12 if roof["unit"] == "Tops/s"
                        else dk["bytes"] / (us_dom * 1e-6) / 1e9)
    roof["frac"] = roof["achieved"] / roof["peak"]
    if roof["unit"] == "GB/s":
        roof["frac_of_copy"] = roof["achieved"] / roof["copy_GBps"]
        roof["frac_of_mix_ceiling"] = roof["achieved"] / roof["mix_ceiling_GBps"]
    roof["timing"] = ("%d back-to-back cold launches after one 1 GiB read sweep, events on the kernels' stream"
                      % (2 * len(dom_fns)))
    roof["us_per_launch"] = us_dom
    roof["us_per_launch_cold_groups"] = dk["us"]
    roof["us_per_launch_cache_assisted"] = dk["us_cache_assisted"]
    roof["algorithmic_bytes_per_launch"] = dk["bytes"]
    roof["device_kernel"] = dom_kernel
    roof["traffic"] = committed_traffic(roof["device_kernel"])

    res = {
        "metric": "custom-FP elements/s & % VALU/HBM peak, bit-exact; batched vs per-vector launch",
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_ms": settle_ms,
        "ms_per_step": ms_step,
        "ms_per_step_instrumented": ms_step_instrumented,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "add/sub/mul, 2^%d elements, formats (5,10) and (8,7), RNE, 64-element lane "
                               "words, pack+3 ops+unpack per format" % args.n_log2,
                   "n": n, "formats": ["(5,10)", "(8,7)"], "words_per_lane": 2},
        "wall_s_timed": wall,
        "roofline": roof,
        "kernels": {k: {x: v[x] for x in ("us", "launches", "GB/s", "hbm_frac", "Tops/s", "valu_frac",
                                          "us_cache_assisted", "hbm_frac_cache_assisted",
                                          "valu_frac_cache_assisted", "frac_of_mix_ceiling", "frac_of_probe")
                                 if x in v}
                    for k, v in kernels.items()},
    }
    def section(name, fn, *a, **kw):
        """A secondary section that raises is recorded with its error (and
        its traceback on stderr) so the headline line is still printed."""
        try:
            res[name] = fn(*a, **kw)
        except Exception as exc:  # noqa: BLE001
            import traceback
            traceback.print_exc()
            res[name] = {"error": "%s: %s" % (type(exc).__name__, exc)}

    if not args.no_sweep:
        section("sweep", bench_sweep, torch, bfp, dev, args.sweep_n_log2)
    if not args.no_layout_methods:
        section("layout_methods", bench_layout_methods, torch, bfp, dev, n)
    if not args.no_batched:
        section("batched", bench_batched, torch, bfp, dev, args.batched_reps, graphs=not args.batched_no_graph)
    if not args.no_serving:
        section("serving", bench_serving, torch, bfp, dev, args.serving_requests)
    if not args.no_div:
        section("div", bench_div, torch, bfp, dev, n, args.div_reps)
    if not args.no_chain:
        section("chain", bench_chain, torch, bfp, dev, n, args.div_reps)
    if not args.no_int:
        section("int", bench_int, torch, bfp, dev, n, args.div_reps)
    if not args.no_wide:
        section("wide", bench_wide, torch, bfp, dev, n, args.div_reps)
    if not args.no_small:
        section("small", bench_small, torch, bfp, dev)
    if not args.no_cpu_baseline:
        section("cpu_baseline", cpu_baseline)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
