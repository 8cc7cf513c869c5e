"""Python driver of the serving loop (``bfp_server_*`` in libbfp).

The scheduler, the HBM ledger and all device work are native; this module
owns a server handle, builds a resident operand pool, generates request
streams (Poisson arrivals, log-uniform lengths, random format and op) and
turns completion timestamps into latency percentiles and throughput.
"""
from __future__ import annotations

import atexit
import ctypes
import time

import numpy as np

from . import bfp, inputs

OPS = ("add", "sub", "mul")           # the request mix of the serving measurement
ALL_OPS = ("add", "sub", "mul", "div")


_LIVE = set()


def _close_all():
    for s in list(_LIVE):
        s.close()


atexit.register(_close_all)


class Server:
    def __init__(self, budget_bytes: int, slots: int):
        self.h = bfp.bfp_server_create(budget_bytes, slots)
        self._buf = (bfp.bfp_completion * 4096)()
        self._cnt = ctypes.c_uint32()
        _LIVE.add(self)

    def put(self, f, std_dev) -> int:
        return bfp.bfp_server_put(self.h, f, std_dev, std_dev.numel())

    def submit(self, op, f, a: int, b: int, n: int) -> int:
        return bfp.bfp_server_submit(self.h, op, f, a, b, n)

    def poll(self):
        st = bfp.lib().bfp_server_poll(self.h, self._buf, 4096, ctypes.byref(self._cnt))
        if st != 0:
            raise bfp.BfpError(st, "bfp_server_poll")
        return [self._buf[i] for i in range(self._cnt.value)]

    def free(self, handle: int):
        bfp.bfp_server_free(self.h, handle)

    def cancel(self, req_id: int):
        bfp.bfp_server_cancel(self.h, req_id)

    def set_tick_limit(self, max_bytes: int):
        bfp.bfp_server_set_tick_limit(self.h, max_bytes)

    def set_queue_timeout(self, timeout_ns: int):
        bfp.bfp_server_set_queue_timeout(self.h, timeout_ns)

    def get(self, handle: int, f, out_dev):
        bfp.bfp_server_get(self.h, handle, f, out_dev)

    def view(self, handle: int):
        return bfp.bfp_server_view(self.h, handle)

    def stats(self) -> dict:
        return bfp.bfp_server_stats_get(self.h)

    def replay(self, reqs) -> int:
        return bfp.bfp_server_replay(self.h, reqs)

    def set_autofree(self, on: bool):
        bfp.bfp_server_set_autofree(self.h, on)

    def wait_idle(self, timeout_ms: int = 60000):
        bfp.bfp_server_wait_idle(self.h, timeout_ms)

    def close(self):
        if self.h:
            bfp.bfp_server_destroy(self.h)
            self.h = None
        _LIVE.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_pool(server: Server, formats, n: int, seed: int, device, sample_log2: int = 18, host_out=None):
    """Two resident operands of n elements per format, values from the sweep
    recipe (a 2^sample_log2-element draw repeated to length n: the circuits'
    cost does not depend on the values).  If host_out is a dict, it receives
    host_out[(e, m)] = (xa, xb): the draws put, element i of an operand being
    x[i % len(x)]."""
    import torch
    pool = {}
    for i, (e, m) in enumerate(formats):
        f = bfp.fmt(e, m)
        hs = []
        xs = []
        for j in range(2):
            k = min(n, 1 << sample_log2)
            x = inputs.sweep_operands(e, m, k, seed * 100 + 2 * i + j)
            reps = (n + k - 1) // k
            t = torch.from_numpy(np.tile(x, reps)[:n].copy()).to(device)
            hs.append(server.put(f, t))
            xs.append(x)
        pool[(e, m)] = (hs[0], hs[1], n)
        if host_out is not None:
            host_out[(e, m)] = (xs[0], xs[1])
    torch.cuda.synchronize()
    return pool


def request_stream(count: int, formats, seed: int, nmin_log2: float = 10, nmax_log2: float = 22, nmax=None,
                   ops=OPS):
    """(op, (e, m), n) with n = floor(2^U(nmin_log2, nmax_log2)), uniform format and op."""
    rng = np.random.default_rng(seed)
    ns = np.floor(np.exp2(rng.uniform(nmin_log2, nmax_log2, count))).astype(np.int64)
    if nmax is not None:
        ns = np.minimum(ns, nmax)
    fi = rng.integers(0, len(formats), count)
    oi = rng.integers(0, len(ops), count)
    return [(ops[oi[i]], formats[fi[i]], int(max(1, ns[i]))) for i in range(count)]


def run(server: Server, pool, reqs, rate=None, rnd: int = 0, seed: int = 0, keep_results: bool = False,
        stall_s: float = 30.0, skip: int = 0):
    """Submit `reqs` (all at once if rate is None, else at Poisson arrival
    times of `rate` per second), free each result as it completes (unless
    keep_results), and return the measurements over all but the first `skip`
    requests (warm-up).  Raises if no request completes for `stall_s` seconds
    while some are outstanding."""
    rng = np.random.default_rng(seed)
    n_req = len(reqs)
    if rate is None:
        arrivals = np.zeros(n_req)
    else:
        arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
    comp = {}
    ids = []
    t0 = time.perf_counter()
    i = 0
    last_progress = time.perf_counter()
    while len(comp) < n_req:
        now = time.perf_counter() - t0
        if time.perf_counter() - last_progress > stall_s:
            raise RuntimeError("serving stalled: %d of %d requests complete, stats %s"
                               % (len(comp), n_req, server.stats()))
        while i < n_req and arrivals[i] <= now:
            op, (e, m), n = reqs[i]
            a, b, _n0 = pool[(e, m)]
            ids.append(server.submit(op, bfp.fmt(e, m, rnd), a, b, n))
            i += 1
        for c in server.poll():
            last_progress = time.perf_counter()
            comp[c.req_id] = (c.status, c.result, c.t_submit_ns, c.t_done_ns, c.t_launch_ns)
            if c.status == 0 and not keep_results:
                server.free(c.result)
        if i < n_req and rate is not None:
            time.sleep(0)  # yield between arrivals
    wall = time.perf_counter() - t0
    meas = ids[skip:]
    lat = np.array([(comp[r][3] - comp[r][2]) / 1e3 for r in meas])  # us
    t_first = min(comp[r][2] for r in meas)
    t_last = max(comp[r][3] for r in meas)
    window = (t_last - t_first) / 1e9
    elements = sum(reqs[k][2] for k in range(skip, n_req))
    bad = sum(1 for r in ids if comp[r][0] != 0)
    return {"requests": len(meas), "errors": bad, "elements": elements, "wall_s": wall, "window_s": window,
            "requests_per_s": len(meas) / window, "elements_per_s": elements / window,
            "p50_us": float(np.percentile(lat, 50)), "p99_us": float(np.percentile(lat, 99)),
            "mean_us": float(lat.mean()), "rate": rate, "ids": ids, "completions": comp}


def run_native(server: Server, pool, reqs, rate=None, rnd: int = 0, seed: int = 0, skip: int = 0,
               timeout_s: float = 120.0):
    """Like run(), but the arrival schedule is submitted by bfp_server_replay
    from native code and results are freed by the server on completion, so
    the measurement is of the server, not of a Python loop."""
    rng = np.random.default_rng(seed)
    n_req = len(reqs)
    if rate is None:
        arrivals = np.zeros(n_req, dtype=np.int64)
    else:
        arrivals = np.floor(np.cumsum(rng.exponential(1e9 / rate, n_req))).astype(np.int64)
    sched = []
    for k, (op, (e, m), n) in enumerate(reqs):
        a, b, _n0 = pool[(e, m)]
        sched.append((op, bfp.fmt(e, m, rnd), a, b, n, int(arrivals[k])))
    server.set_autofree(True)
    first = server.replay(sched)
    comp = {}
    deadline = time.perf_counter() + timeout_s
    while len(comp) < n_req:
        got = server.poll()
        for c in got:
            comp[c.req_id] = (c.status, c.result, c.t_submit_ns, c.t_done_ns, c.t_launch_ns, c.t_admit_ns)
        if not got:
            if time.perf_counter() > deadline:
                raise RuntimeError("serving stalled: %d of %d complete, stats %s" % (len(comp), n_req,
                                                                                     server.stats()))
            time.sleep(0.0005)
    server.set_autofree(False)
    ids = list(range(first, first + n_req))
    meas = ids[skip:]
    lat = np.array([(comp[r][3] - comp[r][2]) / 1e3 for r in meas])
    t_first = min(comp[r][2] for r in meas)
    t_last = max(comp[r][3] for r in meas)
    window = (t_last - t_first) / 1e9
    elements = sum(reqs[k][2] for k in range(skip, n_req))
    bad = sum(1 for r in ids if comp[r][0] != 0)
    # where the time goes: queued (submit -> launch: waiting for a slot, the
    # budget or a free stream) and on the device (launch -> completion seen)
    queue = np.array([(comp[r][4] - comp[r][2]) / 1e3 for r in meas])
    dev = np.array([(comp[r][3] - comp[r][4]) / 1e3 for r in meas])
    slow = lat >= np.percentile(lat, 99)
    return {"requests": len(meas), "errors": bad, "elements": elements, "window_s": window,
            "requests_per_s": len(meas) / window, "elements_per_s": elements / window,
            "p50_us": float(np.percentile(lat, 50)), "p99_us": float(np.percentile(lat, 99)),
            "mean_us": float(lat.mean()), "rate": rate,
            "queue_p50_us": float(np.percentile(queue, 50)), "queue_p99_us": float(np.percentile(queue, 99)),
            "device_p50_us": float(np.percentile(dev, 50)), "device_p99_us": float(np.percentile(dev, 99)),
            "slowest1pct_queue_us": float(queue[slow].mean()), "slowest1pct_device_us": float(dev[slow].mean())}
