"""Serving scheduler core and arena on the CPU, with a fake executor whose
batches finish only when the test says so: admission never exceeds the
budget or the slot count, requests wait in FIFO order, a second batch starts
while the first runs (continuous batching), failures release their results."""
import ctypes
import os

import numpy as np
import pytest

from paper_1602_04716_amd import build

U64, U32, I32, VP = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_void_p


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(build.HOSTSIM):
        build.build()
    L = ctypes.CDLL(build.HOSTSIM)
    sig = {
        "simsrv_create": (VP, [U64, ctypes.c_int]), "simsrv_destroy": (None, [VP]),
        "simsrv_put": (U32, [VP, U64, U64]), "simsrv_free": (ctypes.c_int, [VP, U32]),
        "simsrv_submit": (U64, [VP, U64, U64]), "simsrv_step": (ctypes.c_int, [VP]),
        "simsrv_collect": (ctypes.c_int, [VP]), "simsrv_launch_commit": (None, [VP]),
        "simsrv_release": (None, [VP, ctypes.c_int]), "simsrv_fail_next": (None, [VP]),
        "simsrv_running_ticks": (ctypes.c_int, [VP]),
        "simsrv_take": (ctypes.c_int, [VP, VP, VP, VP, ctypes.c_int]), "simsrv_stats": (None, [VP, VP]),
        "simarena_create": (VP, [U64]), "simarena_destroy": (None, [VP]),
        "simarena_alloc": (ctypes.c_int64, [VP, U64]), "simarena_release": (U64, [VP, U64]),
        "simarena_stats": (None, [VP, VP]),
    }
    for k, (r, a) in sig.items():
        getattr(L, k).restype = r
        getattr(L, k).argtypes = a
    return L


def stats(L, s):
    out = np.zeros(11, dtype=np.uint64)
    L.simsrv_stats(s, out.ctypes.data)
    keys = ["used", "high", "cap", "pending", "inflight", "ticks", "max_tick", "max_inflight_ticks",
            "deferred", "admitted", "completed"]
    return dict(zip(keys, map(int, out)))


def take(L, s, max_n=1000):
    ids = np.zeros(max_n, dtype=np.uint64)
    hs = np.zeros(max_n, dtype=np.uint32)
    st = np.zeros(max_n, dtype=np.int32)
    k = L.simsrv_take(s, ids.ctypes.data, hs.ctypes.data, st.ctypes.data, max_n)
    return list(zip(ids[:k].tolist(), hs[:k].tolist(), st[:k].tolist()))


def test_arena_fuzz(L):
    rng = np.random.default_rng(0)
    cap = 1 << 20
    a = L.simarena_create(cap)
    live = {}
    for it in range(20000):
        if live and (rng.random() < 0.45 or len(live) > 200):
            off = list(live)[int(rng.integers(0, len(live)))]
            assert L.simarena_release(a, off) == live.pop(off)
        else:
            size = int(rng.integers(1, 20000))
            off = L.simarena_alloc(a, size)
            if off >= 0:
                sz = (size + 255) // 256 * 256
                assert off % 256 == 0 and off + sz <= cap
                for o, z in live.items():
                    assert off + sz <= o or o + z <= off, "overlap"
                live[off] = sz
        st = np.zeros(5, dtype=np.uint64)
        L.simarena_stats(a, st.ctypes.data)
        assert int(st[0]) == sum(live.values()) and int(st[1]) <= cap and int(st[3]) == len(live)
    for off in list(live):
        L.simarena_release(a, off)
    st = np.zeros(5, dtype=np.uint64)
    L.simarena_stats(a, st.ctypes.data)
    assert int(st[0]) == 0 and int(st[4]) == 1  # everything coalesced back into one range
    assert L.simarena_release(a, 12345) == 0  # not a live allocation
    L.simarena_destroy(a)


def test_budget_admission_fifo(L):
    cap = 64 * 1024
    s = L.simsrv_create(cap, 1000)
    pool = L.simsrv_put(s, 24 * 1024, 100)
    assert pool
    ids = [L.simsrv_submit(s, 100, 8 * 1024) for _ in range(20)]  # 40 KiB left: 5 results fit
    L.simsrv_step(s)
    st = stats(L, s)
    assert st["admitted"] == 5 and st["pending"] == 15 and st["used"] <= cap and st["deferred"] >= 1
    done = []
    for _ in range(200):
        L.simsrv_release(s, 1)
        L.simsrv_step(s)
        for (rid, h, status) in take(L, s):
            assert status == 0 and h
            done.append(rid)
            assert L.simsrv_free(s, h) == 0
        L.simsrv_step(s)
        assert stats(L, s)["used"] <= cap
        if len(done) == 20:
            break
    assert done == ids  # FIFO
    st = stats(L, s)
    assert st["high"] <= cap and st["completed"] == 20 and st["used"] == 24 * 1024
    L.simsrv_destroy(s)


def test_slot_limit(L):
    s = L.simsrv_create(1 << 30, 3)
    for _ in range(10):
        L.simsrv_submit(s, 10, 256)
    for _ in range(50):
        L.simsrv_step(s)
        st = stats(L, s)
        assert st["inflight"] + 0 <= 3
        L.simsrv_release(s, 1)
    L.simsrv_release(s, 100)
    for _ in range(20):
        L.simsrv_step(s)
    assert stats(L, s)["completed"] == 10
    L.simsrv_destroy(s)


def test_continuous_batching_two_streams(L):
    s = L.simsrv_create(1 << 30, 1000)
    a = [L.simsrv_submit(s, 10, 256) for _ in range(4)]
    L.simsrv_step(s)                      # tick 1 runs
    assert L.simsrv_running_ticks(s) == 1
    b = [L.simsrv_submit(s, 10, 256) for _ in range(3)]
    L.simsrv_step(s)                      # tick 2 starts while tick 1 still runs
    assert L.simsrv_running_ticks(s) == 2
    c = [L.simsrv_submit(s, 10, 256) for _ in range(2)]
    L.simsrv_step(s)                      # both streams busy: admitted, waits
    assert L.simsrv_running_ticks(s) == 2 and stats(L, s)["admitted"] == 9
    L.simsrv_release(s, 1)
    L.simsrv_step(s)                      # tick 1 done, tick 3 launches
    assert [x[0] for x in take(L, s)] == a
    assert L.simsrv_running_ticks(s) == 2
    L.simsrv_release(s, 2)
    L.simsrv_step(s)
    L.simsrv_step(s)
    assert [x[0] for x in take(L, s)] == b + c
    st = stats(L, s)
    assert st["ticks"] == 3 and st["max_inflight_ticks"] == 2 and st["max_tick"] == 4
    L.simsrv_destroy(s)


def test_launch_failure_releases_results(L):
    s = L.simsrv_create(1 << 20, 100)
    used0 = stats(L, s)["used"]
    L.simsrv_fail_next(s)
    ids = [L.simsrv_submit(s, 10, 4096) for _ in range(3)]
    L.simsrv_step(s)
    out = take(L, s)
    assert [x[0] for x in out] == ids and all(x[2] == -5 and x[1] == 0 for x in out)
    assert stats(L, s)["used"] == used0
    L.simsrv_destroy(s)


def test_split_step_submissions_during_launch(L):
    """The worker collects a batch under the lock and launches it unlocked:
    requests submitted in between count against the slots the batch holds,
    wait in FIFO order, and go out in the next tick on the other stream."""
    s = L.simsrv_create(1 << 30, 6)
    a = [L.simsrv_submit(s, 10, 256) for _ in range(4)]
    assert L.simsrv_collect(s) == 4                      # batch taken, stream reserved
    st = stats(L, s)
    assert st["inflight"] == 4 and st["pending"] == 0
    b = [L.simsrv_submit(s, 10, 256) for _ in range(4)]  # arrive during the launch
    assert stats(L, s)["pending"] == 4
    L.simsrv_launch_commit(s)
    assert L.simsrv_running_ticks(s) == 1
    assert L.simsrv_collect(s) == 2                      # 2 slots left; the second stream is free
    L.simsrv_launch_commit(s)
    st = stats(L, s)
    assert L.simsrv_running_ticks(s) == 2 and st["inflight"] == 6 and st["pending"] == 2
    assert L.simsrv_collect(s) == 0                      # no slot and no stream
    L.simsrv_release(s, 1)
    L.simsrv_step(s)                                     # first tick done; its slots admit b[2:]
    assert [x[0] for x in take(L, s)] == a
    L.simsrv_release(s, 2)
    L.simsrv_step(s)
    L.simsrv_step(s)
    assert [x[0] for x in take(L, s)] == b
    st = stats(L, s)
    assert st["ticks"] == 3 and st["max_inflight_ticks"] == 2 and st["inflight"] == 0
    L.simsrv_destroy(s)


def test_split_step_failure_releases_results(L):
    s = L.simsrv_create(1 << 20, 100)
    used0 = stats(L, s)["used"]
    ids = [L.simsrv_submit(s, 10, 4096) for _ in range(3)]
    assert L.simsrv_collect(s) == 3
    more = [L.simsrv_submit(s, 10, 4096) for _ in range(2)]
    L.simsrv_fail_next(s)
    L.simsrv_launch_commit(s)
    out = take(L, s)
    assert [x[0] for x in out] == ids and all(x[2] == -5 and x[1] == 0 for x in out)
    st = stats(L, s)
    assert st["inflight"] == 0 and st["pending"] == 2 and st["used"] == used0
    L.simsrv_step(s)
    L.simsrv_release(s, 1)
    L.simsrv_step(s)
    done = take(L, s)
    assert [x[0] for x in done] == more and all(x[2] == 0 for x in done)
    for (_id, h, _st) in done:
        assert L.simsrv_free(s, h) == 0
    assert stats(L, s)["used"] == used0
    L.simsrv_destroy(s)
