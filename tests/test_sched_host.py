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
    I64 = ctypes.c_int64
    sig = {
        "simsrv_create": (VP, [U64, ctypes.c_int]), "simsrv_destroy": (None, [VP]),
        "simsrv_put": (U64, [VP, U64, U64]), "simsrv_free": (ctypes.c_int, [VP, U64]),
        "simsrv_offset": (I64, [VP, U64]),
        "simsrv_submit": (I64, [VP, U64, U64, U64, U64]), "simsrv_step": (ctypes.c_int, [VP]),
        "simsrv_cancel": (ctypes.c_int, [VP, U64]), "simsrv_set_timeout": (None, [VP, I64]),
        "simsrv_set_tick_limit": (None, [VP, U64]),
        "simsrv_collect": (ctypes.c_int, [VP]), "simsrv_launch_commit": (None, [VP]),
        "simsrv_release": (None, [VP, ctypes.c_int]), "simsrv_fail_next": (None, [VP]),
        "simsrv_running_ticks": (ctypes.c_int, [VP]),
        "simsrv_running_operands": (ctypes.c_int, [VP, VP, ctypes.c_int]),
        "simsrv_take": (ctypes.c_int, [VP, VP, VP, VP, ctypes.c_int]), "simsrv_stats": (None, [VP, VP]),
        "simarena_create": (VP, [U64]), "simarena_destroy": (None, [VP]),
        "simarena_alloc": (I64, [VP, U64]), "simarena_release": (U64, [VP, U64]),
        "simarena_stats": (None, [VP, VP]),
        "simlayout_gpad": (U64, [U64]), "simlayout_data_words": (U64, [U64]),
        "simlayout_word_mask": (U32, [U64, U64]),
    }
    for k, (r, a) in sig.items():
        getattr(L, k).restype = r
        getattr(L, k).argtypes = a
    return L


E_ARG, E_FORMAT, E_BUDGET, E_CANCELLED, E_TIMEOUT, E_BUSY = -6, -1, -8, -11, -12, -13
POOL_N = 1 << 20


def stats(L, s):
    out = np.zeros(16, dtype=np.uint64)
    L.simsrv_stats(s, out.ctypes.data)
    keys = ["used", "high", "cap", "pending", "inflight", "ticks", "max_tick", "max_inflight_ticks",
            "deferred", "admitted", "completed", "deferred_frees", "cancelled", "timed_out", "live", "slots"]
    return dict(zip(keys, map(int, out)))


def take(L, s, max_n=1000):
    ids = np.zeros(max_n, dtype=np.uint64)
    hs = np.zeros(max_n, dtype=np.uint64)
    st = np.zeros(max_n, dtype=np.int32)
    k = L.simsrv_take(s, ids.ctypes.data, hs.ctypes.data, st.ctypes.data, max_n)
    return list(zip(ids[:k].tolist(), hs[:k].tolist(), st[:k].tolist()))


def submitter(L, s, pool_bytes=256):
    """A pool operand of POOL_N elements and a submit(n, c_bytes) on it."""
    pool = L.simsrv_put(s, pool_bytes, POOL_N)
    assert pool

    def submit(n, c_bytes):
        rid = L.simsrv_submit(s, pool, pool, n, c_bytes)
        assert rid > 0, rid
        return rid
    return pool, submit


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
    pool, submit = submitter(L, s, 24 * 1024)
    ids = [submit(100, 8 * 1024) for _ in range(20)]  # 40 KiB left: 5 results fit
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
    _, submit = submitter(L, s)
    for _ in range(10):
        submit(10, 256)
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
    _, submit = submitter(L, s)
    a = [submit(10, 256) for _ in range(4)]
    L.simsrv_step(s)                      # tick 1 runs
    assert L.simsrv_running_ticks(s) == 1
    b = [submit(10, 256) for _ in range(3)]
    L.simsrv_step(s)                      # tick 2 starts while tick 1 still runs
    assert L.simsrv_running_ticks(s) == 2
    c = [submit(10, 256) for _ in range(2)]
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
    _, submit = submitter(L, s)
    used0 = stats(L, s)["used"]
    L.simsrv_fail_next(s)
    ids = [submit(10, 4096) for _ in range(3)]
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
    _, submit = submitter(L, s)
    a = [submit(10, 256) for _ in range(4)]
    assert L.simsrv_collect(s) == 4                      # batch taken, stream reserved
    st = stats(L, s)
    assert st["inflight"] == 4 and st["pending"] == 0
    b = [submit(10, 256) for _ in range(4)]  # arrive during the launch
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
    _, submit = submitter(L, s)
    used0 = stats(L, s)["used"]
    ids = [submit(10, 4096) for _ in range(3)]
    assert L.simsrv_collect(s) == 3
    more = [submit(10, 4096) for _ in range(2)]
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


def drain(L, s, rounds=50):
    out = []
    for _ in range(rounds):
        L.simsrv_release(s, 100)
        L.simsrv_step(s)
        out += take(L, s)
    return out


def test_free_operand_while_running_defers_release(L):
    """An operand freed while a running tick reads it keeps its arena range
    until that tick completes: a put in between lands elsewhere."""
    s = L.simsrv_create(1 << 20, 100)
    a = L.simsrv_put(s, 64 * 1024, POOL_N)
    b = L.simsrv_put(s, 64 * 1024, POOL_N)
    off_a = L.simsrv_offset(s, a)
    rid = L.simsrv_submit(s, a, b, 1000, 4096)
    assert rid > 0
    L.simsrv_step(s)
    assert L.simsrv_running_ticks(s) == 1
    assert L.simsrv_free(s, a) == 0                  # accepted, handle retired at once
    assert L.simsrv_offset(s, a) == -1
    assert L.simsrv_free(s, a) == -1                 # a second free of the same handle is refused
    assert L.simsrv_submit(s, a, b, 10, 256) == E_ARG  # and so is a new request on it
    st = stats(L, s)
    assert st["deferred_frees"] == 1
    c = L.simsrv_put(s, 64 * 1024, POOL_N)
    off_c = L.simsrv_offset(s, c)
    assert not (off_c < off_a + 64 * 1024 and off_a < off_c + 64 * 1024), "new vector overlaps a running operand"
    ops = np.zeros(8, dtype=np.uint64)
    k = L.simsrv_running_operands(s, ops.ctypes.data, 8)
    assert k == 2 and int(ops[0]) == off_a
    used_before = stats(L, s)["used"]
    done = drain(L, s)
    assert [(d[0], d[2]) for d in done] == [(rid, 0)]
    assert stats(L, s)["used"] == used_before - 64 * 1024   # a's range returned on completion
    L.simsrv_destroy(s)


def test_free_operand_while_queued(L):
    """Freeing an operand of queued requests: they still run on it, and its
    range is reused only after the last of them completes."""
    s = L.simsrv_create(1 << 20, 1)                   # one slot: the others queue
    a = L.simsrv_put(s, 32 * 1024, POOL_N)
    off_a = L.simsrv_offset(s, a)
    ids = [L.simsrv_submit(s, a, a, 100, 256) for _ in range(3)]
    L.simsrv_step(s)
    assert L.simsrv_free(s, a) == 0
    for _ in range(3):
        x = L.simsrv_put(s, 32 * 1024, POOL_N)
        ox = L.simsrv_offset(s, x)
        assert not (ox < off_a + 32 * 1024 and off_a < ox + 32 * 1024)
    done = drain(L, s)
    assert [d[0] for d in done] == ids and all(d[2] == 0 for d in done)
    for (_id, h, _st) in done:
        assert L.simsrv_free(s, h) == 0
    y = L.simsrv_put(s, 32 * 1024, POOL_N)
    assert L.simsrv_offset(s, y) == off_a              # first fit finds a's range again
    L.simsrv_destroy(s)


def test_handles_recycle_slots_and_reject_stale(L):
    s = L.simsrv_create(1 << 20, 10)
    h1 = L.simsrv_put(s, 1024, 100)
    assert L.simsrv_free(s, h1) == 0
    h2 = L.simsrv_put(s, 1024, 100)
    assert (h2 & 0xFFFFFFFF) == (h1 & 0xFFFFFFFF) and h2 != h1   # same slot, next generation
    assert L.simsrv_offset(s, h1) == -1 and L.simsrv_free(s, h1) == -1
    assert L.simsrv_submit(s, h1, h2, 10, 256) == E_ARG
    assert L.simsrv_offset(s, h2) >= 0
    assert L.simsrv_free(s, 0) == -1 and L.simsrv_free(s, 12345) == -1
    # many put/free cycles and request results keep the table small
    pool = L.simsrv_put(s, 1024, POOL_N)
    for i in range(3000):
        h = L.simsrv_put(s, 2048, 100)
        assert h and L.simsrv_free(s, h) == 0
        rid = L.simsrv_submit(s, pool, pool, 100, 512)
        assert rid > 0
        L.simsrv_step(s)
        L.simsrv_release(s, 10)
        L.simsrv_step(s)
        for (_id, hr, st) in take(L, s):
            assert st == 0 and L.simsrv_free(s, hr) == 0
    drain(L, s)
    st = stats(L, s)
    assert st["slots"] <= 8 and st["live"] == 2, st   # h2 and the pool
    L.simsrv_destroy(s)


def test_submit_validation(L):
    s = L.simsrv_create(1 << 16, 10)
    a = L.simsrv_put(s, 1024, 500)
    b = L.simsrv_put(s, 1024, 300)
    assert L.simsrv_submit(s, a, b, 301, 256) == E_ARG      # longer than b
    assert L.simsrv_submit(s, a, b, 0, 256) == E_ARG
    assert L.simsrv_submit(s, a, 999, 10, 256) == E_ARG     # not a handle
    assert L.simsrv_submit(s, a, b, 300, 1 << 17) == E_BUDGET  # could never fit
    assert L.simsrv_submit(s, a, b, 300, 256) > 0
    L.simsrv_destroy(s)


def test_cancel(L):
    s = L.simsrv_create(1 << 20, 2)
    pool, submit = submitter(L, s)
    r1, r2, r3, r4 = (submit(10, 1024) for _ in range(4))
    used0 = stats(L, s)["used"]
    assert L.simsrv_collect(s) == 2               # r1, r2 handed to the executor
    L.simsrv_launch_commit(s)
    assert L.simsrv_cancel(s, r1) == E_BUSY       # on the device
    assert L.simsrv_cancel(s, r4) == 0            # queued
    assert L.simsrv_cancel(s, r4) == E_ARG        # already withdrawn
    assert L.simsrv_cancel(s, 777) == E_ARG
    out = take(L, s)
    assert out == [(r4, 0, E_CANCELLED)]
    L.simsrv_release(s, 1)
    L.simsrv_step(s)                              # r1, r2 done; r3 admitted and launched
    done = take(L, s)
    assert [d[0] for d in done] == [r1, r2]
    for (_id, h, _st) in done:
        L.simsrv_free(s, h)
    assert L.simsrv_cancel(s, r3) == E_BUSY
    done = drain(L, s)
    assert [d[0] for d in done] == [r3]
    L.simsrv_free(s, done[0][1])
    st = stats(L, s)
    assert st["cancelled"] == 1 and st["used"] == used0 and st["inflight"] == 0
    assert L.simsrv_free(s, pool) == 0 and stats(L, s)["used"] == 0
    L.simsrv_destroy(s)


def test_cancel_admitted_waiting_for_a_stream(L):
    """Both streams busy: an admitted request waits with its result
    allocated; cancelling it frees that result."""
    s = L.simsrv_create(1 << 20, 100)
    _, submit = submitter(L, s)
    submit(10, 256)
    L.simsrv_step(s)
    submit(10, 256)
    L.simsrv_step(s)
    assert L.simsrv_running_ticks(s) == 2
    used0 = stats(L, s)["used"]
    r = submit(10, 4096)
    L.simsrv_step(s)                               # admitted, no stream free
    assert stats(L, s)["used"] == used0 + 4096
    assert L.simsrv_cancel(s, r) == 0
    assert stats(L, s)["used"] == used0
    assert take(L, s) == [(r, 0, E_CANCELLED)]
    L.simsrv_destroy(s)


def test_queue_timeout(L):
    s = L.simsrv_create(1 << 20, 1)
    _, submit = submitter(L, s)
    r1 = submit(10, 256)
    L.simsrv_step(s)                               # r1 runs and holds the only slot
    r2 = submit(10, 256)
    L.simsrv_set_timeout(s, 1_000_000)             # 1 ms
    import time
    time.sleep(0.01)
    L.simsrv_step(s)
    assert take(L, s) == [(r2, 0, E_TIMEOUT)]
    L.simsrv_set_timeout(s, 0)
    done = drain(L, s)
    assert [(d[0], d[2]) for d in done] == [(r1, 0)]
    assert stats(L, s)["timed_out"] == 1
    L.simsrv_destroy(s)


def test_fuzz_no_put_lands_on_memory_a_request_holds(L):
    """Random puts, frees, submits, cancels and tick completions: a new
    vector never overlaps an operand that an unfinished request reads, and
    every request completes exactly once."""
    rng = np.random.default_rng(7)
    s = L.simsrv_create(1 << 22, 16)
    live = {}          # handle -> (offset, bytes, n)
    retired = {}       # freed handle -> (offset, bytes)
    outstanding = {}   # request id -> (a, b)
    seen = set()
    for it in range(6000):
        x = rng.random()
        if x < 0.25 or not live:
            nb = int(rng.integers(1, 64)) * 256
            n = int(rng.integers(1, 5000))
            h = L.simsrv_put(s, nb, n)
            if h:
                off = L.simsrv_offset(s, h)
                for rid, (a, b) in outstanding.items():
                    for hh in (a, b):
                        if hh in retired:
                            o2, z2 = retired[hh]
                            assert not (off < o2 + z2 and o2 < off + nb), "put overlaps a held operand"
                live[h] = (off, nb, n)
        elif x < 0.4:
            h = list(live)[int(rng.integers(0, len(live)))]
            off, nb, _ = live.pop(h)
            assert L.simsrv_free(s, h) == 0
            retired[h] = (off, nb)
        elif x < 0.75:
            ks = list(live)
            a = ks[int(rng.integers(0, len(ks)))]
            b = ks[int(rng.integers(0, len(ks)))]
            n = int(rng.integers(1, min(live[a][2], live[b][2]) + 1))
            rid = L.simsrv_submit(s, a, b, n, int(rng.integers(1, 16)) * 256)
            assert rid > 0
            outstanding[rid] = (a, b)
        elif x < 0.8 and outstanding:
            rid = list(outstanding)[int(rng.integers(0, len(outstanding)))]
            assert L.simsrv_cancel(s, rid) in (0, E_BUSY)
        else:
            L.simsrv_release(s, int(rng.integers(0, 3)))
        L.simsrv_step(s)
        for (rid, h, st) in take(L, s):
            assert rid in outstanding and rid not in seen
            seen.add(rid)
            del outstanding[rid]
            assert st in (0, E_CANCELLED)
            if st == 0:
                assert L.simsrv_free(s, h) == 0
    for (rid, h, st) in drain(L, s, 200):
        del outstanding[rid]
        if st == 0:
            L.simsrv_free(s, h)
    assert not outstanding
    for h in list(live):
        assert L.simsrv_free(s, h) == 0
    st = stats(L, s)
    assert st["used"] == 0 and st["live"] == 0 and st["inflight"] == 0 and st["pending"] == 0
    L.simsrv_destroy(s)


def test_layout_prefix_reads_stay_inside_operands(L):
    """The plane stride rule is not monotonic in n (the 8 KiB skew), so a
    prefix computation must not walk the result's stride over an operand:
    the words the batch kernel reads, ceil(n/32), fit every operand plane."""
    assert L.simlayout_gpad(65000) == 2304 and L.simlayout_gpad(66000) == 2112
    assert L.simlayout_gpad(65000) > L.simlayout_gpad(66000)   # the case that read past an operand
    rng = np.random.default_rng(3)
    cases = [(66000, 65000), (66000, 1), (65536, 65535), (1 << 20, (1 << 20) - 1)]
    cases += [(int(na), int(rng.integers(1, na + 1))) for na in rng.integers(1, 1 << 22, 2000)]
    for na, n in cases:
        assert L.simlayout_data_words(n) <= L.simlayout_gpad(na)
        assert L.simlayout_data_words(n) == -(-n // 32)
    for n in (1, 31, 32, 33, 65000, 66000):
        for w in range(max(0, n // 32 - 2), n // 32 + 3):
            want = sum(1 << j for j in range(32) if 32 * w + j < n)
            assert L.simlayout_word_mask(w, n) == want


def test_tick_limit_splits_backlog_in_fifo_order(L):
    """With a tick limit, a backlog of admitted requests goes out as several
    ticks in FIFO order, each within the limit (a request larger than the
    limit goes alone)."""
    s = L.simsrv_create(1 << 30, 1000)
    _, submit = submitter(L, s)
    L.simsrv_set_tick_limit(s, 3 * 3 * 4096)          # three requests of 4096-byte results
    ids = [submit(10, 4096) for _ in range(7)] + [submit(10, 65536)] + [submit(10, 4096)]
    sizes = []
    done = []
    for _ in range(40):
        n = L.simsrv_collect(s)
        if n:
            sizes.append(n)
            L.simsrv_launch_commit(s)
        else:
            L.simsrv_release(s, 1)
        done += [d[0] for d in take(L, s)]
    assert sizes == [3, 3, 1, 1, 1], sizes
    assert done == ids
    L.simsrv_destroy(s)
