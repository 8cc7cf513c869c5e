"""Host tests of the rocprofv3 summary code on small synthetic databases with
the tables and columns rocprofv3 writes (kernel dispatches, top kernels,
counter records): cold-run detection after the cache flush, calibration of
the byte counters, main-grid filtering, and the source-hash gate on stored
traffic figures.  No GPU and no profiler are needed."""
import os
import sqlite3

import pytest

from paper_1602_04716_amd import profiling as P

K = "void bfp::(anonymous namespace)::k_unpack<2>(unsigned int const*, unsigned short*, unsigned long)"
FLUSH = "void bfp::k_sweep_read(float4 const*, unsigned long)"
CALIB = "void at::native::direct_copy_kernel_cuda(...)"
OTHER = "void bfp::k_pack<2>(unsigned short const*, unsigned int*, unsigned long)"


def _trace_db(path, rows):
    """rows: (name, duration_ns, grid_x) dispatched back to back."""
    c = sqlite3.connect(path)
    c.execute("create table kernels (name text, start integer, end integer, grid_x integer)")
    c.execute("create table top_kernels (name text, total_calls integer, total_duration real, "
              "average real, percentage real)")
    t = 0
    for name, ns, grid in rows:
        c.execute("insert into kernels values (?,?,?,?)", (name, t, t + ns, grid))
        t += ns + 1000
    names = sorted({r[0] for r in rows})
    for n in names:
        d = [r[1] for r in rows if r[0] == n]
        c.execute("insert into top_kernels values (?,?,?,?,?)", (n, len(d), sum(d), sum(d) / len(d), 1.0))
    c.commit()
    c.close()


def _counter_db(path, rows, with_grid=True):
    """rows: (kernel name, counter name, value, grid size)."""
    c = sqlite3.connect(path)
    if with_grid:
        c.execute("create table counters_collection (kernel_name text, counter_name text, value real, "
                  "grid_size integer)")
        c.executemany("insert into counters_collection values (?,?,?,?)", rows)
    else:
        c.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
        c.executemany("insert into counters_collection values (?,?,?)", [r[:3] for r in rows])
    c.commit()
    c.close()


def test_short_name_strips_signature_and_anonymous_namespace():
    assert P.short_name(K) == "bfp::k_unpack<2>"
    assert P.short_name("void bfp::k_binop<5, 10, false, 0, 2, 1>(Args)") == "bfp::k_binop<5, 10, false, 0, 2, 1>"


def test_cold_runs_follow_the_flush_and_keep_the_main_grid(tmp_path):
    db = str(tmp_path / "t.db")
    big, small = 1 << 20, 1 << 10
    rows = [(OTHER, 5000, big), (K, 9000, big),          # not after a flush
            (FLUSH, 100000, 4096), (K, 50000, big), (K, 52000, big), (K, 51000, big),  # run of 3
            (OTHER, 5000, big), (K, 40000, big),          # warm again
            (FLUSH, 100000, 4096), (K, 60000, big),       # run of 1
            (FLUSH, 100000, 4096), (K, 3000, small)]      # smaller grid: not the workload
    _trace_db(db, rows)
    ca = P.cold_average(db, "bfp::k_unpack<2>")
    assert ca["cold_grid"] == big
    assert ca["cold_dispatches"] == 4
    assert ca["longest_run"] == 3
    assert ca["longest_run_avg_us"] == pytest.approx(51.0)
    assert ca["cold_avg_us"] == pytest.approx((50 + 52 + 51 + 60) / 4)
    assert ca["other_dispatches"] == 2
    assert ca["other_avg_us"] == pytest.approx((9 + 40) / 2)
    assert P.main_grids(db)["bfp::k_unpack<2>"] == big
    assert P.main_grid_durations(db)["bfp::k_unpack<2>"] == pytest.approx((9 + 50 + 52 + 51 + 40 + 60) / 6)


@pytest.mark.parametrize("with_grid", [True, False])
def test_byte_counters_are_calibrated_and_filtered(tmp_path, monkeypatch, with_grid):
    tdb, fdb, wdb = (str(tmp_path / n) for n in ("t.db", "f.db", "w.db"))
    big, small = 1 << 20, 1 << 10
    _trace_db(tdb, [(CALIB, 80000, 1 << 26), (FLUSH, 1000, 4096), (K, 50000, big), (K, 50000, big)])
    calib_kib = P.CALIB_BYTES / 1024
    # The counters read 0.5x the true bytes on fetch and 0.8x on write.
    _counter_db(fdb, [(CALIB, "FETCH_SIZE", calib_kib * 0.5, 1 << 26),
                      (K, "FETCH_SIZE", 1000.0, big), (K, "FETCH_SIZE", 1002.0, big),
                      (K, "FETCH_SIZE", 7.0, small)], with_grid)
    _counter_db(wdb, [(CALIB, "WRITE_SIZE", calib_kib * 0.8, 1 << 26),
                      (K, "WRITE_SIZE", 400.0, big), (K, "WRITE_SIZE", 400.0, big),
                      (K, "WRITE_SIZE", 1.0, small)], with_grid)
    monkeypatch.setattr(P, "source_hash", lambda: "abc123")
    out = str(tmp_path / "summary")
    chosen, ca = P.summarize(tdb, fdb, wdb, "bfp::k_unpack<2>", out, {"trace": "cmd"})
    if with_grid:
        fetch, write = 1001.0 * 2 * 1024, 400.0 / 0.8 * 1024
    else:  # no grid column: every dispatch counts
        fetch, write = (1000.0 + 1002.0 + 7.0) / 3 * 2 * 1024, (800.0 + 1.0) / 3 / 0.8 * 1024
    assert chosen[0] == "bfp::k_unpack<2>"
    assert chosen[1] == pytest.approx(fetch)
    assert chosen[2] == pytest.approx(write)
    text = open(out + ".md").read()
    assert "factors are 2.0000 (fetch) and 1.2500 (write)" in text
    tr = P.read_traffic(out + ".traffic.txt")
    assert tr["kernel"] == "bfp::k_unpack<2>"
    assert tr["bytes"] == pytest.approx(fetch + write, abs=1)
    # A stored figure taken with other kernel sources is not used.
    monkeypatch.setattr(P, "source_hash", lambda: "def456")
    assert P.read_traffic(out + ".traffic.txt") is None


def test_calibration_kernel_must_be_present(tmp_path):
    fdb = str(tmp_path / "f.db")
    _counter_db(fdb, [(K, "FETCH_SIZE", 1.0, 64)])
    with pytest.raises(RuntimeError):
        P._calib(P.counter_per_dispatch(fdb))


def test_valu_rows_only_for_kernels_counted_at_the_traced_grid(tmp_path, monkeypatch):
    tdb, pdb = str(tmp_path / "t.db"), str(tmp_path / "p.db")
    n = 1 << 26
    main = "void bfp::k_binop<5, 10, false, 0, 2, 1>(Args)"
    swept = "void bfp::k_binop<3, 1, false, 0, 4, 1>(Args)"
    # Traced at the workload's grid; the counter pass ran `swept` only on a
    # small grid, so its instructions cannot be divided by n.
    _trace_db(tdb, [(main, 60000, n // 64), (swept, 7000, n // 128)])
    _counter_db(pdb, [(main, "SQ_INSTS_VALU", 1.0e7, n // 64), (swept, "SQ_INSTS_VALU", 5.0e4, 4096)])
    gates = {"bfp::k_binop<5, 10, false, 0, 2, 1>": 404, "bfp::k_binop<3, 1, false, 0, 4, 1>": 128}
    monkeypatch.setattr(P, "_gates", lambda k: gates.get(k))
    monkeypatch.setattr(P, "source_hash", lambda: "abc123")
    out = str(tmp_path / "valu")
    P.valu_summary(tdb, pdb, n, out, {"trace": "cmd"})
    text = open(out + ".md").read()
    assert "k_binop<5, 10, false, 0, 2, 1>" in text
    assert "k_binop<3, 1, false, 0, 4, 1>" not in text
    # 1e7 wave instructions x 64 lanes over n/32 groups = 305 lane-instr per 32 elements.
    row = [l for l in text.splitlines() if "k_binop<5, 10" in l][0]
    assert "| 305 | 404 |" in row


def test_sq_summary_fractions_and_wave_life(tmp_path, monkeypatch):
    tdb, pdb = str(tmp_path / "t.db"), str(tmp_path / "p.db")
    k = "void bfp::k_binop_std<5, 2, false, 0>(Args)"
    _trace_db(tdb, [(k, 3400, 2048), (k, 3300, 2048)])
    rows = []
    for _ in range(2):
        rows += [(k, "SQ_WAVES", 32.0, 2048), (k, "SQ_WAVE_CYCLES", 57600.0, 2048),
                 (k, "SQ_BUSY_CYCLES", 57600.0, 2048), (k, "SQ_WAIT_ANY", 28800.0, 2048),
                 (k, "SQ_WAIT_INST_ANY", 576.0, 2048), (k, "SQ_ACTIVE_INST_ANY", 14400.0, 2048)]
    rows.append((k, "SQ_WAVES", 1.0, 64))  # a smaller launch: not averaged in
    _counter_db(pdb, rows)
    monkeypatch.setattr(P, "source_hash", lambda: "abc123")
    out = str(tmp_path / "sq")
    P.sq_summary(tdb, pdb, ["bfp::k_binop_std<5, 2, false, 0>"], out, {"pmc": "cmd"}, cycle_unit=4)
    text = open(out + ".md").read()
    row = [l for l in text.splitlines() if "k_binop_std" in l][0].split("|")
    cells = [c.strip() for c in row[1:-1]]
    # columns: kernel, dispatches, 6 counters (sorted), 3 fractions, wave life, waves per CU, trace us.
    # 57600 counts x 4 cycles / 32 waves at 2.4 GHz = 3.00 us per wave; over the 3.35 us
    # trace average that is 57600 x 4 / 8040 cycles = 28.66 waves, 0.11 per CU.
    assert cells[1] == "2"
    assert cells[8:] == ["0.50", "0.01", "0.25", "3.00", "0.1", "3.35"]


def test_wave_cycle_unit_from_the_one_wave_kernel(tmp_path, monkeypatch):
    tdb, pdb = str(tmp_path / "t.db"), str(tmp_path / "p.db")
    clock = "void bfp::k_wave_clock(float*, int)"
    k = "void bfp::k_binop_std<5, 2, false, 0>(Args)"
    # 7.36 ms at 2.4 GHz = 17.664e6 cycles; a count of 4.40e6 is 4.01 cycles per count.
    _trace_db(tdb, [(clock, 7360000, 64), (k, 3400, 2048)])
    _counter_db(pdb, [(clock, "SQ_WAVE_CYCLES", 4.40e6, 64), (clock, "SQ_WAVES", 1.0, 64),
                      (k, "SQ_WAVES", 32.0, 2048), (k, "SQ_WAVE_CYCLES", 1700.0 * 32, 2048)])
    unit, ratio, nd = P.wave_cycle_unit(tdb, pdb)
    assert unit == 4.0 and ratio == pytest.approx(4.0145, rel=1e-3) and nd == 1
    monkeypatch.setattr(P, "source_hash", lambda: "abc123")
    out = str(tmp_path / "sq")
    P.sq_summary(tdb, pdb, ["bfp::k_binop_std<5, 2, false, 0>"], out, {"pmc": "cmd"})
    text = open(out + ".md").read()
    assert "one count is 4 shader cycles" in text
    row = [l for l in text.splitlines() if "k_binop_std" in l][0]
    # 1700 counts x 4 cycles / 2.4 GHz = 2.83 us per wave
    assert "| 2.83 |" in row
    # without the calibration kernel no unit is assumed
    _counter_db(str(tmp_path / "q.db"), [(k, "SQ_WAVES", 32.0, 2048), (k, "SQ_WAVE_CYCLES", 54400.0, 2048)])
    assert P.wave_cycle_unit(tdb, str(tmp_path / "q.db")) is None


def test_tick_bursts_split_runs_and_measure_busy_share(tmp_path):
    db = str(tmp_path / "t.db")
    c = sqlite3.connect(db)
    c.execute("create table kernels (name text, start integer, end integer, grid_x integer)")
    c.execute("create table top_kernels (name text, total_calls integer, total_duration real, "
              "average real, percentage real)")
    k0, k1 = "void bfp::k_batch<0>(Args)", "void bfp::k_batch<1>(Args)"
    us = 1000
    # run 1: two overlapping ticks then one after a 10 us gap: busy 30 of 40 us
    rows = [(k0, 0, 20 * us), (k0, 10 * us, 20 * us), (k1, 30 * us, 40 * us)]
    # run 2, 50 ms later: back-to-back ticks, fully busy
    t = 50_000 * us
    rows += [(k0, t, t + 5 * us), (k0, t + 5 * us, t + 10 * us), ("void other(Args)", t + 10 * us, t + 90 * us)]
    c.executemany("insert into kernels values (?,?,?,0)", rows)
    c.commit()
    c.close()
    b = P.tick_bursts(db)
    assert [x["dispatches"] for x in b] == [3, 2]
    assert b[0]["window_ms"] == pytest.approx(0.04) and b[0]["busy_frac"] == pytest.approx(0.75)
    assert b[1]["busy_frac"] == pytest.approx(1.0) and b[1]["median_us"] == pytest.approx(5.0)
    out = str(tmp_path / "ticks")
    P.ticks_summary(db, out, {"trace": "cmd"}, ["first", "second"])
    text = open(out + ".md").read()
    assert "| first | 3 | 0.04 | 75.0% |" in text and "| second | 2 |" in text
