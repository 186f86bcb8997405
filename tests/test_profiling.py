"""Host logic of the profile summaries (paper_2212_09642_amd.profiling) on a
small hand-built database with the tables and views the summaries read:
the timed region between the two marker kernels, Lanczos steps counted once
under concurrent tile chains, the busy span of the step unit and the
traffic per step scaled by a copy calibration."""
import json
import sqlite3
import types

import pytest

from paper_2212_09642_amd import profiling

GUID = "g"


def _db(path, dispatches, counters=()):
    """dispatches: (dispatch id, kernel name, stream, start, end);
    counters: (dispatch id, counter, value)."""
    con = sqlite3.connect(path)
    con.execute("create table rocpd_info_kernel_symbol (id integer, guid text, display_name text)")
    con.execute("create table rocpd_kernel_dispatch (dispatch_id integer, guid text, kernel_id integer, "
                "stream_id integer, start integer, end integer)")
    con.execute("create table counters_collection (dispatch_id integer, kernel_name text, counter_name text, "
                "value real)")
    names = sorted({d[1] for d in dispatches})
    kid = {n: i for i, n in enumerate(names)}
    con.executemany("insert into rocpd_info_kernel_symbol values (?, ?, ?)", [(i, GUID, n) for n, i in kid.items()])
    con.executemany("insert into rocpd_kernel_dispatch values (?, ?, ?, ?, ?, ?)",
                    [(d, GUID, kid[n], s, a, b) for d, n, s, a, b in dispatches])
    byid = {d[0]: d[1] for d in dispatches}
    con.executemany("insert into counters_collection values (?, ?, ?, ?)",
                    [(d, byid[d], c, v) for d, c, v in counters])
    con.execute("create view top_kernels as select S.display_name as name, count(*) as total_calls, "
                "sum(K.end - K.start) / 1000.0 as total_duration, "
                "(sum(K.end - K.start) / count(*)) / 1000.0 as average from rocpd_kernel_dispatch K "
                "join rocpd_info_kernel_symbol S on S.id = K.kernel_id group by name")
    con.commit()
    con.close()


MARK = "at::cuda::spin_kernel(long)"
NORM, STEP, LONG = "vne::k_normalize<float, 4, false>", "vne::k_lanczos_step<float, 4, 64, false, true>", \
    "vne::k_long_rows<float, 4, 64, false, true>"
RED, FIN = "vne::k_reduce_partials", "vne::k_finalize"


def _trace():
    """Warm-up on stream 1, marker, 3 unchained steps on stream 1, 4 steps in
    two concurrent chains (streams 2 and 3), marker, 5 more steps."""
    d, t, out = [0], [0], []

    def add(name, stream, dur, start=None):
        d[0] += 1
        a = t[0] if start is None else start
        out.append((d[0], name, stream, a, a + dur))
        if start is None:
            t[0] = a + dur
        return d[0]

    def step(stream):
        for name, dur in ((NORM, 10), (STEP, 100), (LONG, 5), (RED, 3), (FIN, 2)):
            add(name, stream, dur)

    for _ in range(2):
        step(1)                        # warm-up: not in the region
    add(MARK, 1, 1)
    t[0] += 50
    for _ in range(3):
        step(1)                        # 3 x 120 ns busy
    t0 = t[0] + 20
    for i in range(4):                 # chain A: one step per 120 ns; chain B offset by 60 ns
        for c, off in ((2, 0), (3, 60)):
            a = t0 + 120 * i + off
            for name, dur in ((NORM, 10), (STEP, 100), (LONG, 5), (RED, 3), (FIN, 2)):
                add(name, c, dur, start=a)
                a += dur
    t[0] = t0 + 120 * 4 + 60 + 30
    add(MARK, 1, 1)
    for _ in range(5):
        step(1)                        # after the region
    return out


def test_region_and_logical_steps(tmp_path):
    db = str(tmp_path / "kt.db")
    _db(db, _trace())
    disp = profiling._dispatches(sqlite3.connect(db))
    region, main = profiling._region(disp)
    assert main == 1
    assert not any(profiling.MARKER in x[1] for x in region)
    # 3 steps on the markers' stream, 4 on each chain stream: 7 steps
    assert sum(1 for x in region if "k_lanczos_step" in x[1]) == 3 + 2 * 4
    assert profiling._logical_steps(region, main) == 7
    # busy span: 3 x 120 ns unchained; chains cover [t0, t0 + 3 * 120 + 60 + 120)
    assert profiling._busy_ns(region, profiling.UNIT_KERNELS) == 3 * 120 + (3 * 120 + 60 + 120)
    # without markers every step dispatch counts
    nomark = [x for x in disp if profiling.MARKER not in x[1]]
    r2, m2 = profiling._region(nomark)
    assert m2 is None and profiling._logical_steps(r2, m2) == 2 + 3 + 8 + 5


def test_busy_union_of_intervals():
    mk = lambda a, b: (0, "vne::k_finalize", 1, a, b)
    assert profiling._busy_ns([mk(0, 10), mk(5, 20), mk(30, 31), mk(31, 40)], ("k_finalize",)) == 20 + 10
    assert profiling._busy_ns([], ("k_finalize",)) == 0


def test_stats_summary(tmp_path):
    db = str(tmp_path / "kt.db")
    _db(db, _trace())
    out = str(tmp_path / "s.md")
    line = tmp_path / "bench.log"
    line.write_text("warm-up done\n" + json.dumps({"roofline": {"launches": 7, "avg_launch_ms": 0.00013,
                                                                "frac": 0.25}}) + "\n")
    profiling.cmd_stats(types.SimpleNamespace(db=db, out=out, cmd="cmd", bench_line=str(line)))
    text = open(out).read()
    assert "7 steps on 3 stream(s)" in text
    assert "%.2f us per step" % ((3 * 120 + 540) / 1e3 / 7) in text
    assert "timed 7 step launches at 0.13 us each" in text


def test_traffic_per_step(tmp_path):
    tr = _trace()
    # 2 KiB fetched and 1 KiB written per step-unit dispatch, 7 KiB by the marker
    fetch = [(x[0], "FETCH_SIZE", 7.0 if profiling.MARKER in x[1] else 2.0) for x in tr]
    write = [(x[0], "WRITE_SIZE", 7.0 if profiling.MARKER in x[1] else 1.0) for x in tr]
    _db(str(tmp_path / "f.db"), tr, fetch)
    _db(str(tmp_path / "w.db"), tr, write)
    copy = [(1, "__amd_rocclr_copyBuffer", 1, 0, 10), (2, "__amd_rocclr_copyBuffer", 1, 20, 30)]
    _db(str(tmp_path / "cf.db"), copy, [(1, "FETCH_SIZE", 512.0), (2, "FETCH_SIZE", 512.0)])
    _db(str(tmp_path / "cw.db"), copy, [(1, "WRITE_SIZE", 1024.0), (2, "WRITE_SIZE", 1024.0)])
    out = str(tmp_path / "t.json")
    profiling.cmd_traffic(types.SimpleNamespace(
        fetch_db=str(tmp_path / "f.db"), write_db=str(tmp_path / "w.db"), copy_fetch_db=str(tmp_path / "cf.db"),
        copy_write_db=str(tmp_path / "cw.db"), out=out, workload="w", copy_bytes=1024.0 * 1024, copies=2,
        cmd="cmd"))
    d = json.load(open(out))
    assert d["steps"] == 7
    assert d["copy_calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert d["copy_calibration"]["write_scale"] == pytest.approx(1.0)
    # 11 step units of 5 dispatches in the region: (2 KiB x 2 + 1 KiB) x 55 over 7 steps
    assert d["hbm_bytes_per_launch"] == pytest.approx(5.0 * 1024 * 55 / 7)
