"""Summaries of rocprofv3 output databases (the rocpd SQLite files that
``rocprofv3 -d DIR -o run`` writes) for the files kept under profiles/.

    python -m paper_2212_09642_amd.profiling stats DB OUT.md --cmd "..."
    python -m paper_2212_09642_amd.profiling traffic FETCH_DB WRITE_DB COPY_FETCH_DB \
        COPY_WRITE_DB OUT.json --workload NAME --copy-bytes B --cmd "..."
    python -m paper_2212_09642_amd.profiling serve BENCH_LINE.json OUT.md --cmd "..."
    python -m paper_2212_09642_amd.profiling counters OUT.md --kernel NAME DB [DB ...] --cmd "..."

The Lanczos step unit is the normalize pass (two-pass schedule), the SpMM +
recurrence kernel, the long-row kernel and the partial-sum reductions of one
step.  bench.py brackets its timed region with two marker kernels (torch's
spin kernel); the summaries count only the dispatches between them, which
leaves out warm-up, tile tuning and what a run does afterwards.  A loop may
run its column tiles as concurrent chains on streams of their own, each
chain dispatching every step for its tiles: a Lanczos step is then counted
once, from the step kernels of the stream that carries the markers (loops
run as one chain) plus those of the busiest other stream (the first chain
takes part in every chained loop).
"""
import argparse
import collections
import json
import os
import sqlite3
import sys

STEP_KERNELS = ("k_normalize", "k_lanczos_step", "k_long_rows")
UNIT_KERNELS = STEP_KERNELS + ("k_reduce_partials", "k_finalize")
MARKER = "spin_kernel"


def _short(name):
    return name.split("(")[0].replace("void ", "").replace("vne::", "")


def kernel_stats(db):
    con = sqlite3.connect(db)
    rows = list(con.execute("select name, total_calls, total_duration, average from top_kernels"))
    # the top_kernels view reports microseconds
    return [(n, int(c), float(t), float(a)) for n, c, t, a in rows]


def _dispatches(con):
    """(dispatch id, kernel name, stream id, start ns, end ns) of every
    dispatch, by start time."""
    return con.execute(
        "select K.dispatch_id, S.display_name, K.stream_id, K.start, K.end from rocpd_kernel_dispatch K "
        "join rocpd_info_kernel_symbol S on S.id = K.kernel_id and S.guid = K.guid "
        "order by K.start, K.dispatch_id").fetchall()


def _region(disp):
    """The dispatches between the two marker kernels (after the first when
    there is one only) and the markers' stream; all dispatches and None
    without a marker.  Everything in the region was issued after the first
    marker ended and before the second started (the host synchronizes in
    between), so start times order them."""
    marks = [i for i, d in enumerate(disp) if MARKER in d[1]]
    if not marks:
        return disp, None
    hi = marks[1] if len(marks) > 1 else len(disp)
    return disp[marks[0] + 1:hi], disp[marks[0]][2]


def _logical_steps(disp, main):
    """Lanczos steps among the dispatches (see the module's docstring)."""
    per = collections.Counter(d[2] for d in disp if "k_lanczos_step" in d[1])
    if main is None:
        return sum(per.values())
    return per.get(main, 0) + max([v for st, v in per.items() if st != main], default=0)


def _busy_ns(disp, names):
    """Length of the union of the intervals of the dispatches whose kernel
    name contains one of names."""
    total, lo, hi = 0, None, None
    for a, b in sorted((d[3], d[4]) for d in disp if any(k in d[1] for k in names)):
        if hi is None or a > hi:
            if hi is not None:
                total += hi - lo
            lo, hi = a, b
        else:
            hi = max(hi, b)
    return total + (hi - lo if hi is not None else 0)


def cmd_stats(args):
    rows = kernel_stats(args.db)
    tot = sum(r[2] for r in rows)
    out = ["# rocprofv3 kernel statistics", "", "Command:", "", "```", args.cmd, "```", "",
           "Whole run (warm-up and tile tuning included):", "",
           "| kernel | calls | total ms | avg us | share |", "|---|---:|---:|---:|---:|"]
    for n, c, t, a in rows:
        out.append("| `%s` | %d | %.3f | %.2f | %.1f%% |" % (_short(n), c, t / 1e3, a, 100 * t / tot))
    out += ["", "All kernels: %.3f ms." % (tot / 1e3)]
    region, main = _region(_dispatches(sqlite3.connect(args.db)))
    if main is not None:
        steps = _logical_steps(region, main)
        busy = _busy_ns(region, UNIT_KERNELS) / 1e3
        per = collections.defaultdict(list)
        for d in region:
            per[_short(d[1])].append((d[4] - d[3]) / 1e3)
        out += ["", "Timed region (between the marker kernels):", "",
                "| kernel | calls | total ms | avg us |", "|---|---:|---:|---:|"]
        for k in sorted(per, key=lambda k: -sum(per[k])):
            out.append("| `%s` | %d | %.3f | %.2f |" % (k, len(per[k]), sum(per[k]) / 1e3,
                                                        sum(per[k]) / len(per[k])))
        n_streams = len({d[2] for d in region if "k_lanczos_step" in d[1]})
        out += ["", "Lanczos step unit (normalize, SpMM/recurrence, long rows, partial reductions, finalize) "
                    "in the timed region: %d steps on %d stream(s); the union of its kernels' intervals is "
                    "%.3f ms, %.2f us per step." % (steps, n_streams, busy / 1e3, busy / max(steps, 1))]
    if args.bench_line:
        # the JSON line the profiled bench.py run printed: its own HIP-event
        # timing of the same steps, for comparison with the trace
        with open(args.bench_line) as fh:
            line = [x for x in fh.read().splitlines() if x.startswith("{")][-1]
        r = json.loads(line)["roofline"]
        out += ["", "The profiled bench.py run timed %d step launches at %.2f us each with HIP events "
                    "(roofline fraction %.4f under the profiler)." % (r["launches"], 1e3 * r["avg_launch_ms"],
                                                                     r["frac"])]
    with open(args.out, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("\n".join(out))


def _counter(db, name_filter=None):
    """Counter sums and dispatch counts per (kernel, counter) over the
    timed region's dispatches whose kernel name contains one of name_filter
    (the whole run without markers), and the region's Lanczos steps."""
    con = sqlite3.connect(db)
    region, main = _region(_dispatches(con))
    keep = {d[0] for d in region}
    acc = collections.defaultdict(float)
    calls = collections.Counter()
    rows = con.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection "
                       "order by dispatch_id").fetchall()
    for did, kname, ctr, val in rows:
        if did not in keep or (name_filter and not any(k in kname for k in name_filter)):
            continue
        acc[(kname, ctr)] += float(val)
        calls[(kname, ctr)] += 1
    return acc, calls, _logical_steps(region, main)


def cmd_traffic(args):
    fetch, _, steps = _counter(args.fetch_db, UNIT_KERNELS)
    write, _, steps_w = _counter(args.write_db, UNIT_KERNELS)
    if steps != steps_w:
        sys.exit("the FETCH_SIZE and WRITE_SIZE runs hold %d and %d Lanczos steps" % (steps, steps_w))
    cf, _, _ = _counter(args.copy_fetch_db, ("copyBuffer",))
    cw, _, _ = _counter(args.copy_write_db, ("copyBuffer",))
    # calibration: what the counters read (KiB per dispatch) for a plain copy
    # of known size, one dispatch per copy
    copy_fetch_kib = sum(cf.values()) / max(args.copies, 1)
    copy_write_kib = sum(cw.values()) / max(args.copies, 1)
    f_scale = args.copy_bytes / (copy_fetch_kib * 1024.0)
    w_scale = args.copy_bytes / (copy_write_kib * 1024.0)
    fetch_kib = sum(fetch.values())
    write_kib = sum(write.values())
    per_step = (fetch_kib * f_scale + write_kib * w_scale) * 1024.0 / max(steps, 1)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    d = {"workload": args.workload, "kernel": "Lanczos step unit (" + ", ".join(UNIT_KERNELS) + ")",
         "steps": steps, "fetch_kib_total": fetch_kib, "write_kib_total": write_kib,
         "copy_calibration": {"bytes_each_way": args.copy_bytes, "fetch_kib": copy_fetch_kib,
                              "write_kib": copy_write_kib, "fetch_scale": f_scale, "write_scale": w_scale},
         "hbm_bytes_per_launch": per_step, "kernel_source_hash": bench.kernel_source_hash(),
         "command": args.cmd}
    with open(args.out, "w") as fh:
        json.dump(d, fh, indent=1)
    print(json.dumps(d, indent=1))


def cmd_serve(args):
    """Rate table of a `bench.py --workload serve` line."""
    with open(args.line) as fh:
        d = json.loads(fh.read().strip().splitlines()[-1])
    c = d["config"]
    out = ["# Serving loop: Poisson arrivals at several rates", "", "Command:", "", "```", args.cmd, "```", "",
           "Workload `%s`: %d graphs, relative accuracy %g per query, %d queries per rate, group slots of "
           "up to %d tasks, tasks stopped on the %s." % (
               c["workload"], c["graphs"], c["rel_eps"], c["queries_per_rate"], c.get("max_group", 2),
               {"bound": "upper bound of each bracket (eq. (4.9))",
                "estimate": "geometric mean of each bracket (eq. (4.10))"}[c.get("stop", "bound")]),
           "",
           "| offered /s | completed /s | p50 ms | p99 ms | algorithmic GB/s | mean probes | mean steps | "
           "sampling target met | within 1e-3 of the exact entropy | running tasks per tick | tasks in group slots |",
           "|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in d["rates"]:
        pairs = "%d/%d" % (r["tasks_in_group_slots"], r["tasks"]) if "tasks" in r else "-"
        exact = ("%d/%d" % (r["within_1e-3_of_exact"], r["queries_with_exact_entropy"])
                 if "queries_with_exact_entropy" in r else "-")
        out.append("| %g | %.1f | %.1f | %.1f | %.0f | %.0f | %.1f | %d/%d | %s | %.2f | %s |" % (
            r["offered_per_s"], r["completed_per_s"], r["p50_ms"], r["p99_ms"], r["algorithmic_GBps"],
            r["mean_probes"], r["mean_steps"], r["sampling_target_met"], r["queries"], exact, r["slot_occupancy"],
            pairs))
    out += ["", "Saturated throughput: %.1f queries/s." % d["value"]]
    with open(args.out, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("\n".join(out))


def _ratio(tab, num, den, scale=1.0):
    if num in tab and den in tab and tab[den] > 0:
        return scale * tab[num] / tab[den]
    return None


def cmd_counters(args):
    """Per-dispatch averages of the counters of several --pmc runs for the
    dispatches whose kernel name contains --kernel, and the ratios read from
    them."""
    if args.kernel == "auto":
        # the step kernel with the most dispatches in the first run's timed region
        region, _ = _region(_dispatches(sqlite3.connect(args.dbs[0])))
        top = collections.Counter(d[1] for d in region if "k_lanczos_step" in d[1]).most_common(1)
        if not top:
            sys.exit("no step kernel in the timed region of " + args.dbs[0])
        args.kernel = _short(top[0][0])
    tab = {}
    for db in args.dbs:
        acc, calls, _ = _counter(db, (args.kernel,))
        per = collections.defaultdict(float)
        cnt = collections.Counter()
        for (k, ctr), v in acc.items():
            per[ctr] += v
            cnt[ctr] += calls[(k, ctr)]
        for ctr in per:
            tab[ctr] = per[ctr] / max(cnt[ctr], 1)
    out = ["# Hardware counters of `%s`" % args.kernel, "", "Commands (one rocprofv3 --pmc pass each):", "", "```"]
    out += args.cmd
    out += ["```", "", "| counter | per dispatch |", "|---|---:|"]
    for ctr in sorted(tab):
        out.append("| `%s` | %.4g |" % (ctr, tab[ctr]))
    derived = [
        ("L2 hit rate, TCC_HIT / (TCC_HIT + TCC_MISS)",
         _ratio({"h": tab.get("TCC_HIT_sum", 0.0), "t": tab.get("TCC_HIT_sum", 0.0) + tab.get("TCC_MISS_sum", 0.0)},
                "h", "t")),
        ("mean L1-to-L2 read latency, cycles", _ratio(tab, "TCP_TCC_READ_REQ_LATENCY_sum", "TCP_TCC_READ_REQ_sum")),
        ("wave-cycles waiting on a counter (s_waitcnt), SQ_WAIT_ANY / SQ_WAVE_CYCLES",
         _ratio(tab, "SQ_WAIT_ANY", "SQ_WAVE_CYCLES")),
        ("wave-cycles issuing, SQ_ACTIVE_INST_ANY / SQ_WAVE_CYCLES", _ratio(tab, "SQ_ACTIVE_INST_ANY", "SQ_WAVE_CYCLES")),
        ("TA busy per CU over GPU-active cycles (TA_TA_BUSY_sum / 256 CUs, GRBM_GUI_ACTIVE / 8 XCDs)",
         _ratio({"a": tab.get("TA_TA_BUSY_sum", 0.0) / 256.0, "b": tab.get("GRBM_GUI_ACTIVE", 0.0) / 8.0}, "a", "b")),
        ("TD cycles stalled on the L1 (TD_TC_STALL_sum / 256 CUs, over GRBM_GUI_ACTIVE / 8 XCDs)",
         _ratio({"a": tab.get("TD_TC_STALL_sum", 0.0) / 256.0, "b": tab.get("GRBM_GUI_ACTIVE", 0.0) / 8.0}, "a", "b")),
        ("L1-to-L2 read requests per vector-memory read instruction",
         _ratio(tab, "TCP_TCC_READ_REQ_sum", "SQ_INSTS_VMEM_RD")),
        ("L2-to-memory read requests that went to DRAM, TCC_EA0_RDREQ_DRAM / TCC_EA0_RDREQ",
         _ratio(tab, "TCC_EA0_RDREQ_DRAM_sum", "TCC_EA0_RDREQ_sum")),
    ]
    out += ["", "| derived | value |", "|---|---:|"]
    for name, v in derived:
        if v is not None:
            out.append("| %s | %.3g |" % (name, v))
    with open(args.out, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("\n".join(out))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("out")
    s.add_argument("--cmd", required=True)
    s.add_argument("--bench-line", help="output of the profiled bench.py run (its JSON line)")
    t = sub.add_parser("traffic")
    for k in ("fetch_db", "write_db", "copy_fetch_db", "copy_write_db", "out"):
        t.add_argument(k)
    t.add_argument("--workload", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--copies", type=int, default=3)
    t.add_argument("--cmd", required=True)
    v = sub.add_parser("serve")
    v.add_argument("line")
    v.add_argument("out")
    v.add_argument("--cmd", required=True)
    c = sub.add_parser("counters")
    c.add_argument("out")
    c.add_argument("dbs", nargs="+")
    c.add_argument("--kernel", required=True)
    c.add_argument("--cmd", action="append", required=True)
    args = ap.parse_args()
    {"stats": cmd_stats, "traffic": cmd_traffic, "serve": cmd_serve, "counters": cmd_counters}[args.what](args)


if __name__ == "__main__":
    main()
