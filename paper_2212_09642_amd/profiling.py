"""Summaries of rocprofv3 output databases (the rocpd SQLite files that
``rocprofv3 -d DIR -o run`` writes) for the files kept under profiles/.

    python -m paper_2212_09642_amd.profiling stats DB OUT.md --cmd "..."
    python -m paper_2212_09642_amd.profiling traffic FETCH_DB WRITE_DB COPY_FETCH_DB \
        COPY_WRITE_DB OUT.json --workload NAME --copy-bytes B --cmd "..."
    python -m paper_2212_09642_amd.profiling serve BENCH_LINE.json OUT.md --cmd "..."
    python -m paper_2212_09642_amd.profiling counters OUT.md --kernel NAME DB [DB ...] --cmd "..."

The Lanczos step unit is the normalize pass (two-pass schedule), the SpMM +
recurrence kernel and the long-row kernel of one step; its average duration
is what bench.py times with HIP events around each step.
"""
import argparse
import collections
import json
import os
import sqlite3
import sys

STEP_KERNELS = ("k_normalize", "k_lanczos_step", "k_long_rows")


def _short(name):
    return name.split("(")[0].replace("void ", "").replace("vne::", "")


def kernel_stats(db):
    con = sqlite3.connect(db)
    rows = list(con.execute("select name, total_calls, total_duration, average from top_kernels"))
    # the top_kernels view reports microseconds
    return [(n, int(c), float(t), float(a)) for n, c, t, a in rows]


def step_unit(rows):
    steps = sum(c for n, c, t, a in rows if "k_lanczos_step" in n)
    total = sum(t for n, c, t, a in rows if any(k in n for k in STEP_KERNELS))
    return steps, total


def cmd_stats(args):
    rows = kernel_stats(args.db)
    tot = sum(r[2] for r in rows)
    out = ["# rocprofv3 kernel statistics", "", "Command:", "", "```", args.cmd, "```", "",
           "| kernel | calls | total ms | avg us | share |", "|---|---:|---:|---:|---:|"]
    for n, c, t, a in rows:
        out.append("| `%s` | %d | %.3f | %.2f | %.1f%% |" % (_short(n), c, t / 1e3, a, 100 * t / tot))
    steps, st = step_unit(rows)
    out += ["", "All kernels: %.3f ms." % (tot / 1e3),
            "Lanczos step unit (normalize + SpMM/recurrence + long rows): %d steps, %.3f ms total, "
            "%.2f us average per step." % (steps, st / 1e3, st / max(steps, 1))]
    with open(args.out, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("\n".join(out))


def _counter(db, name_filter=None, skip_steps=0, max_steps=0):
    """Counter sums per (kernel, counter) over the dispatches matching
    name_filter, in dispatch order.  skip_steps / max_steps (with step
    kernels in the filter) keep the dispatches from the (skip_steps + 1)-th
    Lanczos step kernel on, for max_steps steps (0: all): a step's normalize
    pass comes before its step kernel, its long rows after."""
    con = sqlite3.connect(db)
    acc = collections.defaultdict(float)
    calls = collections.Counter()
    rows = con.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection "
                       "order by dispatch_id").fetchall()
    step_no = 0          # index of the step the current dispatch belongs to
    seen_step = False
    for _, kname, ctr, val in rows:
        if name_filter and not any(k in kname for k in name_filter):
            continue
        if "k_normalize" in kname and seen_step:
            step_no += 1
            seen_step = False
        if "k_lanczos_step" in kname:
            seen_step = True
        if step_no < skip_steps or (max_steps and step_no >= skip_steps + max_steps):
            continue
        acc[(kname, ctr)] += float(val)
        calls[(kname, ctr)] += 1
    return acc, calls


def cmd_traffic(args):
    fetch, fcalls = _counter(args.fetch_db, STEP_KERNELS, args.skip_steps, args.max_steps)
    write, wcalls = _counter(args.write_db, STEP_KERNELS, args.skip_steps, args.max_steps)
    cf, _ = _counter(args.copy_fetch_db, ("copyBuffer",))
    cw, _ = _counter(args.copy_write_db, ("copyBuffer",))
    # calibration: what the counters read (KiB per dispatch) for a plain copy
    # of known size, one dispatch per copy
    copy_fetch_kib = sum(cf.values()) / max(args.copies, 1)
    copy_write_kib = sum(cw.values()) / max(args.copies, 1)
    f_scale = args.copy_bytes / (copy_fetch_kib * 1024.0)
    w_scale = args.copy_bytes / (copy_write_kib * 1024.0)
    steps = sum(c for (k, _), c in fcalls.items() if "k_lanczos_step" in k)
    fetch_kib = sum(fetch.values())
    write_kib = sum(write.values())
    per_step = (fetch_kib * f_scale + write_kib * w_scale) * 1024.0 / max(steps, 1)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    d = {"workload": args.workload, "kernel": "Lanczos step unit (" + ", ".join(STEP_KERNELS) + ")",
         "steps": steps, "fetch_kib_total": fetch_kib, "write_kib_total": write_kib,
         "copy_calibration": {"bytes_each_way": args.copy_bytes, "fetch_kib": copy_fetch_kib,
                              "write_kib": copy_write_kib, "fetch_scale": f_scale, "write_scale": w_scale},
         "hbm_bytes_per_launch": per_step, "kernel_source_hash": bench.kernel_source_hash(),
         "skip_steps": args.skip_steps, "max_steps": args.max_steps, "command": args.cmd}
    with open(args.out, "w") as fh:
        json.dump(d, fh, indent=1)
    print(json.dumps(d, indent=1))


def cmd_serve(args):
    """Rate table of a `bench.py --workload serve` line."""
    with open(args.line) as fh:
        d = json.loads(fh.read().strip().splitlines()[-1])
    c = d["config"]
    out = ["# Serving loop: Poisson arrivals at several rates", "", "Command:", "", "```", args.cmd, "```", "",
           "Workload `%s`: %d graphs, relative accuracy %g per query, %d queries per rate."
           % (c["workload"], c["graphs"], c["rel_eps"], c["queries_per_rate"]), "",
           "| offered /s | completed /s | p50 ms | p99 ms | algorithmic GB/s | mean probes | mean steps | "
           "sampling target met | running tasks per tick | tasks in pair slots |",
           "|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in d["rates"]:
        pairs = "%d/%d" % (r["tasks_in_pair_slots"], r["tasks"]) if "tasks" in r else "-"
        out.append("| %g | %.1f | %.1f | %.1f | %.0f | %.0f | %.1f | %d/%d | %.2f | %s |" % (
            r["offered_per_s"], r["completed_per_s"], r["p50_ms"], r["p99_ms"], r["algorithmic_GBps"],
            r["mean_probes"], r["mean_steps"], r["sampling_target_met"], r["queries"], r["slot_occupancy"],
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
    tab = {}
    for db in args.dbs:
        acc, calls = _counter(db, (args.kernel,))
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
    t = sub.add_parser("traffic")
    for k in ("fetch_db", "write_db", "copy_fetch_db", "copy_write_db", "out"):
        t.add_argument(k)
    t.add_argument("--workload", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--copies", type=int, default=3)
    t.add_argument("--skip-steps", type=int, default=0, help="leave out the first Lanczos steps (autotuning)")
    t.add_argument("--max-steps", type=int, default=0, help="count this many steps after those (0: all)")
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
