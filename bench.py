#!/usr/bin/env python3
"""Throughput of the Lanczos-quadrature entropy hot path on one MI355X.

One step is one whole entropy estimate of the workload (probe block, every
Lanczos step, quadrature, estimator combine, results copied back to the
host), with the matrix already resident in HBM.  The default workload is the
single-large-graph configuration: Barabasi-Albert n = 200000, 3 edges per new
node, rho = L / tr(L), Hutch++ with 128 sketch + 128 Hutchinson Rademacher
vectors, 60 Lanczos steps, FP32 vectors with FP64 coefficients.

value = algorithmic bytes of all Lanczos step launches in the timed steps
divided by the timed wall-clock (GB/s).  Algorithmic bytes of one step
launch: 4 (n + 1) + nnz (4 + 4) + 3 n m 4 (CSR once; v_j gathered once,
v_{j-1} read once, v_{j+1} written once).  The roofline object reports the
same bytes over the step kernel's own HIP-event time.

The batch workload (512 ER/BA graphs, n log-uniform in [1e3, 5e4], 64
Rademacher probes each, 50 steps, FP32) runs every graph in one stacked
launch per Lanczos step; its line also reports the same queries issued one
graph at a time (one captured launch sequence per graph) and the speedup.

The serve workload submits Poisson streams of 1e-3 relative-accuracy
queries (probe count and steps from the serving error rule) on a pool of
ER / BA / WS graphs to the serving loop and reports completed queries/s and
p50/p99 latency per arrival rate.

The default line (large workload) also carries, measured in the same run,
a `serve` object (200 served 1e-3 queries at a light rate, 20/s, and near
saturation, 200/s: completed queries/s, p50/p99 latency, the fraction that
meets the sampling target and, for queries on the pool graphs small enough
for a dense eigendecomposition, the fraction within 1e-3 of the exact
entropy) and a `batch` object (the 512-graph stacked launch against the
same queries one graph per call, at equal accuracy).  `estimates_per_s`
and `estimate_p50_ms` / `estimate_p99_ms` of the line are back-to-back
large Hutch++ estimates, not served queries.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--workload large|tiny|probing|batch|serve|probing-eps|rational|
                                   hutchpp-adaptive]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def kernel_source_hash():
    """Hash of the sources that fix what the Lanczos step unit (normalize,
    step and long-row kernels) reads and writes per launch: the part of
    kernels.hip up to the finalize kernels, kernels.h up to the quadrature
    declarations, the work schedule builder and the runtime's schedule
    choice.  Counter figures taken on other sources are not reused."""
    csrc = os.path.join(ROOT, "paper_2212_09642_amd", "csrc")

    def text(name):
        with open(os.path.join(csrc, name)) as fh:
            return fh.read()

    def upto(src, marker):
        i = src.find(marker)
        if i < 0:
            raise RuntimeError("marker %r missing" % marker)
        return src[:i]

    parts = [upto(text("kernels.hip"), "// Finalize a step:"),
             upto(text("kernels.h"), "// Gauss quadrature of every column"),
             text("host_graph.cpp")]
    rt = text("runtime.hip")
    i = rt.find("Schedule set_schedule(")
    parts.append(rt[i:rt.find("\n}\n", i)] if i >= 0 else rt)
    h = hashlib.sha256()
    for part in parts:
        h.update(part.encode())
    return h.hexdigest()[:16]


def oracle_check(golden, estimate, **match):
    """The estimate against the oracle's FP64 value of the same problem (same
    graph, probes and sizes), read from a committed golden file written by a
    script under tests/golden/ that calls only the oracle; None when the file
    is missing or describes another problem."""
    path = os.path.join(ROOT, "tests", "golden", golden)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if any(d.get(k) != v for k, v in match.items()):
        return None
    ref = d["estimate"]
    return {"oracle_estimate": ref, "rel_err": abs(estimate - ref) / abs(ref), "bar": 1e-5,
            "oracle_rounding_spread": d.get("estimate_spread"), "golden": "tests/golden/" + golden}


def load_traffic(workload):
    """HBM bytes per step launch from the committed rocprofv3 counter summary
    (null when missing or taken on a different kernel source)."""
    path = os.path.join(ROOT, "profiles", "lanczos_step_%s_traffic.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def reorder_csr(g, how):
    """Relabel the rows of a registered-form CSR (experiment: locality of the
    gathers).  Row keys keep the original node ids, so the probes are the same."""
    import numpy as np
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    A = sp.csr_matrix((g["values"], g["col_idx"], g["row_ptr"]), shape=(g["n"], g["n"]))
    if how == "rcm":
        perm = reverse_cuthill_mckee(A, symmetric_mode=True)
    elif how == "degree":
        deg = np.diff(g["row_ptr"])
        perm = np.argsort(-deg, kind="stable")
    elif how == "random":
        perm = np.random.default_rng(12345).permutation(g["n"])
    else:
        raise SystemExit("unknown reorder %s" % how)
    B = A[perm][:, perm].tocsr()
    B.sort_indices()
    return dict(n=g["n"], row_ptr=B.indptr.astype(np.int32), col_idx=B.indices.astype(np.int32),
                values=B.data.astype(g["values"].dtype), node_ids=g["node_ids"][perm], scale=g["scale"])


def build_workload(name, reorder=None):
    import numpy as np
    import paper_2212_09642_amd as vne
    from synth import workloads
    if name == "large":
        w = workloads.large()
        m = w["n_sketch"] + w["n_hutch"]
        spec = dict(kind=vne.PROBE_HUTCHPP, m=m, k=w["k"], mode=vne.MODE_DESING,
                    seed=w["probe_seed"], n_sketch=w["n_sketch"])
    elif name == "tiny":
        w = workloads.tiny()
        spec = dict(kind=vne.PROBE_RADEMACHER, m=w["m"], k=w["k"],
                    mode=vne.MODE_DESING | vne.MODE_F64, seed=w["probe_seed"], n_sketch=0)
    elif name == "probing":
        w = workloads.probing()
        spec = dict(kind=vne.PROBE_COLORING, m=None, k=w["k"], mode=vne.MODE_DESING, seed=0,
                    n_sketch=0)
    else:
        raise SystemExit("unknown workload %s" % name)
    fp64 = bool(spec["mode"] & vne.MODE_F64)
    g = vne.laplacian_from_edges(w["n_nodes"], w["edges"], np.float64 if fp64 else np.float32)
    if reorder:
        g = reorder_csr(g, reorder)
    if name == "probing":
        col, s = vne.color_greedy(g["row_ptr"], g["col_idx"], g["values"], w["d"])
        spec["colors"] = col
        spec["m"] = s
    return w, g, spec


def region_marker():
    """One tiny kernel (torch's spin kernel) on the current stream: a pair of
    them brackets the timed region in a rocprofv3 trace, so the profile
    summaries leave out warm-up, tile tuning and what runs after.  Issued
    outside the timed interval."""
    import torch
    torch.cuda._sleep(1)


def cpu_baseline(g, spec, sample_cols, k):
    """The oracle (plain FP64 Lanczos + quadrature) on a bounded sample of the
    same workload: sample_cols Rademacher columns, all k steps."""
    import numpy as np
    import oracle
    import scipy.sparse as sp
    A = sp.csr_matrix((np.asarray(g["values"], np.float64) * g["scale"], g["col_idx"], g["row_ptr"]),
                      shape=(g["n"], g["n"]))
    B = oracle.rademacher_block(spec["seed"], g["node_ids"], np.arange(sample_cols))
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):        # one core, as reported
        t0 = time.perf_counter()
        oracle.quadforms(A, B, k, oracle.breakdown_tau(False))
        dt = time.perf_counter() - t0
    n, nnz = g["n"], len(g["col_idx"])
    bytes_equiv = k * (4.0 * (n + 1) + nnz * 8.0 + 3.0 * n * sample_cols * 4.0)
    return dict(value=bytes_equiv / dt / 1e9, unit="GB/s", cores=1, kind="oracle",
                sample="oracle Lanczos + Gauss quadrature on %d Rademacher columns x %d steps "
                       "of the same graph (%.1f s); GB/s counts the bytes the FP32 path would move "
                       "for the same steps" % (sample_cols, k, dt),
                host=host_cpu())


def host_cpu():
    """The host CPU the oracle ran on: model name, logical CPUs of the
    machine and CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def measure_batch(warmup, steps, cpu_seconds=None):
    """512 graphs, one stacked launch per step, against the same queries
    issued one graph per call.  Returns the timings, the kernel timing, the
    speedup at equal accuracy and (cpu_seconds given) the oracle's rate."""
    import numpy as np
    import torch
    import paper_2212_09642_amd as vne
    from synth import workloads
    specs = workloads.batch_specs()
    m, k, seed0 = 64, 50, workloads.PROBE_SEED
    t0 = time.perf_counter()
    graphs = [vne.laplacian_from_edges(*workloads.batch_graph(sp), np.float32) for sp in specs]
    stream = torch.cuda.current_stream().cuda_stream
    ctx = vne.Context(0, stream=stream)
    gids = [ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
            for g in graphs]
    queries = [dict(gid=gid, kind=vne.PROBE_RADEMACHER, m=m, k=k, seed=seed0 + q)
               for q, gid in enumerate(gids)]
    mode = vne.MODE_DESING
    n_tot = sum(g["n"] for g in graphs)
    nnz_tot = sum(len(g["col_idx"]) for g in graphs)
    print("batch workload: %d graphs, n=%d, nnz=%d (%.1f s to build and register)"
          % (len(graphs), n_tot, nnz_tot, time.perf_counter() - t0), file=sys.stderr, flush=True)

    def one():
        return ctx.estimate_batch(queries, mode)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    ctx.enable_kernel_timing(True)
    ctx.kernel_timing(reset=True)
    lat = []
    region_marker()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        outs = one()
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    region_marker()
    kt = ctx.kernel_timing(reset=True)
    ctx.enable_kernel_timing(False)
    print("batch timed: %.1f ms per batch" % (wall / steps * 1e3), file=sys.stderr, flush=True)

    # the same queries, one graph per call (each graph's own captured step
    # loop): one untimed pass (capture, tile choice), one timed pass
    def per_graph():
        return [ctx.estimate(q["gid"], q["kind"], q["m"], q["k"], mode, seed=q["seed"], want_coeffs=False)
                for q in queries]
    solo = per_graph()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    solo = per_graph()
    torch.cuda.synchronize()
    solo_s = time.perf_counter() - ts
    rel = max(abs(a["estimate"] - b["estimate"]) / abs(b["estimate"]) for a, b in zip(outs, solo))
    relq = max(float(np.max(np.abs(a["quad"] - b["quad"]) / np.abs(b["quad"]))) for a, b in zip(outs, solo))
    print("per-graph pass: %.1f ms" % (solo_s * 1e3), file=sys.stderr, flush=True)
    res = dict(name="batch512_er_ba_n1e3_5e4_hutchinson64_k50_f32", graphs=len(graphs), n_total=n_tot,
               nnz_total=nnz_tot, m=m, k=k, wall=wall, steps=steps, lat=lat, kt=kt,
               per_graph=dict(ms_per_batch=round(solo_s * 1e3, 3), queries_per_s=round(len(queries) / solo_s, 3),
                              speedup_of_stacked_launch=round(solo_s / (wall / steps), 3),
                              max_rel_diff_of_estimates=rel, max_rel_diff_of_quadratic_forms=relq))
    if cpu_seconds is not None:
        import oracle
        import scipy.sparse as sp
        from threadpoolctl import threadpool_limits
        limit = threadpool_limits(limits=1)   # one core, as reported
        t0 = time.perf_counter()
        done, by = 0, 0.0
        for q, g in enumerate(graphs):
            A = sp.csr_matrix((np.asarray(g["values"], np.float64) * g["scale"], g["col_idx"], g["row_ptr"]),
                              shape=(g["n"], g["n"]))
            B = oracle.rademacher_block(seed0 + q, g["node_ids"], np.arange(m))
            oracle.quadforms(A, B, k, oracle.breakdown_tau(False))
            done += 1
            by += k * (4.0 * (g["n"] + 1) + len(g["col_idx"]) * 8.0 + 3.0 * g["n"] * m * 4.0)
            if time.perf_counter() - t0 > cpu_seconds:
                break
        dt = time.perf_counter() - t0
        limit.restore_original_limits()
        res["cpu_baseline"] = dict(value=by / dt / 1e9, unit="GB/s", cores=1, kind="oracle",
                                   queries_per_s=done / dt,
                                   sample="oracle Lanczos + Gauss quadrature on the first %d graphs of the "
                                          "batch, 64 Rademacher columns x 50 steps each (%.1f s); GB/s counts "
                                          "the bytes the FP32 path would move for the same steps" % (done, dt))
    ctx.close()
    return res


def batch_summary(b):
    """The batch object of a bench line: stacked launch against per-graph
    launches at equal accuracy."""
    return {"workload": b["name"], "graphs": b["graphs"], "n_total": b["n_total"], "m": b["m"], "k": b["k"],
            "stacked_ms_per_batch": round(b["wall"] / b["steps"] * 1e3, 3),
            "stacked_queries_per_s": round(b["graphs"] * b["steps"] / b["wall"], 3),
            "per_graph_ms_per_batch": b["per_graph"]["ms_per_batch"],
            "per_graph_queries_per_s": b["per_graph"]["queries_per_s"],
            "speedup_of_stacked_launch": b["per_graph"]["speedup_of_stacked_launch"],
            "max_rel_diff_of_estimates": b["per_graph"]["max_rel_diff_of_estimates"],
            "max_rel_diff_of_quadratic_forms": b["per_graph"]["max_rel_diff_of_quadratic_forms"],
            "step_unit_avg_ms": round(b["kt"]["total_ms"] / max(b["kt"]["launches"], 1), 5)}


def run_batch(args):
    """512 graphs, one stacked launch per step, against per-graph launches."""
    import numpy as np
    b = measure_batch(args.warmup, args.steps, None if args.no_cpu_baseline else args.cpu_seconds)
    kt, wall, lat = b["kt"], b["wall"], b["lat"]
    value = kt["bytes"] / wall / 1e9
    achieved = kt["bytes"] / (kt["total_ms"] / 1e3) / 1e9 if kt["total_ms"] > 0 else 0.0
    name = b["name"]
    res = {
        "metric": "Lanczos SpMM GB/s (% HBM peak); entropy queries/s + p99 latency at 1e-3 rel",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": name, "graphs": b["graphs"], "n_total": b["n_total"], "nnz_total": b["nnz_total"],
                   "m": b["m"], "k": b["k"], "estimator": "hutchinson",
                   "graph_seed": __import__("synth").workloads.GRAPH_SEED_BATCH,
                   "probe_seed": __import__("synth").workloads.PROBE_SEED},
        "batch_queries_per_s": round(b["graphs"] * args.steps / wall, 3),
        "batch_p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
        "batch_p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4),
        "per_graph_launches": b["per_graph"],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": load_traffic(name),
                     "kernel": "k_lanczos_step", "launches": kt["launches"],
                     "avg_launch_ms": round(kt["total_ms"] / max(kt["launches"], 1), 5),
                     "algorithmic_bytes_per_launch": round(kt["bytes"] / max(kt["launches"], 1))},
        "cpu_baseline": b.get("cpu_baseline"),
    }
    print(json.dumps(res), flush=True)


def exact_entropy_dense(g):
    """S(rho) = -sum lambda log lambda over the eigenvalues of the dense
    rho = scale * L (eq. (2.1)); for the small graphs of the serving pool."""
    import numpy as np
    import scipy.sparse as sp
    L = sp.csr_matrix((np.asarray(g["values"], np.float64), g["col_idx"], g["row_ptr"]),
                      shape=(g["n"], g["n"])).toarray()
    lam = np.linalg.eigvalsh(L) * g["scale"]
    lam = lam[lam > 0]
    return float(-np.sum(lam * np.log(lam)))


def measure_serve(rates, queries, pool_size=24, arena_gb=96.0, max_slots=256, max_cols=256, zipf=0.0, pilot=0,
                  exact_n_max=4000, max_group=0, stop="bound"):
    """Poisson streams of 1e-3 relative-accuracy queries on a pool of ER / BA
    / WS graphs (n log-uniform in [1e3, 2e6]).  Per rate: completed queries/s,
    p50/p99 latency, the fraction that meet the sampling target, and on the
    pool graphs with n <= exact_n_max the fraction within 1e-3 of the exact
    entropy (dense eigendecomposition)."""
    import numpy as np
    import torch
    import paper_2212_09642_amd as vne
    from synth import workloads
    specs = workloads.serve_pool_specs(pool_size)
    stream = torch.cuda.current_stream().cuda_stream
    ctx = vne.Context(0, stream=stream)
    pool, exact = [], {}
    t0 = time.perf_counter()
    for i, sp in enumerate(specs):
        g = vne.laplacian_from_edges(*workloads.serve_graph(sp), np.float32)
        gid = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
        pool.append((gid, g["n"], len(g["col_idx"]), sp[0]))
        if g["n"] <= exact_n_max:
            exact[i] = exact_entropy_dense(g)
    print("serve pool: %d graphs, n %d..%d, exact entropy of %d (%.1f s)"
          % (len(pool), min(p[1] for p in pool), max(p[1] for p in pool), len(exact), time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    eps = 1e-3
    rules = [stop] if isinstance(stop, str) else list(stop)
    rows_by_rule = {}
    for rule in rules:
        rows_by_rule[rule] = serve_rates(ctx, vne, np, workloads, pool, exact, rates, queries, eps, arena_gb,
                                         max_slots, max_cols, zipf, pilot, max_group, rule)
    ctx.close()
    return dict(pool=len(pool), exact_graphs=len(exact), rows=rows_by_rule[rules[0]], rows_by_rule=rows_by_rule,
                rel_eps=eps)


def serve_rates(ctx, vne, np, workloads, pool, exact, rates, queries, eps, arena_gb, max_slots, max_cols, zipf,
                pilot, max_group, stop):
    """One server on the pool with the given stopping rule: Poisson streams at
    each rate; one result row per rate."""
    srv = vne.Server(ctx, vne.MODE_DESING, arena_bytes=int(arena_gb * (1 << 30)), max_slots=max_slots,
                     max_cols=max_cols, max_probes=4096, pilot_probes=pilot, max_group=max_group,
                     stop={"bound": vne.STOP_BOUND, "estimate": vne.STOP_ESTIMATE}[stop])
    # untimed: one query per graph (device arrays of every graph, first launches)
    for gid, *_ in pool:
        srv.poll(srv.submit(gid, rel_eps=eps, seed=1))
    rows = []
    prev = srv.stats()
    for rate in rates:
        rng = np.random.Generator(np.random.PCG64(workloads.GRAPH_SEED_SERVE + int(rate)))
        gaps = rng.exponential(1.0 / rate, queries)
        if zipf > 0:
            # skewed popularity: graph i (pool order) drawn with weight 1 / (i + 1)^s
            w = 1.0 / np.arange(1, len(pool) + 1) ** zipf
            picks = rng.choice(len(pool), size=queries, p=w / w.sum())
        else:
            picks = rng.integers(0, len(pool), queries)
        tickets = []
        t0 = time.perf_counter()
        due = t0
        for i in range(queries):
            due += gaps[i]
            now = time.perf_counter()
            if due > now:
                time.sleep(due - now)
            tickets.append((srv.submit(pool[picks[i]][0], rel_eps=eps, seed=1000 + i), picks[i]))
        res = [(srv.poll(t), pk) for t, pk in tickets]
        wall = time.perf_counter() - t0
        lat = np.array([r["latency_ms"] for r, _ in res])
        ok = sum(r["status"] == 0 for r, _ in res)
        # algorithmic bytes: per step CSR once + 3 n N vector words (FP32)
        by = sum(r["steps"] * (4.0 * (pool[pk][1] + 1) + 8.0 * pool[pk][2] + 12.0 * pool[pk][1] * r["probes"])
                 for r, pk in res)
        met = sum(2.576 * r["std_error"] <= 0.5 * eps * abs(r["estimate"]) for r, _ in res)
        with_exact = [(r, pk) for r, pk in res if pk in exact]
        within = sum(abs(r["estimate"] - exact[pk]) <= eps * exact[pk] for r, pk in with_exact)
        worst = max((abs(r["estimate"] - exact[pk]) / exact[pk] for r, pk in with_exact), default=None)
        info = srv.stats()
        # this rate's share of the server's running counters
        dt_ticks = max(1, info["ticks"] - prev["ticks"])
        occ = (info["slot_occupancy"] * info["ticks"] - prev["slot_occupancy"] * prev["ticks"]) / dt_ticks
        tasks, grouped = info["tasks"] - prev["tasks"], info["group_tasks"] - prev["group_tasks"]
        prev = info
        row = {"offered_per_s": rate, "queries": queries, "completed": ok,
               "completed_per_s": round(ok / wall, 3), "p50_ms": round(float(np.percentile(lat, 50)), 3),
               "p99_ms": round(float(np.percentile(lat, 99)), 3), "algorithmic_GBps": round(by / wall / 1e9, 2),
               "mean_probes": round(float(np.mean([r["probes"] for r, _ in res])), 1),
               "mean_steps": round(float(np.mean([r["steps"] for r, _ in res])), 1),
               "sampling_target_met": met, "fraction_sampling_target_met": round(met / queries, 4),
               "queries_with_exact_entropy": len(with_exact), "within_1e-3_of_exact": within,
               "worst_rel_err_vs_exact": worst,
               "slot_occupancy": round(occ, 2), "tasks": tasks, "tasks_in_group_slots": grouped}
        print("rate (stop %s) %s" % (stop, json.dumps(row)), file=sys.stderr, flush=True)
        rows.append(row)
    srv.stop()
    return rows


def serve_summary(sv, rates, queries):
    """The serve object of the default line: the rates under the first
    stopping rule measured (the upper bound, eq. (4.9)), and under each other
    rule (the eq. (4.10) estimate) on the same pool and arrivals."""
    rules = list(sv["rows_by_rule"])
    out = {"workload": "serve_pool%d_er_ba_ws_n1e3_2e6_eps1e-3_f32" % sv["pool"], "rel_eps": sv["rel_eps"],
           "pool_graphs": sv["pool"], "pool_seed": __import__("synth").workloads.GRAPH_SEED_SERVE,
           "arrivals": "Poisson, seed %d + rate" % __import__("synth").workloads.GRAPH_SEED_SERVE,
           "queries_per_rate": queries, "exact_entropy_graphs": sv["exact_graphs"], "stop": rules[0],
           "rates": sv["rows_by_rule"][rules[0]]}
    for rule in rules[1:]:
        out["stop_" + rule] = {"stop": rule, "rates": sv["rows_by_rule"][rule]}
    return out


def run_serve(args):
    """Poisson stream of 1e-3 relative-accuracy queries on a pool of ER / BA /
    WS graphs (n log-uniform in [1e3, 2e6]) at several arrival rates."""
    rates = [float(r) for r in args.rates.split(",")]
    sv = measure_serve(rates, args.queries, args.pool, args.arena_gb, args.max_slots, args.max_cols, args.zipf,
                       args.pilot, max_group=args.group, stop=args.stop)
    rows = sv["rows"]
    best = max(rows, key=lambda r: r["completed_per_s"])
    res = {
        "metric": "Lanczos SpMM GB/s (% HBM peak); entropy queries/s + p99 latency at 1e-3 rel",
        "value": best["completed_per_s"], "unit": "queries/s", "n_gpus": 1, "steps": args.queries,
        "warmup": sv["pool"], "ms_per_step": round(1e3 / max(best["completed_per_s"], 1e-9), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serve_pool%d_er_ba_ws_n1e3_2e6_eps1e-3_f32" % sv["pool"], "graphs": sv["pool"],
                   "rel_eps": sv["rel_eps"], "rates": args.rates, "queries_per_rate": args.queries,
                   "zipf": args.zipf, "pilot": args.pilot or 16, "max_group": args.group or 2, "max_slots": args.max_slots,
                   "stop": args.stop,
                   "graph_seed": __import__("synth").workloads.GRAPH_SEED_SERVE},
        "p50_ms": best["p50_ms"], "p99_ms": best["p99_ms"], "rates": rows,
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)


def _dense_quadform(g, c):
    """c^T f(rho) c by a dense eigendecomposition (eq. (2.1) applied to one
    form; small graphs only)."""
    import numpy as np
    import scipy.sparse as sp
    L = sp.csr_matrix((np.asarray(g["values"], np.float64), g["col_idx"], g["row_ptr"]),
                      shape=(g["n"], g["n"])).toarray() * g["scale"]
    lam, U = np.linalg.eigh(L)
    pr = (U.T @ c) ** 2
    pos = lam > 0
    return float(-np.sum(pr[pos] * lam[pos] * np.log(lam[pos]))), lam


def run_rational(args):
    """Rational Krylov cross-check against the Lanczos path at equal error:
    one desingularised random-sign form on an ill-conditioned path graph
    (n = 1000) and a 40 x 40 grid, relative error 1e-6 against a dense
    eigendecomposition.  Lanczos: the smallest k that meets it (one
    application of A per step).  Rational: poles at infinity, then 12
    negative poles log-spaced over [-lambda_max, -lambda_2] once the switch
    rule (ell = 3, c = 0.75, on Theorem 4.8's upper bound over [lambda_2,
    lambda_max]) fires; and separately a fixed sequence of 3
    poles at infinity followed by log-spaced poles over the rest of the
    basis.  Applications of A = basis vectors + conjugate-gradient
    iterations of the shifted solves (relative residual 1e-12).  Times are
    wall-clock per call (median of repeats, results copied to the host)."""
    import numpy as np
    import synth
    import paper_2212_09642_amd as vne
    tol = 1e-6
    mode = vne.MODE_F64 | vne.MODE_DESING
    ctx = vne.Context(0)
    cases = []
    for name in ("path1000", "grid40x40"):
        n0, e = synth.path_graph(1000) if name == "path1000" else synth.grid2d_graph(40, 40)
        g = vne.laplacian_from_edges(n0, e, np.float64)
        gid = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
        n = g["n"]
        b = np.random.default_rng(3).choice([-1.0, 1.0], size=(n, 1))
        c = b[:, 0] - b[:, 0].mean()
        exact, lam = _dense_quadform(g, c)
        lam = lam[lam > 1e-12 * lam[-1]]
        pr = dict(dense=b)

        def timed(fn, reps):
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                fn()
                ts.append((time.perf_counter() - t0) * 1e3)
            return float(np.median(ts))

        lanczos = None
        for k in range(1, 129):
            q = ctx.estimate(gid, vne.PROBE_DENSE, 1, k, mode, want_coeffs=False, **pr)["quad"][0]
            if abs(q - exact) <= tol * abs(exact):
                lanczos = k
                break
        row = dict(case=name, n=n, kappa=float(lam[-1] / lam[0]), rel_tol=tol)
        if lanczos is not None:
            ms = timed(lambda: ctx.estimate(gid, vne.PROBE_DENSE, 1, lanczos, mode, want_coeffs=False, **pr), 20)
            row["lanczos"] = dict(steps=lanczos, apps=lanczos, ms=ms)
        else:
            row["lanczos"] = None
        fin = list(-np.geomspace(lam[-1], lam[0], 12))
        sw = dict(finite_poles=fin, ell=3, c=0.75, cg_tol=1e-12, lam_lo=0.999 * lam[0], lam_hi=1.001 * lam[-1])
        r = ctx.rational(gid, vne.PROBE_DENSE, 1, mode, 48, **sw, **pr)
        err = np.abs(r["psi_steps"][0] - exact) / abs(exact)
        ok = np.nonzero(err <= tol)[0]
        row["switch_rule"] = None
        if ok.size:
            j = int(ok[0]) + 1
            rr = ctx.rational(gid, vne.PROBE_DENSE, 1, mode, j, **sw, **pr)
            ms = timed(lambda: ctx.rational(gid, vne.PROBE_DENSE, 1, mode, j, **sw, **pr), 5)
            row["switch_rule"] = dict(steps=j, apps=int(rr["apps_steps"][0, -1]),
                                      cg_iterations=int(rr["cg_iterations"]),
                                      switch_step=int(rr["switch_step"][0]), ms=ms)
        row["fixed_poles"] = None
        for mm in range(4, 49):
            poles = [np.inf] * 3 + list(-np.geomspace(lam[-1], lam[0], mm - 4))
            rr = ctx.rational(gid, vne.PROBE_DENSE, 1, mode, mm, poles=poles, cg_tol=1e-12, **pr)
            if abs(rr["quad"][0] - exact) <= tol * abs(exact):
                ms = timed(lambda: ctx.rational(gid, vne.PROBE_DENSE, 1, mode, mm, poles=poles, cg_tol=1e-12,
                                                **pr), 5)
                row["fixed_poles"] = dict(steps=mm, apps=int(rr["apps_steps"][0, -1]),
                                          cg_iterations=int(rr["cg_iterations"]), ms=ms)
                break
        cases.append(row)
        print(json.dumps(row), flush=True)
    ctx.close()
    print(json.dumps({"metric": "rational_vs_lanczos_at_equal_error", "unit": "applications of A", "n_gpus": 1,
                      "dtype": "f64", "data": "synthetic", "higher_is_better": False,
                      "config": {"workload": "rational_path1000_grid40x40_tol1e-6"}, "cases": cases}), flush=True)


def run_hutchpp_adaptive(args):
    """Adaptive Hutch++ (vne_hutchpp_adaptive) on the large workload's graph
    (BA n = 2e5, FP32 vectors, k = 60 steps per Krylov run) at relative
    targets 1e-2 (the paper's setting for large matrices) and 1e-3 with
    delta = 1e-2, beside the fixed 128 + 128 Hutch++ of the large workload.
    Wall-clock per estimate: median of --steps calls after --warmup (plans
    and tiles are made in the warm-up)."""
    import numpy as np
    import paper_2212_09642_amd as vne
    from synth import workloads
    w = workloads.large()
    g = vne.laplacian_from_edges(w["n_nodes"], w["edges"], np.float32)
    ctx = vne.Context(0)
    gid = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
    k, seed, mode = w["k"], w["probe_seed"], vne.MODE_DESING

    def timed(fn):
        for _ in range(max(args.warmup, 1)):
            out = fn()
        ts = []
        for _ in range(max(args.steps, 1)):
            t0 = time.perf_counter()
            out = fn()
            ts.append((time.perf_counter() - t0) * 1e3)
        return out, float(np.median(ts))

    m = w["n_sketch"] + w["n_hutch"]
    fixed, fixed_ms = timed(lambda: ctx.estimate(gid, vne.PROBE_HUTCHPP, m, k, mode, seed=seed,
                                                 n_sketch=w["n_sketch"], want_coeffs=False))
    rows = []
    for eps in (1e-2, 1e-3):
        out, ms = timed(lambda: ctx.hutchpp_adaptive(gid, k, rel_eps=eps, delta=1e-2, mode=mode, seed=seed))
        chk = oracle_check("hutchpp_adaptive_large.json", out["estimate"], rel_eps=eps, delta=1e-2, k=k,
                           probe_seed=seed, n=g["n"], nnz=len(g["col_idx"]))
        rows.append(dict(rel_eps=eps, delta=1e-2, ms=round(ms, 3), n_sketch=out["n_sketch"], n_hutch=out["n_hutch"],
                         oracle_check=chk,
                         rounds=[(r["nr"], r["nh"]) for r in out["rounds"]], krylov_runs=out["krylov_runs"],
                         estimate=out["estimate"], std_error=out["std_error"], eps_hat=out["eps_hat"],
                         capped=out["capped"],
                         vs_fixed_sigmas=abs(out["estimate"] - fixed["estimate"]) / max(out["std_error"], 1e-300)))
        print(json.dumps(rows[-1]), flush=True)
    ctx.close()
    print(json.dumps({"metric": "adaptive_hutchpp_ms_per_estimate", "unit": "ms", "n_gpus": 1, "dtype": "f32",
                      "data": "synthetic", "higher_is_better": False,
                      "config": {"workload": w["name"].replace("hutchpp256", "hutchpp_adaptive"), "k": k},
                      "fixed_hutchpp_128_128": {"ms": round(fixed_ms, 3), "estimate": fixed["estimate"],
                                                "krylov_runs": 128 + 256},
                      "adaptive": rows}), flush=True)


def ring_lattice_entropy(n, k):
    """Exact S(rho) of the ring lattice Laplacian (circulant: eigenvalues
    k - 2 sum_{r=1..k/2} cos(2 pi j r / n))."""
    import numpy as np
    j = np.arange(n, dtype=np.float64)
    lam = np.full(n, float(k))
    for r in range(1, k // 2 + 1):
        lam -= 2.0 * np.cos(2.0 * np.pi * j * r / n)
    rho = lam / lam.sum()
    rho = rho[rho > 0]
    return float(-np.sum(rho * np.log(rho)))


def run_probing_eps(args):
    """Algorithm 2 end to end: colourings on the host, per-colour stopping on
    the GPU.  Wall time per estimate; the step kernels' roofline from a
    separate pass with kernel timing on (timed runs use the captured chunk
    graphs, timing runs plain launches)."""
    import numpy as np
    import torch
    import paper_2212_09642_amd as vne
    from synth import workloads
    w = workloads.probing_eps(args.graph, rel_eps=args.rel_eps)
    g = vne.laplacian_from_edges(w["n_nodes"], w["edges"], np.float32)
    n, nnz = g["n"], len(g["col_idx"])
    stream = torch.cuda.current_stream().cuda_stream
    ctx = vne.Context(0, stream=stream)
    gid = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])

    stop = {"bound": vne.STOP_BOUND, "estimate": vne.STOP_ESTIMATE}[args.stop]

    def one():
        return ctx.probing(gid, w["rel_eps"], d_max=16, k_max=128, mode=vne.MODE_DESING, stop=stop)

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    lat, outs = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        outs.append(one())
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.enable_kernel_timing(True)
    ctx.kernel_timing(reset=True)
    one()
    kt = ctx.kernel_timing(reset=True)
    ctx.enable_kernel_timing(False)
    o = outs[-1]
    achieved = kt["bytes"] / (kt["total_ms"] / 1e3) / 1e9 if kt["total_ms"] > 0 else 0.0
    res = {
        "metric": "Algorithm 2 estimates/s (probing with a relative target)",
        "value": round(args.steps / wall, 4), "unit": "estimates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w["name"], "n": n, "nnz": nnz, "rel_eps": w["rel_eps"], "d_max": 16, "k_max": 128,
                   "graph_seed": w["graph_seed"], "krylov_stop": args.stop},
        "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
        "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
        "estimate": o["estimate"], "d": o["d"], "n_colors": o["n_colors"], "passes": o["passes"],
        "fallback": o["fallback"], "capped": o["capped"], "t_pre": o["t_pre"], "eps_hat": o["eps_hat"],
        "vector_steps": o["vector_steps"], "block_steps": o["block_steps"], "unconverged": o["unconverged"],
        "color_ms": round(o["color_ms"], 3), "lanczos_ms": round(o["lanczos_ms"], 3),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "k_lanczos_step",
                     "launches": kt["launches"], "avg_launch_ms": round(kt["total_ms"] / max(kt["launches"], 1), 5),
                     "algorithmic_bytes_per_launch": round(kt["bytes"] / max(kt["launches"], 1))},
        "cpu_baseline": None,
    }
    if w["graph"] == "ring":
        S = ring_lattice_entropy(n, 10)
        res["exact_entropy"] = S
        res["rel_err_vs_exact"] = abs(o["estimate"] - S) / S
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = probing_eps_cpu_baseline(w)
    ctx.close()
    print(json.dumps(res), flush=True)


def probing_eps_cpu_baseline(w, n_small=20_000):
    """The oracle's Algorithm 2 on the same graph family at n = 2e4 (its
    colouring forms powers of the pattern, so the full graph is out of reach
    in seconds); the rate is scaled by n to the full size."""
    import oracle
    from oracle import probing as oprobing
    from synth import graphs, workloads
    from threadpoolctl import threadpool_limits
    if w["graph"] == "ring":
        nn, e = graphs.ring_lattice(n_small, 10)
    else:
        nn, e = graphs.watts_strogatz(n_small, 10, 0.1, workloads.GRAPH_SEED_PROBING)
    ref = oracle.laplacian_from_edges(nn, e)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        out = oprobing.probing_entropy(ref, w["rel_eps"], d_max=16, k_max=128)
        dt = time.perf_counter() - t0
    scale = n_small / float(w["n_nodes"])
    return dict(value=scale / dt, unit="estimates/s", cores=1, kind="oracle",
                sample="oracle Algorithm 2 on the same family at n=%d (%.1f s, d=%d, %d colours); "
                       "rate scaled by n to n=%d" % (n_small, dt, out["d"], out["final"]["n_colors"],
                                                      w["n_nodes"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--cpu-sample-cols", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--reorder", default=None, help="experiment: relabel rows (rcm | degree | random)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="batch workload: seconds of oracle work in the CPU baseline sample")
    ap.add_argument("--rates", default="10,50,200,1000,2000", help="serve workload: arrival rates (1/s)")
    ap.add_argument("--queries", type=int, default=200, help="serve workload: queries per rate")
    ap.add_argument("--pool", type=int, default=24, help="serve workload: graphs in the pool")
    ap.add_argument("--arena-gb", type=float, default=96.0, help="serve workload: server arena (GiB)")
    ap.add_argument("--max-slots", type=int, default=256, help="serve workload: tasks running at once")
    ap.add_argument("--max-cols", type=int, default=256, help="serve workload: probe columns per task")
    ap.add_argument("--pilot", type=int, default=0,
                    help="serve workload: pilot probes of a query (0: the server's default, 16)")
    ap.add_argument("--group", type=int, default=0,
                    help="serve workload: largest group slot of 16-column tasks, 1, 2 or 4 (0: the server's default)")
    ap.add_argument("--zipf", type=float, default=0.0,
                    help="serve workload: Zipf exponent of graph popularity (0: uniform)")
    ap.add_argument("--graph", default="ws", help="probing-eps workload: ws (small-world) or ring (lattice)")
    ap.add_argument("--rel-eps", type=float, default=1e-3, help="probing-eps workload: relative target")
    ap.add_argument("--stop", default="bound", choices=("bound", "estimate"),
                    help="probing-eps and serve workloads: Krylov stopping rule, the upper bound of the "
                         "bracket (eq. (4.9)) or its geometric mean (eq. (4.10))")
    ap.add_argument("--no-extras", action="store_true",
                    help="large workload: skip the serve and batch objects of the default line")
    ap.add_argument("--serve-rates", default="20,300",
                    help="large workload: arrival rates of the serve object (a light one, one near saturation)")
    ap.add_argument("--serve-queries", type=int, default=200, help="large workload: queries per serve rate")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 2 GiB device copy (for counter calibration)")
    ap.add_argument("--copy-rate", action="store_true",
                    help="time a plain 2 GiB device copy (read + write GB/s)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2212_09642_amd as vne

    if args.copy_calibration:
        x = torch.ones(1 << 29, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": x.numel() * 4, "copies": 3}))
        return
    if args.copy_rate:
        # the read + write rate a plain 2 GiB device copy reaches (context for
        # the step kernels' measured HBM traffic)
        x = torch.ones(1 << 29, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        print(json.dumps({"copy_bytes_each_way": x.numel() * 4, "copy_ms": round(ms, 4),
                          "copy_read_write_GBps": round(2 * x.numel() * 4 / (ms * 1e-3) / 1e9, 1)}))
        return

    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "serve":
        run_serve(args)
        return
    if args.workload == "probing-eps":
        run_probing_eps(args)
        return
    if args.workload == "rational":
        run_rational(args)
        return
    if args.workload == "hutchpp-adaptive":
        run_hutchpp_adaptive(args)
        return

    w, g, spec = build_workload(args.workload, args.reorder)
    n, nnz = g["n"], len(g["col_idx"])
    stream = torch.cuda.current_stream().cuda_stream
    ctx = vne.Context(0, stream=stream)
    gid = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
    if spec.get("colors") is not None:
        # the colouring is an input: resident in HBM before the timed region
        spec["colors"] = torch.from_numpy(np.ascontiguousarray(spec["colors"], np.int32)).to("cuda")

    def one():
        return ctx.estimate(gid, spec["kind"], spec["m"], spec["k"], spec["mode"], seed=spec["seed"],
                            n_sketch=spec["n_sketch"], colors=spec.get("colors"), want_coeffs=False)

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    ctx.enable_kernel_timing(True)
    ctx.kernel_timing(reset=True)
    lat = []
    region_marker()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        out = one()
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    region_marker()
    kt = ctx.kernel_timing(reset=True)
    ctx.enable_kernel_timing(False)

    value = kt["bytes"] / wall / 1e9
    achieved = kt["bytes"] / (kt["total_ms"] / 1e3) / 1e9 if kt["total_ms"] > 0 else 0.0
    traffic = load_traffic(w["name"])
    fp64 = bool(spec["mode"] & vne.MODE_F64)
    res = {
        "metric": "Lanczos SpMM GB/s (% HBM peak); entropy queries/s + p99 latency at 1e-3 rel",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if fp64 else "f32",
        "data": "synthetic",
        "config": {"workload": w["name"], "n": n, "nnz": nnz, "m": spec["m"], "k": spec["k"],
                   "estimator": {vne.PROBE_HUTCHPP: "hutch++", vne.PROBE_RADEMACHER: "hutchinson",
                                 vne.PROBE_COLORING: "probing"}[spec["kind"]],
                   "n_sketch": spec["n_sketch"], "graph_seed": w.get("graph_seed"), "probe_seed": spec["seed"]},
        "estimates_per_s": round(args.steps / wall, 3),
        "estimate_p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
        "estimate_p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4),
        "estimate": out["estimate"],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "traffic_counts": "bytes leaving L2 per step launch (FETCH_SIZE and WRITE_SIZE scaled by "
                                       "a plain 2 GiB copy); the Infinity Cache serves part of them",
                     "kernel": "k_lanczos_step", "launches": kt["launches"],
                     "avg_launch_ms": round(kt["total_ms"] / max(kt["launches"], 1), 5),
                     "algorithmic_bytes_per_launch": round(kt["bytes"] / max(kt["launches"], 1))},
        "cpu_baseline": None,
    }
    if args.workload == "large":
        res["oracle_check"] = oracle_check("hutchpp_large.json", out["estimate"], workload=w["name"], n=n, nnz=nnz,
                                           n_sketch=spec["n_sketch"], k=spec["k"], probe_seed=spec["seed"])
    if not args.no_cpu_baseline and args.workload in ("large", "tiny"):
        res["cpu_baseline"] = cpu_baseline(g, spec, min(args.cpu_sample_cols, spec["m"]), spec["k"])
    ctx.close()
    if args.workload == "large" and not args.no_extras:
        # the other halves of the metric, measured in the same run: served
        # 1e-3 queries (a light and a near-saturation rate) and the 512-graph
        # batch against per-graph launches
        rates = [float(r) for r in args.serve_rates.split(",")]
        sv = measure_serve(rates, args.serve_queries, stop=("bound", "estimate"))
        res["serve"] = serve_summary(sv, rates, args.serve_queries)
        res["batch"] = batch_summary(measure_batch(1, 3))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
