"""GPU tests of the serving loop (continuous batching with HBM-budget
admission): results against the FP64 oracle, the same bits alone and in a
mix of concurrent queries, admission under a small arena, the error rule's
accuracy on graphs whose entropy is known exactly, and error paths."""
import time

import numpy as np
import pytest

import oracle
import synth
import paper_2212_09642_amd as vne
from gpu_common import TOL, ctx, _say, _rel, _order_sensitivity, _bar, _assert_within  # noqa: F401

pytestmark = pytest.mark.gpu

MODE = vne.MODE_DESING


def _reg(ctx, n, e, fp64=False):
    g = vne.laplacian_from_edges(n, e, np.float64 if fp64 else np.float32)
    ref = oracle.laplacian_from_edges(n, e)
    gid = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
    return gid, ref


@pytest.fixture(scope="module")
def pool(ctx):
    makers = [lambda: synth.erdos_renyi(3000, 8.0, 41), lambda: synth.barabasi_albert(5000, 3, 42),
              lambda: synth.watts_strogatz(4000, 10, 0.1, 43), lambda: synth.star_graph(700),
              lambda: synth.grid2d_graph(40, 30), lambda: synth.erdos_renyi(20000, 6.0, 44)]
    return [_reg(ctx, *mk()) for mk in makers]


def _run_one(srv, gid, m, k, seed):
    t = srv.submit(gid, m=m, k=k, seed=seed)
    return srv.poll(t, want_quad=True)


def test_server_explicit_queries_match_oracle(ctx, pool):
    _say("case server: explicit m, k against the oracle")
    with vne.Server(ctx, MODE, arena_bytes=1 << 30) as srv:
        tickets = []
        for i, (gid, ref) in enumerate(pool[:5]):
            m, k = (8, 33, 64, 5, 300)[i], (20, 30, 25, 10, 15)[i]
            tickets.append((srv.submit(gid, m=m, k=k, seed=500 + i), gid, ref, m, k, 500 + i))
        for t, gid, ref, m, k, seed in tickets:
            r = srv.poll(t, want_quad=True)
            _say("  n=%d m=%d k=%d status=%d latency %.2f ms" % (ref.n, m, k, r["status"], r["latency_ms"]))
            assert r["status"] == 0, r["message"]
            assert r["probes"] == m and r["steps"] == k
            B = oracle.rademacher_block(seed, ref.node_ids, np.arange(m))
            want = oracle.quadforms(ref.scipy(), B, k, oracle.breakdown_tau(False))
            sens = _order_sensitivity(ref.scipy(), B, k, False)
            _assert_within(_rel(r["quad"], want["psi"]), _bar(False, sens), "n=%d m=%d k=%d" % (ref.n, m, k))
            assert abs(r["estimate"] - r["quad"].mean()) <= 1e-13 * abs(r["estimate"])


def test_server_same_bits_alone_and_in_a_mix(ctx, pool):
    _say("case server: a query alone and among concurrent queries")
    gid, ref = pool[1]
    with vne.Server(ctx, MODE, arena_bytes=1 << 30) as srv:
        alone = _run_one(srv, gid, 40, 30, 77)
        assert alone["status"] == 0
        # the same query submitted while other queries of other sizes run,
        # arrive and leave
        rng = np.random.default_rng(0)
        tickets = []
        for i in range(12):
            g2, _ = pool[int(rng.integers(0, len(pool)))]
            tickets.append(srv.submit(g2, m=int(rng.integers(1, 300)), k=int(rng.integers(5, 60)), seed=i))
            if i == 5:
                mine = srv.submit(gid, m=40, k=30, seed=77)
            time.sleep(0.002)
        mixed = srv.poll(mine, want_quad=True)
        others = [srv.poll(t) for t in tickets]
        info = srv.stats()
    assert all(o["status"] == 0 for o in others)
    assert mixed["status"] == 0
    assert np.array_equal(alone["quad"], mixed["quad"])
    assert alone["estimate"] == mixed["estimate"]
    _say("  ticks %d, mean running tasks per tick %.2f" % (info["ticks"], info["slot_occupancy"]))
    assert info["slot_occupancy"] > 1.0


def test_server_adaptive_same_bits_alone_and_in_a_mix(ctx, pool):
    """rel_eps queries stop on the a-posteriori bound; the step the device
    records decides the result, so a query alone and in a mix agree bitwise."""
    _say("case server: adaptive query alone and in a mix")
    gid, ref = pool[1]
    with vne.Server(ctx, MODE, arena_bytes=1 << 30) as srv:
        alone = srv.poll(srv.submit(gid, rel_eps=1e-3, seed=5), want_quad=True)
        tickets = []
        for i in range(10):
            tickets.append(srv.submit(pool[i % len(pool)][0], rel_eps=1e-3, seed=100 + i))
            if i == 4:
                mine = srv.submit(gid, rel_eps=1e-3, seed=5)
            time.sleep(0.001)
        mixed = srv.poll(mine, want_quad=True)
        others = [srv.poll(t) for t in tickets]
    assert alone["status"] == 0 and mixed["status"] == 0 and all(o["status"] == 0 for o in others)
    _say("  steps %d, probes %d" % (alone["steps"], alone["probes"]))
    assert alone["probes"] == mixed["probes"]
    assert np.array_equal(alone["quad"], mixed["quad"])
    assert alone["estimate"] == mixed["estimate"]


@pytest.mark.parametrize("group", [2, 4, 1])
def test_server_group_slots_same_bits_as_alone(ctx, pool, group):
    """16-column tasks of one graph with the same step cap share group slots
    of up to `group` tasks; each gives the bits it gives alone, and matches
    the oracle."""
    _say("case server: group slots of up to %d 16-column tasks" % group)
    gid, ref = pool[5]                       # ER n = 20000
    gid2, _ = pool[1]
    # ER (no long rows) and BA (hub rows split into segments) pairs
    work = ([(gid, 16, 30, s) for s in range(1, 7)] + [(gid, 16, 25, 7), (gid2, 16, 30, 8), (gid, 40, 30, 9)]
            + [(gid2, 16, 30, 10), (gid2, 16, 30, 11)])
    with vne.Server(ctx, MODE, arena_bytes=1 << 30, max_group=1) as srv:
        alone = [_run_one(srv, *w) for w in work]
        assert srv.stats()["group_tasks"] == 0
    with vne.Server(ctx, MODE, arena_bytes=1 << 30, max_group=group) as srv:
        ts = [srv.submit(g, m=m, k=k, seed=sd) for g, m, k, sd in work]
        mixed = [srv.poll(t, want_quad=True) for t in ts]
        info = srv.stats()
    fours = info["group_tasks"] - 2 * info["pair_slots"]
    _say("  %d of %d tasks in group slots (%d pair slots)" % (info["group_tasks"], info["tasks"], info["pair_slots"]))
    # submissions race the worker: most tasks join a group
    if group == 1:
        assert info["group_tasks"] == 0
    elif group == 2:
        assert info["pair_slots"] >= 3 and fours == 0
    else:
        assert fours >= 4
    for a, b in zip(alone, mixed):
        assert a["status"] == 0 and b["status"] == 0
        assert np.array_equal(a["quad"], b["quad"])
        assert a["estimate"] == b["estimate"]
    B = oracle.rademacher_block(3, ref.node_ids, np.arange(16))
    want = oracle.quadforms(ref.scipy(), B, 30, oracle.breakdown_tau(False))
    sens = _order_sensitivity(ref.scipy(), B, 30, False)
    _assert_within(_rel(mixed[2]["quad"], want["psi"]), _bar(False, sens), "group member vs oracle")


@pytest.mark.parametrize("group", [2, 4])
def test_server_adaptive_groups_same_bits_as_alone(ctx, pool, group):
    """rel_eps queries on one graph: their 16-column pilots share group slots,
    each member stops on its own record, and every query gives the bits it
    gives alone."""
    _say("case server: adaptive queries in group slots of up to %d" % group)
    gid, _ = pool[5]
    seeds = [21, 22, 23, 24, 25, 26]
    with vne.Server(ctx, MODE, arena_bytes=1 << 30, max_group=1) as srv:
        alone = [srv.poll(srv.submit(gid, rel_eps=1e-3, seed=sd), want_quad=True) for sd in seeds]
    with vne.Server(ctx, MODE, arena_bytes=1 << 30, max_group=group) as srv:
        ts = [srv.submit(gid, rel_eps=1e-3, seed=sd) for sd in seeds]
        mixed = [srv.poll(t, want_quad=True) for t in ts]
        info = srv.stats()
    _say("  %d of %d tasks in group slots (%d pair slots); steps %s"
         % (info["group_tasks"], info["tasks"], info["pair_slots"], [r["steps"] for r in alone]))
    assert info["group_tasks"] >= 4
    for a, b in zip(alone, mixed):
        assert a["status"] == 0 and b["status"] == 0
        assert a["probes"] == b["probes"]
        assert np.array_equal(a["quad"], b["quad"])
        assert a["estimate"] == b["estimate"]


def test_server_fp64_matches_oracle_and_mix(ctx):
    """An FP64 server (FP64 vectors; slot kernels with two columns per lane):
    explicit queries of several widths against the oracle at the FP64 bar,
    and adaptive queries give the same bits alone and together."""
    _say("case server: FP64 mode")
    graphs = [_reg(ctx, *synth.erdos_renyi(2500, 7.0, 61), fp64=True),
              _reg(ctx, *synth.watts_strogatz(3000, 8, 0.1, 62), fp64=True)]
    mode = vne.MODE_DESING | vne.MODE_F64
    with vne.Server(ctx, mode, arena_bytes=1 << 30) as srv:
        work = [(0, 8, 20, 1), (1, 16, 25, 2), (0, 40, 30, 3), (1, 130, 18, 4)]
        ts = [srv.submit(graphs[g][0], m=m, k=k, seed=sd) for g, m, k, sd in work]
        got = [srv.poll(t, want_quad=True) for t in ts]
        for (g, m, k, sd), r in zip(work, got):
            ref = graphs[g][1]
            assert r["status"] == 0, r["message"]
            B = oracle.rademacher_block(sd, ref.node_ids, np.arange(m))
            want = oracle.quadforms(ref.scipy(), B, k, oracle.breakdown_tau(True))
            sens = _order_sensitivity(ref.scipy(), B, k, True)
            _assert_within(_rel(r["quad"], want["psi"]), _bar(True, sens), "n=%d m=%d k=%d" % (ref.n, m, k))
        alone = [srv.poll(srv.submit(graphs[i % 2][0], rel_eps=1e-3, seed=70 + i), want_quad=True)
                 for i in range(4)]
        ts = [srv.submit(graphs[i % 2][0], rel_eps=1e-3, seed=70 + i) for i in range(4)]
        mixed = [srv.poll(t, want_quad=True) for t in ts]
        assert srv.stats()["group_tasks"] == 0       # group slots are FP32 only
    for a, b in zip(alone, mixed):
        assert a["status"] == 0 and b["status"] == 0
        assert np.array_equal(a["quad"], b["quad"]) and a["estimate"] == b["estimate"]


def test_server_admission_under_small_arena(ctx, pool):
    _say("case server: admission with an arena for about two tasks")
    gid, ref = pool[5]                       # n = 20000
    work = [(gid, 128, 20, s) for s in range(6)] + [(pool[0][0], 64, 25, 9)]
    with vne.Server(ctx, MODE, arena_bytes=1 << 30) as big:
        want = [_run_one(big, *w) for w in work]
    small_bytes = 2 * (4 * ref.n * 128 * 4) + (8 << 20)
    with vne.Server(ctx, MODE, arena_bytes=small_bytes, max_cols=1024) as srv:
        ts = [srv.submit(g, m=m, k=k, seed=s) for g, m, k, s in work]
        got = [srv.poll(t, want_quad=True) for t in ts]
        info = srv.stats()
        # a query whose single task cannot fit the arena fails alone
        too_big = srv.poll(srv.submit(gid, m=2048, k=10, seed=1))
    assert info["arena_peak"] <= small_bytes
    for a, b in zip(want, got):
        assert b["status"] == 0
        assert np.array_equal(a["quad"], b["quad"])
    assert too_big["status"] == -2
    assert "arena" in too_big["message"]


def test_server_error_rule_accuracy(ctx):
    """rel_eps = 1e-3 queries on graphs small enough for the exact entropy."""
    _say("case server: error rule at rel_eps = 1e-3")
    cases = [synth.erdos_renyi(1500, 8.0, 51), synth.barabasi_albert(1200, 3, 52),
             synth.watts_strogatz(2000, 8, 0.1, 53), synth.grid2d_graph(30, 40)]
    regs = [_reg(ctx, *c) for c in cases]
    with vne.Server(ctx, MODE, arena_bytes=1 << 30) as srv:
        ts = [srv.submit(gid, rel_eps=1e-3, seed=900 + i) for i, (gid, _) in enumerate(regs)]
        res = [srv.poll(t, want_quad=True) for t in ts]
    errs = []
    for (gid, ref), r in zip(regs, res):
        rho = oracle.dense_matrix(ref)
        S = oracle.exact_entropy(rho)
        lam_ub = np.abs(rho).sum(1).max()
        k_want = vne.plan_steps(float(ref.n), lam_ub, -np.log((rho * rho).sum()), 1e-3, 0.5, 100)
        err = abs(r["estimate"] - S) / S
        _say("  n=%d N=%d k=%d (a-priori %d) rel err %.2e (std err %.2e)"
             % (ref.n, r["probes"], r["steps"], k_want, err, r["std_error"] / S))
        # the a-priori count is the cap; the a-posteriori bound stops earlier
        assert r["status"] == 0 and 3 <= r["steps"] <= k_want and r["probes"] >= 16
        assert len(r["quad"]) == r["probes"]
        errs.append(err)
    # the rule targets 1e-3 with probability 1 - 1e-2 per query
    assert sum(e <= 1e-3 for e in errs) >= 3 and max(errs) <= 2e-3


def test_server_estimate_stop_rule(ctx, pool):
    """A server whose tasks stop on the eq. (4.10) estimate (the geometric
    mean of each bracket) instead of its upper bound: no more steps than the
    bound rule, estimates on graphs with exact entropy still within the
    target, and a query gives the same bits alone and among others."""
    _say("case server: stop on the eq. (4.10) estimate")
    cases = [synth.erdos_renyi(1500, 8.0, 51), synth.barabasi_albert(1200, 3, 52),
             synth.watts_strogatz(2000, 8, 0.1, 53), synth.grid2d_graph(30, 40)]
    regs = [_reg(ctx, *c) for c in cases]
    got = {}
    for rule in (vne.STOP_BOUND, vne.STOP_ESTIMATE):
        with vne.Server(ctx, MODE, arena_bytes=1 << 30, stop=rule) as srv:
            got[rule] = [srv.poll(srv.submit(gid, rel_eps=1e-3, seed=900 + i), want_quad=True)
                         for i, (gid, _) in enumerate(regs)]
    errs = []
    for (gid, ref), rb, re_ in zip(regs, got[vne.STOP_BOUND], got[vne.STOP_ESTIMATE]):
        S = oracle.exact_entropy(oracle.dense_matrix(ref))
        err = abs(re_["estimate"] - S) / S
        _say("  n=%d steps %d (bound rule %d), probes %d (%d), rel err %.2e (bound rule %.2e)"
             % (ref.n, re_["steps"], rb["steps"], re_["probes"], rb["probes"], err, abs(rb["estimate"] - S) / S))
        assert re_["status"] == 0 and 3 <= re_["steps"] <= rb["steps"]
        errs.append(err)
    assert sum(e <= 1e-3 for e in errs) >= 3 and max(errs) <= 2e-3
    # same bits alone and in a mix under the estimate rule
    gid, _ = pool[1]
    with vne.Server(ctx, MODE, arena_bytes=1 << 30, stop=vne.STOP_ESTIMATE) as srv:
        alone = srv.poll(srv.submit(gid, rel_eps=1e-3, seed=5), want_quad=True)
        ts = [srv.submit(pool[i % len(pool)][0], rel_eps=1e-3, seed=100 + i) for i in range(6)]
        mine = srv.submit(gid, rel_eps=1e-3, seed=5)
        mixed = srv.poll(mine, want_quad=True)
        assert all(srv.poll(t)["status"] == 0 for t in ts)
    assert np.array_equal(alone["quad"], mixed["quad"]) and alone["estimate"] == mixed["estimate"]


@pytest.mark.parametrize("fp64", [False, True])
@pytest.mark.parametrize("rule", ["bound", "estimate"])
def test_server_stop_step_matches_oracle(ctx, rule, fp64):
    """The a-posteriori check of a served task against the oracle: with
    max_probes = pilot_probes = 16 a rel_eps query is its 16-column pilot
    alone, so its step count is the task's stop step.  The oracle runs
    Lanczos on the same (desingularized) probes and takes the first check
    step (3, 5, ... below the a-priori cap) where every column's bracket on
    [1e-12 lambda_ub, lambda_ub] (256 points; Theorem 4.8) has its upper
    bound, or its eq. (4.10) estimate, within tol = (rel_eps / 2) S_lower;
    the steps must be equal and the 16 forms must match the oracle's at that
    step, at the bar of the server's mode (Remarks 5.1, 5.2; Theorem 4.8)."""
    from oracle import probing as oprobing
    _say("case server: stop step of the %s rule against the oracle (%s)" % (rule, "FP64" if fp64 else "FP32"))
    eps = 1e-3
    cases = [synth.erdos_renyi(1500, 8.0, 51), synth.grid2d_graph(30, 40), synth.barabasi_albert(1200, 3, 52)]
    regs = [_reg(ctx, *c, fp64=fp64) for c in cases]
    stop = {"bound": vne.STOP_BOUND, "estimate": vne.STOP_ESTIMATE}[rule]
    mode = MODE | (vne.MODE_F64 if fp64 else 0)
    with vne.Server(ctx, mode, arena_bytes=1 << 30, max_probes=16, pilot_probes=16, stop=stop) as srv:
        res = [srv.poll(srv.submit(gid, rel_eps=eps, seed=700 + i), want_quad=True) for i, (gid, _) in enumerate(regs)]
    for i, ((gid, ref), r) in enumerate(zip(regs, res)):
        assert r["status"] == 0 and r["probes"] == 16, r["message"]
        A = ref.scipy()
        rho = oracle.dense_matrix(ref)
        lam_ub = float(np.abs(rho).sum(1).max())
        s_lower = float(-np.log((rho * rho).sum()))
        K = vne.plan_steps(float(ref.n), lam_ub, s_lower, eps, 0.5, 100)
        tol = 0.5 * eps * s_lower
        B = oracle.rademacher_block(700 + i, ref.node_ids, np.arange(16))
        _, _, _, lz = oprobing.adaptive_quadforms(A, B, K, oracle.breakdown_tau(fp64), np.full(16, tol),
                                                  1e-12 * lam_ub, lam_ub, grid=256, desing=True, rule=rule)
        want_step, margin = K, None
        for j in range(3, K, 2):
            q = np.zeros(16)
            for c in range(16):
                mm = min(int(lz["k_eff"][c]), j)
                if mm > 0 and lz["beta"][c, mm - 1] != 0.0:
                    lo, hi, _ = oracle.bounds.posterior_bracket(lz["alpha"][c], lz["beta"][c], mm, lz["norm2"][c],
                                                                1e-12 * lam_ub, lam_ub, grid=256)
                    q[c] = hi if rule == "bound" else np.sqrt(lo * hi)
            if np.all(q <= tol):
                want_step, margin = j, float(q.max() / tol)
                break
        want = oprobing.gauss_quadrature(lz["alpha"], lz["beta"], np.minimum(lz["k_eff"], want_step), lz["norm2"])
        rel = _rel(r["quad"], want)
        _say("  n=%d cap %d: stop step %d (oracle %d, largest q/tol there %s), forms max rel %.2e"
             % (ref.n, K, r["steps"], want_step, "%.3f" % margin if margin is not None else "-", rel.max()))
        assert r["steps"] == want_step
        sens = _order_sensitivity(A, B, want_step, fp64)
        _assert_within(rel, _bar(fp64, sens), "n=%d %s rule" % (ref.n, rule))


def test_server_side_streams_same_bits(ctx, pool, monkeypatch):
    """The width classes of a tick on one stream or spread over side
    streams: every query of a mix of widths (16-column pilots in pairs,
    lone tasks of 16 to 128 columns) gives the same bits."""
    _say("case server: one stream against side streams")
    work = [(pool[i % len(pool)][0], m, k, 300 + i) for i, (m, k) in
            enumerate([(16, 20), (16, 20), (40, 25), (130, 15), (16, 30), (64, 12), (200, 18), (16, 20)])]
    adaptive = [(pool[i % len(pool)][0], 500 + i) for i in range(6)]
    got = {}
    for streams in ("1", "3"):
        monkeypatch.setenv("VNE_SERVE_STREAMS", streams)
        with vne.Server(ctx, MODE, arena_bytes=1 << 30) as srv:
            ts = [srv.submit(g, m=m, k=k, seed=sd) for g, m, k, sd in work]
            ts += [srv.submit(g, rel_eps=1e-3, seed=sd) for g, sd in adaptive]
            got[streams] = [srv.poll(t, want_quad=True) for t in ts]
    for a, b in zip(got["1"], got["3"]):
        assert a["status"] == 0 and b["status"] == 0
        assert a["probes"] == b["probes"] and a["steps"] == b["steps"]
        assert np.array_equal(a["quad"], b["quad"]) and a["estimate"] == b["estimate"]


def test_server_errors_and_busy_release(ctx, pool):
    _say("case server: error paths")
    gid, ref = pool[5]
    with vne.Server(ctx, MODE, arena_bytes=1 << 30, max_probes=512) as srv:
        with pytest.raises(vne.VneError) as ei:
            srv.submit(10 ** 6, m=4, k=5)
        assert ei.value.status == -1
        with pytest.raises(vne.VneError):
            srv.submit(gid, m=513, k=5)
        with pytest.raises(vne.VneError):
            srv.submit(gid, m=4, k=0)
        with pytest.raises(vne.VneError):
            srv.poll(12345)
        t = srv.submit(gid, m=512, k=100, seed=3)
        with pytest.raises(vne.VneError) as ei:
            ctx.release(gid)
        assert ei.value.status == -5
        assert srv.poll(t)["status"] == 0
    for bad in (3, 8, -1):
        with pytest.raises(vne.VneError) as ei:
            vne.Server(ctx, MODE, arena_bytes=1 << 26, max_group=bad)
        assert ei.value.status == -1
    for bad in (2, -1):
        with pytest.raises(vne.VneError) as ei:
            vne.Server(ctx, MODE, arena_bytes=1 << 26, stop=bad)
        assert ei.value.status == -1
    # a graph without zero row sums cannot run desingularized
    rp = np.arange(11, dtype=np.int32)
    g2 = ctx.register(rp, np.arange(10, dtype=np.int32), np.ones(10, np.float32), 0.1)
    with vne.Server(ctx, MODE, arena_bytes=1 << 26) as srv:
        with pytest.raises(vne.VneError):
            srv.submit(g2, m=4, k=3)
