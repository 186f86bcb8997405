"""Parity at the benchmark sizes, in the benchmark's launch configuration,
on sampled outputs the oracle computes one by one.

* large: BA n = 2e5 (3 edges per node), FP32, k = 60.  The bench's own
  Hutch++ estimate (128 sketch + 128 Hutchinson columns) against the
  oracle's Hutch++ on the same probes, read from tests/golden/
  hutchpp_large.json (written by tests/golden/make_hutchpp_large.py, which
  calls only the oracle): the estimate, the sum of the Q forms and every
  G~ form.  The 256-wide Rademacher block through the same step kernels:
  columns 0, 77, 200, 255 against the oracle, and the Hutch++ estimate
  within five standard errors of that Hutchinson estimate.
* the same graph under adaptive Hutch++ (relative target 1e-2, delta 1e-2)
  against the oracle's run of the same rule, read from tests/golden/
  hutchpp_adaptive_large.json (written by make_hutchpp_adaptive_large.py).
* probing: WS n = 1e6 (k = 10, p = 0.1), distance-2 colouring, k = 80:
  colours 0, 11 and the last one against the oracle; the colouring itself is
  compared bit for bit with the oracle elsewhere (CPU, slow).
* batch: the 512-graph batch (64 probes, k = 50): four sampled graphs
  (smallest, largest, one ER, one BA), four columns each.
* the probing configuration without rewiring (ring lattice): the whole
  estimate against the exact entropy, within Corollary 3.2's bound.
Bars: 1e-5 relative per quadratic form, per column widened to 5x that
column's own rounding-order spread (the oracle in four row orders) where
that is larger.
"""
import numpy as np
import pytest

import oracle
from synth import workloads
import paper_2212_09642_amd as vne
from gpu_common import TOL, ctx, _say, _rel, _orders, _spread, _bar, _assert_within  # noqa: F401

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _sampled_check(A, keys, B, out_quad, cols, k, desing=True):
    import scipy.sparse as sp
    A = sp.csr_matrix(A)
    B = np.asarray(B)
    tau = oracle.breakdown_tau(False)
    want = oracle.quadforms(A, B, k, tau, desing)["psi"]
    runs = [want] + [oracle.quadforms(A[P][:, P], B[P], k, tau, desing)["psi"] for P in _orders(A.shape[0])]
    _assert_within(_rel(out_quad[cols], want), _bar(False, _spread(runs, want)), "sampled columns %s" % list(cols))


def test_large_configuration_sampled(ctx):
    w = workloads.large()
    _say("case full size: BA n=2e5, m=256, k=60")
    g = vne.laplacian_from_edges(w["n_nodes"], w["edges"], np.float32)
    gid = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
    m, k = w["n_sketch"] + w["n_hutch"], w["k"]
    out = ctx.estimate(gid, vne.PROBE_RADEMACHER, m, k, vne.MODE_DESING, seed=w["probe_seed"], want_coeffs=False)
    cols = np.array([0, 77, 200, 255])
    import scipy.sparse as sp
    A = sp.csr_matrix((np.asarray(g["values"], np.float64) * g["scale"], g["col_idx"], g["row_ptr"]),
                      shape=(g["n"], g["n"]))
    B = oracle.rademacher_block(w["probe_seed"], g["node_ids"], cols)
    _sampled_check(A, g["node_ids"], B, out["quad"], cols, k)
    hpp = ctx.estimate(gid, vne.PROBE_HUTCHPP, m, k, vne.MODE_DESING, seed=w["probe_seed"],
                       n_sketch=w["n_sketch"], want_coeffs=False)
    se = out["quad"].std(ddof=1) / np.sqrt(m)
    _say("   Hutch++ %.8f, Hutchinson %.8f +- %.1e" % (hpp["estimate"], out["estimate"], se))
    assert abs(hpp["estimate"] - out["estimate"]) < 5 * se


def test_large_hutchpp_against_oracle(ctx):
    """The bench's configuration itself: Hutch++ on BA n = 2e5 with 128 + 128
    Rademacher columns and 60 steps, FP32 vectors (eq. (3.9) with f(A) Omega
    by eq. (4.3)), against the oracle's Hutch++ on the same probes."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hutchpp_large.json")
    with open(path) as fh:
        gold = json.load(fh)
    w = workloads.large()
    _say("case full size: Hutch++ BA n=2e5, 128 + 128, k=60 against the oracle")
    g = vne.laplacian_from_edges(w["n_nodes"], w["edges"], np.float32)
    assert (g["n"], len(g["col_idx"])) == (gold["n"], gold["nnz"])
    nr, m = w["n_sketch"], w["n_sketch"] + w["n_hutch"]
    assert (nr, m, w["k"], w["probe_seed"]) == (gold["n_sketch"], gold["n_sketch"] + gold["n_hutch"], gold["k"],
                                                gold["probe_seed"])
    gid = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
    out = ctx.estimate(gid, vne.PROBE_HUTCHPP, m, w["k"], vne.MODE_DESING, seed=w["probe_seed"], n_sketch=nr,
                       want_coeffs=False)
    psi = np.array(gold["psi"])
    sens_psi = np.array(gold["psi_spread"]) / np.abs(psi)
    est = gold["estimate"]
    _say("   estimate %.12f, oracle %.12f (spread %.1e), oracle |Q^T Q - I| %.1e"
         % (out["estimate"], est, gold["estimate_spread"], gold["q_orthogonality"]))
    _assert_within(abs(out["estimate"] - est) / abs(est), _bar(False, gold["estimate_spread"] / abs(est)),
                   "estimate")
    sq = gold["sum_q"]
    _assert_within(abs(out["quad"][:nr].sum() - sq) / abs(sq), _bar(False, gold["sum_q_spread"] / abs(sq)),
                   "sum over Q")
    _assert_within(_rel(out["quad"][nr:], psi[nr:]), _bar(False, sens_psi[nr:]), "G~ forms")
    rq = _rel(out["quad"][:nr], psi[:nr])
    _say("   Q forms one by one (FP32 sketch; not asserted): max rel err %.3e" % rq.max())
    assert np.array_equal(out["k_eff"], np.array(gold["k_eff"]))
    ctx.release(gid)


def test_large_adaptive_hutchpp_against_oracle(ctx):
    """Adaptive Hutch++ on the bench's graph (BA n = 2e5, relative target
    1e-2, delta = 1e-2, k = 60, FP32 vectors) against the oracle's run of the
    same rule, read from tests/golden/hutchpp_adaptive_large.json (written by
    tests/golden/make_hutchpp_adaptive_large.py, which calls only the
    oracle): each round's width and count exactly, its estimate, and the
    sample standard deviation of its pilot forms within ||dq|| / sqrt(n - 1)
    (dq: the per-form bars); the final estimate, the sum over Q and every
    deflated form within the usual bars."""
    import json
    import math
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hutchpp_adaptive_large.json")
    with open(path) as fh:
        gold = json.load(fh)
    w = workloads.large()
    _say("case full size: adaptive Hutch++ BA n=2e5, rel_eps %g, k=60 against the oracle" % gold["rel_eps"])
    g = vne.laplacian_from_edges(w["n_nodes"], w["edges"], np.float32)
    assert (g["n"], len(g["col_idx"]), w["k"], w["probe_seed"]) == (gold["n"], gold["nnz"], gold["k"],
                                                                     gold["probe_seed"])
    gid = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
    out = ctx.hutchpp_adaptive(gid, w["k"], rel_eps=gold["rel_eps"], delta=gold["delta"], mode=vne.MODE_DESING,
                               seed=w["probe_seed"], quad_cap=4096)
    assert [(r["nr"], r["nh"]) for r in out["rounds"]] == [(r["nr"], r["nh"]) for r in gold["rounds"]]
    for gr, o in zip(out["rounds"], gold["rounds"]):
        est = o["estimate"]
        _assert_within(abs(gr["estimate"] - est) / abs(est), _bar(False, o["estimate_spread"] / abs(est)),
                       "round %d estimate" % o["nr"])
        q = np.array(o["pilot"])
        dq = np.sqrt(np.sum((_bar(False, np.array(o["pilot_spread"]) / np.abs(q)) * np.abs(q)) ** 2))
        b_sd = dq / math.sqrt(q.size - 1)
        _say("   round N_r=%d: sd %.6e, oracle %.6e (bar %.1e)" % (o["nr"], gr["sd"], o["sd"], b_sd))
        assert abs(gr["sd"] - o["sd"]) <= b_sd
    assert (out["n_sketch"], out["n_hutch"], out["krylov_runs"]) == (gold["n_sketch"], gold["n_hutch"],
                                                                     gold["krylov_runs"])
    est, nr = gold["estimate"], gold["n_sketch"]
    _say("   estimate %.12f, oracle %.12f (spread %.1e)" % (out["estimate"], est, gold["estimate_spread"]))
    _assert_within(abs(out["estimate"] - est) / abs(est), _bar(False, gold["estimate_spread"] / abs(est)),
                   "estimate")
    psi, spread = np.array(gold["psi"]), np.array(gold["psi_spread"])
    sq, sq_spread = gold["sum_q"], gold["sum_q_spread"]
    _assert_within(abs(out["quad"][:nr].sum() - sq) / abs(sq), _bar(False, sq_spread / abs(sq)), "sum over Q")
    _assert_within(_rel(out["quad"][nr:], psi[nr:]), _bar(False, spread[nr:] / np.abs(psi[nr:])), "G~ forms")
    ctx.release(gid)


def test_probing_configuration_sampled(ctx):
    w = workloads.probing()
    _say("case full size: WS n=1e6, distance-2 colouring, k=80")
    g = vne.laplacian_from_edges(w["n_nodes"], w["edges"], np.float32)
    gid = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
    col, s = vne.color_greedy(g["row_ptr"], g["col_idx"], g["values"], w["d"])
    out = ctx.estimate(gid, vne.PROBE_COLORING, s, w["k"], vne.MODE_DESING, colors=col, want_coeffs=False)
    cols = np.array([0, 11, s - 1])
    import scipy.sparse as sp
    A = sp.csr_matrix((np.asarray(g["values"], np.float64) * g["scale"], g["col_idx"], g["row_ptr"]),
                      shape=(g["n"], g["n"]))
    B = oracle.indicator_block(col, s)[:, cols]
    _sampled_check(A, g["node_ids"], B, out["quad"], cols, w["k"])
    assert abs(out["estimate"] - out["quad"].sum()) <= 1e-13 * abs(out["estimate"])


def test_batch_configuration_sampled(ctx):
    _say("case full size: 512-graph batch, 64 probes, k=50")
    specs = workloads.batch_specs()
    graphs = [vne.laplacian_from_edges(*workloads.batch_graph(sp_), np.float32) for sp_ in specs]
    gids = [ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
            for g in graphs]
    queries = [dict(gid=gid, kind=vne.PROBE_RADEMACHER, m=64, k=50, seed=workloads.PROBE_SEED + q)
               for q, gid in enumerate(gids)]
    outs = ctx.estimate_batch(queries, vne.MODE_DESING)
    sizes = np.array([g["n"] for g in graphs])
    picks = [int(sizes.argmin()), int(sizes.argmax()), 2, 3]      # even specs are ER, odd are BA
    import scipy.sparse as sp
    for q in picks:
        g = graphs[q]
        _say("  graph %d (%s) n=%d" % (q, specs[q][0], g["n"]))
        A = sp.csr_matrix((np.asarray(g["values"], np.float64) * g["scale"], g["col_idx"], g["row_ptr"]),
                          shape=(g["n"], g["n"]))
        cols = np.array([0, 21, 42, 63])
        B = oracle.rademacher_block(workloads.PROBE_SEED + q, g["node_ids"], cols)
        _sampled_check(A, g["node_ids"], B, outs[q]["quad"], cols, 50)


def test_probing_ring_lattice_exact_entropy(ctx):
    """The probing configuration without rewiring (ring lattice n = 1e6,
    k = 10): its Laplacian is circulant, so S(rho) has a closed form from the
    eigenvalues 10 - 2 sum_{r=1..5} cos(2 pi j r / n).  The distance-2 probing
    estimate must be within Corollary 3.2's bound n b / (2 (d^2 - 1)) (a = 0,
    b = lambda_max) of it."""
    _say("case full size: ring lattice n=1e6, probing d=2, k=80, exact S")
    import synth
    n, kk, d = 1_000_000, 10, 2
    nn, e = synth.ring_lattice(n, kk)
    g = vne.laplacian_from_edges(nn, e, np.float32)
    gid = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
    col, s = vne.color_greedy(g["row_ptr"], g["col_idx"], g["values"], d)
    out = ctx.estimate(gid, vne.PROBE_COLORING, s, 80, vne.MODE_DESING, colors=col, want_coeffs=False)
    j = np.arange(n, dtype=np.float64)
    lam = np.full(n, float(kk))
    for r in range(1, kk // 2 + 1):
        lam -= 2.0 * np.cos(2.0 * np.pi * j * r / n)
    rho = lam / lam.sum()
    rho_pos = rho[rho > 0]
    S = float(-np.sum(rho_pos * np.log(rho_pos)))
    bound = n * rho.max() / (2 * (d * d - 1))
    err = abs(out["estimate"] - S)
    _say("   colours %d, S = %.10f, estimate %.10f, |err| = %.3e (rel %.2e), Corollary 3.2 bound %.3e"
         % (s, S, out["estimate"], err, err / S, bound))
    assert err <= bound


def test_algorithm_2_ring_lattice_full_size(ctx):
    """Algorithm 2 at eps = 1e-3 on the ring lattice n = 1e6, k = 10 (the
    probing configuration without rewiring) against its closed-form entropy;
    every colour meets its eq. (5.3) tolerance."""
    _say("case full size: Algorithm 2, ring lattice n=1e6, eps=1e-3")
    import bench
    import synth
    n, kk, eps = 1_000_000, 10, 1e-3
    nn, e = synth.ring_lattice(n, kk)
    g = vne.laplacian_from_edges(nn, e, np.float32)
    gid = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
    out = ctx.probing(gid, eps, d_max=16, k_max=128)
    S = bench.ring_lattice_entropy(n, kk)
    err = abs(out["estimate"] - S) / S
    _say("   d=%d colours %d passes %d, estimate %.10f, S %.10f, rel err %.2e, colouring %.0f ms, Lanczos %.0f ms"
         % (out["d"], out["n_colors"], out["passes"], out["estimate"], S, err, out["color_ms"], out["lanczos_ms"]))
    assert out["unconverged"] == 0
    assert err <= eps
    # the probing sums of a Laplacian are lower bounds (Proposition 3.6), up to the Krylov part
    assert max(out["t_pre"]) <= S + out["eps_hat"]
    ctx.release(gid)
