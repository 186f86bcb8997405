"""GPU parity of the probing method with an accuracy target (Algorithm 2)
and of the per-vector stopping rule under it (Theorem 4.8 as a stopping
criterion, tolerances of eq. (5.3)).

* stop decisions: for every vector, the Theorem 4.8 upper bound evaluated by
  the oracle on the GPU's own Lanczos coefficients exceeds the tolerance at
  every earlier check step and meets it at the GPU's stop step (the decision
  itself, taken on the same coefficients); the oracle's decisions on its own
  FP64 coefficients agree except where the tolerance lies within 2% (FP64
  vectors) or 25% (FP32 vectors: the bound is built from beta_m and the last
  eigenvector row, which carry the vectors' rounding long before psi does) of
  its bound, or within 5x the bound's own rounding-order spread (the same
  problem in four row orders);
* psi at the GPU's stop steps against the oracle's Lanczos + Gauss quadrature
  at the same steps (1e-5 / 1e-12 relative, per colour widened to 5x that
  colour's own rounding-order spread);
* Algorithm 2 against the oracle's: the same distance (or a borderline
  one), the same colouring, the same per-colour stop steps of every pass,
  then T_1..T_3, the per-colour psi of the final pass and the estimate at
  1e-5; only a pass in which a stop decision flips (the tolerance within
  the bound's rounding) keeps a 1e-4 bar for its sum.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import probing as oprobing
import synth
import paper_2212_09642_amd as vne
from gpu_common import TOL, C_SENS, ctx, _say, _rel, _setup, _orders, _spread, _bar, _assert_within  # noqa: F401

pytestmark = pytest.mark.gpu

GRID = 256


def _gq_at(res, steps):
    k_use = np.minimum(res["k_eff"], steps)
    return oracle.gauss_quadrature(res["alpha"], res["beta"], k_use, res["norm2"])


def _hi(alpha, beta, k_eff, norm2, s, lam_lo, lam_hi, rule="bound"):
    """The stopping quantity after s steps: the upper bound of Theorem 4.8
    (eq. (4.9)) or the geometric mean of the bracket (eq. (4.10))."""
    mm = min(int(k_eff), s)
    if mm <= 0 or beta[mm - 1] == 0.0:
        return 0.0
    lo, hi, _ = oracle.bounds.posterior_bracket(alpha, beta, mm, norm2, lam_lo, lam_hi, grid=GRID)
    return hi if rule == "bound" else np.sqrt(lo * hi)


RULES = {vne.STOP_BOUND: "bound", vne.STOP_ESTIMATE: "estimate"}


def _check_adaptive(ctx, gid, ref, B, tol, k_max, fp64, kind, colors=None, seed=0, dense=None,
                    stop_rule=vne.STOP_BOUND):
    A = ref.scipy()
    lam_hi = float(np.abs(A).sum(axis=1).max())
    lam_lo = 1e-12 * lam_hi
    mode = vne.MODE_DESING | (vne.MODE_F64 if fp64 else 0)
    m = B.shape[1]
    rule = RULES[stop_rule]
    out = ctx.estimate_adaptive(gid, kind, m, k_max, mode, tol, lam_lo, lam_hi, n_grid=GRID, seed=seed,
                                colors=colors, dense=dense, want_coeffs=True, stop=stop_rule)
    stop = out["steps"]                          # 0: never met its tolerance
    steps = np.where(stop > 0, stop, k_max)
    # 1. the decisions, on the GPU's own coefficients (up to each column's stop
    # step: a stopped column is not computed further)
    for c in range(m):
        s_c = int(steps[c])
        for s in range(3, s_c if stop[c] > 0 else k_max + 1, 2):
            assert _hi(out["alpha"][c], out["beta"][c], out["k_eff"][c], out["norm2"][c], s, lam_lo,
                       lam_hi, rule) > tol[c] * (1 - 1e-9), (c, s, s_c)
        if stop[c] > 0:
            assert s_c >= 3 and s_c % 2 == 1
            h = _hi(out["alpha"][c], out["beta"][c], out["k_eff"][c], out["norm2"][c], s_c, lam_lo, lam_hi, rule)
            assert h <= tol[c] * (1 + 1e-9), (c, s_c, h, tol[c])
    # 2. the oracle's decisions on its FP64 coefficients
    psi_o, steps_o, conv_o, res = oprobing.adaptive_quadforms(A, B, k_max, oracle.breakdown_tau(fp64), tol,
                                                              lam_lo, lam_hi, grid=GRID, rule=rule)
    Asp = sp.csr_matrix(A)
    others = [oracle.lanczos(Asp[P][:, P], oracle.desingularize(np.asarray(B)[P]), k_max,
                             oracle.breakdown_tau(fp64)) for P in _orders(A.shape[0])]
    differ = np.nonzero(((stop > 0) != conv_o) | ((stop > 0) & (steps != steps_o)))[0]
    for c in differ:
        # the decision may differ only where the tolerance lies within the
        # bound's own rounding-order spread (oracle, four row orders)
        s0 = int(min(steps[c], steps_o[c]))
        hs = [_hi(r["alpha"][c], r["beta"][c], r["k_eff"][c], r["norm2"][c], s0, lam_lo, lam_hi, rule)
              for r in [res] + others]
        h = hs[0]
        slack = 0.02 if fp64 else 0.25
        assert abs(h - tol[c]) <= max(slack * tol[c], C_SENS * (max(hs) - min(hs))), (c, steps[c], steps_o[c],
                                                                                     hs, tol[c])
    assert differ.size <= max(1, m // 4)
    # 3. psi at the GPU's steps, per column within TOL or C_SENS x its spread
    want = _gq_at(res, steps)
    sens = _spread([want] + [_gq_at(r, steps) for r in others], want)
    _say("   m=%d steps %d..%d (oracle differs on %d)" % (m, steps.min(), steps.max(), differ.size))
    _assert_within(_rel(out["quad"], want), _bar(fp64, sens), "psi at the GPU's steps")
    assert abs(out["estimate"] - (out["quad"].sum() if kind == vne.PROBE_COLORING else out["quad"].mean())) \
        <= 1e-13 * abs(out["estimate"])
    return out


CASES = [("er", lambda: synth.erdos_renyi(3000, 8.0, 61)), ("ba", lambda: synth.barabasi_albert(2500, 3, 62)),
         ("ws", lambda: synth.watts_strogatz(4000, 10, 0.1, 63)), ("grid", lambda: synth.grid2d_graph(50, 60))]


@pytest.mark.parametrize("name,mk", CASES)
@pytest.mark.parametrize("fp64", [False, True])
def test_adaptive_colour_indicators(ctx, name, mk, fp64):
    _say("case adaptive stopping, colour indicators d=2, %s fp64=%s" % (name, fp64))
    gid, ref = _setup(ctx, *mk(), fp64=fp64)
    col, s = oracle.greedy_distance_coloring(ref.row_ptr, ref.col_idx, ref.n, 2)
    S0 = -np.log((ref.scipy().data ** 2).sum())
    sizes = np.bincount(col, minlength=s)
    tol = 0.5 * 1e-4 * S0 * sizes / ref.n
    out = _check_adaptive(ctx, gid, ref, oracle.indicator_block(col, s), tol, 60, fp64, vne.PROBE_COLORING,
                          colors=col.astype(np.int32))
    ctx.release(gid)
    assert out["steps"].min() >= 3              # every colour met its tolerance


@pytest.mark.parametrize("name,mk", CASES[:2])
@pytest.mark.parametrize("fp64", [False, True])
def test_adaptive_estimate_rule(ctx, name, mk, fp64):
    """The eq. (4.10) stopping rule: the decisions on the device's own
    coefficients, the oracle's decisions and psi at the device's steps as
    for the bound; no column stops later than under the bound rule."""
    _say("case adaptive stopping on the eq. (4.10) estimate, %s fp64=%s" % (name, fp64))
    gid, ref = _setup(ctx, *mk(), fp64=fp64)
    col, s = oracle.greedy_distance_coloring(ref.row_ptr, ref.col_idx, ref.n, 2)
    S0 = -np.log((ref.scipy().data ** 2).sum())
    tol = 0.5 * 1e-4 * S0 * np.bincount(col, minlength=s) / ref.n
    B = oracle.indicator_block(col, s)
    est = _check_adaptive(ctx, gid, ref, B, tol, 60, fp64, vne.PROBE_COLORING, colors=col.astype(np.int32),
                          stop_rule=vne.STOP_ESTIMATE)
    bnd = _check_adaptive(ctx, gid, ref, B, tol, 60, fp64, vne.PROBE_COLORING, colors=col.astype(np.int32))
    assert np.all(est["steps"] <= bnd["steps"]) and est["steps"].min() >= 3
    _say("   vector steps: estimate %d, bound %d" % (est["steps"].sum(), bnd["steps"].sum()))
    ctx.release(gid)


def test_stopped_columns_are_not_computed_further(ctx, monkeypatch):
    """Columns that met their tolerance are skipped (their tiles and normalize
    groups): psi, stop steps and every coefficient up to each column's stop
    step are bitwise those of a run that keeps computing them (VNE_FREEZE=0)."""
    _say("case stopped columns frozen vs computed")
    gid, ref = _setup(ctx, *synth.watts_strogatz(6000, 8, 0.1, 65), fp64=False)
    col, s = oracle.greedy_distance_coloring(ref.row_ptr, ref.col_idx, ref.n, 3)
    S0 = -np.log((ref.scipy().data ** 2).sum())
    tol = 0.5 * 1e-5 * S0 * np.bincount(col, minlength=s) / ref.n
    tol[::5] *= 1e3                                     # some colours stop long before the others
    A = ref.scipy()
    lam_hi = float(np.abs(A).sum(axis=1).max())
    args = (gid, vne.PROBE_COLORING, s, 80, vne.MODE_DESING, tol, 1e-12 * lam_hi, lam_hi)
    frozen = ctx.estimate_adaptive(*args, n_grid=GRID, colors=col.astype(np.int32), want_coeffs=True)
    monkeypatch.setenv("VNE_FREEZE", "0")
    full = ctx.estimate_adaptive(*args, n_grid=GRID, colors=col.astype(np.int32), want_coeffs=True)
    assert np.array_equal(frozen["steps"], full["steps"]) and np.array_equal(frozen["quad"], full["quad"])
    assert frozen["estimate"] == full["estimate"]
    steps = np.where(frozen["steps"] > 0, frozen["steps"], 80)
    for c in range(s):
        assert np.array_equal(frozen["alpha"][c, :steps[c]], full["alpha"][c, :steps[c]])
        assert np.array_equal(frozen["beta"][c, :steps[c]], full["beta"][c, :steps[c]])
    _say("   %d colours, stop steps %d..%d" % (s, steps.min(), steps.max()))
    ctx.release(gid)


def test_adaptive_rademacher_and_unreachable_tolerances(ctx):
    _say("case adaptive stopping, Rademacher, some tolerances out of reach")
    gid, ref = _setup(ctx, *synth.barabasi_albert(3000, 3, 64), fp64=False)
    m, k_max = 40, 24
    B = oracle.rademacher_block(11, ref.node_ids, np.arange(m))
    tol = np.full(m, 1e-3)                       # psi ~ 10: 1e-4 relative
    tol[::7] = 0.0                               # never met: those vectors run to k_max
    out = _check_adaptive(ctx, gid, ref, B, tol, k_max, False, vne.PROBE_RADEMACHER, seed=11)
    assert np.all(out["steps"][::7] == 0)
    ctx.release(gid)


def test_adaptive_dense_invariant_subspace(ctx):
    """A start vector in a 2-dimensional invariant subspace stops at the
    first check with zero error (bound 0 on a recurrence ended by beta = 0)."""
    _say("case adaptive stopping, invariant subspace")
    n = 400
    lam = np.linspace(1.0, 2.0, n) / n
    gid = ctx.register(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), lam, 1.0)
    B = np.zeros((n, 2))
    B[[3, 9], 0] = 1.0
    B[:, 1] = np.random.default_rng(2).standard_normal(n)
    out = ctx.estimate_adaptive(gid, vne.PROBE_DENSE, 2, 30, vne.MODE_F64, [1e-14, 0.0], 0.5 / n, 3.0 / n,
                                dense=B)
    exact = (B * B * oracle.f_entropy(lam)[:, None]).sum(0)
    assert out["steps"][0] == 3 and out["k_eff"][0] == 2 and out["steps"][1] == 0
    assert abs(out["quad"][0] - exact[0]) <= 1e-14 * abs(exact[0])
    ctx.release(gid)


def _exact_S(ref):
    return oracle.exact_entropy(oracle.dense_matrix(ref))


ALG_CASES = [("er", lambda: synth.erdos_renyi(1500, 8.0, 71), 1e-3),
             ("ba", lambda: synth.barabasi_albert(1200, 3, 72), 1e-3),
             ("ws", lambda: synth.watts_strogatz(2000, 8, 0.1, 73), 1e-3),
             ("grid", lambda: synth.grid2d_graph(30, 40), 1e-2),
             ("ring", lambda: synth.ring_lattice(3000, 10), 1e-3)]


def _pass_steps_agree(ctx, gid, ref, run, k_max):
    """The GPU's per-colour stop steps of one distance-d pass (its adaptive
    stopping on the oracle's colouring with the pass's tolerances) against
    the oracle's pass; returns whether every decision agrees."""
    A = ref.scipy()
    lam_hi = float(np.abs(A).sum(axis=1).max())
    s = run["n_colors"]
    out = ctx.estimate_adaptive(gid, vne.PROBE_COLORING, s, k_max, vne.MODE_DESING, run["tol"], 1e-12 * lam_hi,
                                lam_hi, n_grid=GRID, colors=run["colors"].astype(np.int32))
    gpu = np.where(out["steps"] > 0, out["steps"], k_max)
    same = bool(np.array_equal(out["steps"] > 0, run["converged"]) and np.array_equal(gpu, run["steps"]))
    if not same:
        _say("   d=%d: %d of %d stop decisions differ from the oracle's"
             % (run["d"], int(np.sum(gpu != run["steps"])), s))
    return same


@pytest.mark.parametrize("name,mk,eps", ALG_CASES)
def test_algorithm_2_matches_oracle(ctx, name, mk, eps):
    _say("case Algorithm 2, %s, eps=%g" % (name, eps))
    gid, ref = _setup(ctx, *mk(), fp64=False)
    k_max = 100
    got = ctx.probing(gid, eps, d_max=16, k_max=k_max, n=ref.n, quad_cap=4096)
    want = oprobing.probing_entropy(ref, eps, d_max=16, k_max=k_max)
    S = _exact_S(ref)
    err = abs(got["estimate"] - S) / S
    _say("   d=%d (oracle %d) colours %d, T_pre %s, estimate %.10f, S %.10f, rel err %.2e, "
         "vector steps %d, block steps %d, colouring %.1f ms, Lanczos %.1f ms"
         % (got["d"], want["d"], got["n_colors"], np.array2string(np.array(got["t_pre"]), precision=8),
            got["estimate"], S, err, got["vector_steps"], got["block_steps"], got["color_ms"], got["lanczos_ms"]))
    assert got["s_lower"] == pytest.approx(want["s0"], rel=1e-12)
    # T_1..T_3: 1e-5 where every stop decision of the pass agrees, 1e-4 where
    # one flips (the pass then sums a colour's psi one check earlier or later)
    for d in (1, 2, 3):
        same = _pass_steps_agree(ctx, gid, ref, want["runs"][d], k_max)
        _assert_within(abs(got["t_pre"][d - 1] - want["T_pre"][d - 1]) / abs(want["T_pre"][d - 1]),
                       TOL[False] if same else 1e-4, "T_%d" % d)
    if got["d"] != want["d"]:
        # the choice may flip only where the model sits at the target
        fits = oprobing.fit_heuristic(*want["T_pre"])
        dmin = min(got["d"], want["d"])
        assert abs(oprobing.heuristic_error(dmin, fits) - want["eps_hat"]) <= 1e-3 * want["eps_hat"]
    else:
        fin = want["final"]
        assert got["fallback"] == int(want["fallback"]) and got["capped"] == int(want["capped"])
        assert np.array_equal(got["colors"], fin["colors"])
        assert got["n_colors"] == fin["n_colors"]
        s = fin["n_colors"]
        gsteps = np.where(got["steps"][:s] > 0, got["steps"][:s], k_max)
        same = np.array_equal(got["steps"][:s] > 0, fin["converged"]) and np.array_equal(gsteps, fin["steps"])
        if same:
            _assert_within(_rel(got["quad"][:s], fin["psi"]), TOL[False], "final pass psi per colour")
        _assert_within(abs(got["estimate"] - want["estimate"]) / abs(want["estimate"]),
                       TOL[False] if same else 1e-4, "estimate")
    assert got["unconverged"] == 0
    assert err <= eps
    ctx.release(gid)


@pytest.mark.parametrize("name,mk,eps", ALG_CASES[:3])
def test_algorithm_2_with_the_estimate_rule(ctx, name, mk, eps):
    """Algorithm 2 with the eq. (4.10) stopping rule against the oracle's
    with the same rule: the same d and colouring, the final pass's stop
    steps, psi and the estimate at 1e-5 when the decisions agree; fewer
    vector steps than with the bound, and the exact entropy within eps S."""
    _say("case Algorithm 2 with the estimate rule, %s, eps=%g" % (name, eps))
    gid, ref = _setup(ctx, *mk(), fp64=False)
    got = ctx.probing(gid, eps, d_max=16, k_max=100, n=ref.n, quad_cap=4096, stop=vne.STOP_ESTIMATE)
    bnd = ctx.probing(gid, eps, d_max=16, k_max=100)
    want = oprobing.probing_entropy(ref, eps, d_max=16, k_max=100, stop="estimate")
    S = _exact_S(ref)
    err = abs(got["estimate"] - S) / S
    _say("   d=%d (oracle %d), vector steps %d (bound %d), rel err %.2e"
         % (got["d"], want["d"], got["vector_steps"], bnd["vector_steps"], err))
    if got["d"] == want["d"]:
        fin = want["final"]
        s = fin["n_colors"]
        assert np.array_equal(got["colors"], fin["colors"])
        gsteps = np.where(got["steps"][:s] > 0, got["steps"][:s], 100)
        same = np.array_equal(got["steps"][:s] > 0, fin["converged"]) and np.array_equal(gsteps, fin["steps"])
        if same:
            _assert_within(_rel(got["quad"][:s], fin["psi"]), TOL[False], "final pass psi per colour")
        _assert_within(abs(got["estimate"] - want["estimate"]) / abs(want["estimate"]),
                       TOL[False] if same else 1e-4, "estimate")
    assert got["vector_steps"] <= bnd["vector_steps"]
    assert err <= eps
    ctx.release(gid)


def test_algorithm_2_with_the_bound(ctx):
    _say("case Algorithm 2 with Corollary 3.2")
    gid, ref = _setup(ctx, *synth.erdos_renyi(600, 6.0, 74), fp64=False)
    got = ctx.probing(gid, 1e-2, select=vne.SELECT_BOUND, d_max=16, k_max=100, n=ref.n, quad_cap=4096)
    want = oprobing.probing_entropy(ref, 1e-2, d_max=16, k_max=100, select="bound")
    assert (got["d"], got["capped"], got["fallback"]) == (want["d"], int(want["capped"]), 1)
    assert got["passes"] == 1 and got["t_pre"] == [0.0, 0.0, 0.0]
    fin = want["final"]
    s = fin["n_colors"]
    assert np.array_equal(got["colors"], fin["colors"]) and got["n_colors"] == s
    gsteps = np.where(got["steps"][:s] > 0, got["steps"][:s], 100)
    same = np.array_equal(got["steps"][:s] > 0, fin["converged"]) and np.array_equal(gsteps, fin["steps"])
    if same:
        _assert_within(_rel(got["quad"][:s], fin["psi"]), TOL[False], "psi per colour")
    _assert_within(abs(got["estimate"] - want["estimate"]) / abs(want["estimate"]),
                   TOL[False] if same else 1e-4, "estimate")
    S = _exact_S(ref)
    assert abs(got["estimate"] - S) <= 1e-2 * S
    ctx.release(gid)


def test_probing_and_adaptive_errors(ctx):
    _say("case Algorithm 2 / adaptive stopping, error paths")
    gid, ref = _setup(ctx, *synth.erdos_renyi(200, 5.0, 75), fp64=False)
    for bad in [dict(rel_eps=0.0), dict(rel_eps=1.0), dict(select=2), dict(d_max=65), dict(k_max=2),
                dict(k_max=129), dict(lam_lo_fraction=1.0), dict(n_grid=1), dict(mode=8)]:
        args = dict(rel_eps=1e-2)
        args.update(bad)
        with pytest.raises(vne.VneError):
            ctx.probing(gid, **args)
    # not a density matrix
    n = 50
    g2 = ctx.register(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n), 1.0)
    with pytest.raises(vne.VneError):
        ctx.probing(g2, 1e-2, mode=0)
    lam_hi = 1.0
    with pytest.raises(vne.VneError) as ei:
        ctx.estimate_adaptive(gid, vne.PROBE_HUTCHPP, 8, 10, vne.MODE_DESING, 1e-3, 1e-12, lam_hi)
    assert ei.value.status == -4
    for tol, lo, hi, kmax in [(-1.0, 1e-12, 1.0, 10), (np.nan, 1e-12, 1.0, 10), (1e-3, 0.0, 1.0, 10),
                              (1e-3, 1.0, 0.5, 10), (1e-3, 1e-12, 1.0, 2)]:
        with pytest.raises(vne.VneError):
            ctx.estimate_adaptive(gid, vne.PROBE_RADEMACHER, 8, kmax, vne.MODE_DESING, tol, lo, hi)
    ctx.release(g2)
    ctx.release(gid)


def test_algorithm_2_closed_forms(ctx):
    """Closed-form entropies: the complete graph K_n (rho has eigenvalue
    1/(n-1) with multiplicity n-1: S = log(n-1)) and the star S_n (Laplacian
    eigenvalues 0, 1 (n-2 times) and n over tr L = 2(n-1))."""
    _say("case Algorithm 2, complete graph and star")
    for name, mk, S in [("complete", lambda: synth.complete_graph(300), np.log(299.0)),
                        ("star", lambda: synth.star_graph(500),
                         -(498 * (1 / 998) * np.log(1 / 998) + (500 / 998) * np.log(500 / 998)))]:
        gid, ref = _setup(ctx, *mk(), fp64=False)
        assert abs(S - oracle.exact_entropy(oracle.dense_matrix(ref))) < 1e-12 * S
        got = ctx.probing(gid, 1e-3, d_max=16, k_max=64)
        err = abs(got["estimate"] - S) / S
        _say("   %s: d=%d colours %d passes %d, rel err %.2e" % (name, got["d"], got["n_colors"], got["passes"], err))
        assert err <= 1e-3 and got["unconverged"] == 0
        ctx.release(gid)


def test_algorithm_2_reports_unconverged_colours(ctx):
    """With a step cap below what the tolerances need, every colour still
    gets its quadrature after k_max steps and the result says how many did
    not meet their tolerance; the same call with room converges."""
    _say("case Algorithm 2, step cap too small")
    gid, ref = _setup(ctx, *synth.erdos_renyi(2000, 8.0, 81), fp64=False)
    capped = ctx.probing(gid, 1e-5, d_max=3, k_max=3, quad_cap=4096)
    assert capped["unconverged"] > 0
    assert np.all(capped["steps"][capped["steps"] > 0] == 3)
    assert np.isfinite(capped["estimate"])
    free = ctx.probing(gid, 1e-5, d_max=3, k_max=128)
    assert free["unconverged"] == 0
    _say("   capped: %d of %d colours unconverged; with k_max 128: block steps %d"
         % (capped["unconverged"], capped["n_colors"], free["block_steps"]))
    ctx.release(gid)
