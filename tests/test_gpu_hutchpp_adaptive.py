"""GPU parity of adaptive Hutch++ (vne_hutchpp_adaptive; Section 3.2, eq.
(3.10); the adaptive Hutch++ implementation of Section 5) against the
oracle's reading of it (oracle/adaptive_hutchpp.py), through the C ABI.

Both sides run the same rule; its inputs are Hutch++ forms, which the
device computes to the parity bar of plain Hutch++.  Per round the sketch
width must agree exactly, the round estimate and the deflated forms' sample
standard deviation within the bar, and the Hutchinson count exactly (both
sides take the ceiling in FP64 from values that agree to the bar; a flip
would need the count's square root argument within the bar of an integer,
and the test says so if it happens).  The kept round's final run is then
checked like plain Hutch++ (estimate, sum over Q, every deflated form)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
import paper_2212_09642_amd as vne
from oracle.adaptive_hutchpp import adaptive_hutchpp, normal_quantile_two_sided

pytestmark = pytest.mark.gpu

from gpu_common import ctx, _say, _setup, _rel, _bar, _hutchpp_oracle, _check_hutchpp  # noqa: F401


def _compare_rounds(out, ora, A, ids, seed, k, fp64, desing=True, n_pilot=16, delta=1e-2):
    """Round by round against the oracle.  Bars: the round estimate within
    the plain-Hutch++ bar of its own sketch and pilot columns; the sample
    standard deviation within ||dq|| / sqrt(n - 1) (sd(x) = ||x - mean|| /
    sqrt(n - 1), and centring does not lengthen a vector), with dq the
    per-form bars times the forms; the Hutchinson count exactly.  Returns
    False when a count flips at an integer boundary (the later rounds then
    differ by construction)."""
    assert [r["nr"] for r in out["rounds"]] == [r["nr"] for r in ora["rounds"]][:len(out["rounds"])]
    z = normal_quantile_two_sided(delta)
    for g, o in zip(out["rounds"], ora["rounds"]):
        nr = o["nr"]
        Om = oracle.rademacher_block(seed, ids, np.arange(nr))
        G = oracle.rademacher_block(seed, ids, np.arange(128, 128 + n_pilot))
        est, det, sens = _hutchpp_oracle(A, Om, G, k, fp64, desing)
        assert est == o["estimate"]
        b_est = float(np.max(_bar(fp64, sens["estimate"])))
        assert abs(g["estimate"] - o["estimate"]) <= b_est * abs(o["estimate"]), (g, o, b_est)
        q = det["psi"][nr:]
        dq = np.sqrt(np.sum((_bar(fp64, sens["psi"][nr:]) * np.abs(q)) ** 2))
        b_sd = dq / math.sqrt(n_pilot - 1)
        assert abs(g["sd"] - o["sd"]) <= b_sd, (g, o, b_sd)
        if g["nh"] != o["nh"]:
            eh = o["eps_hat"]
            lo = (z * max(o["sd"] - b_sd, 0.0) / (eh * (1 + b_est))) ** 2
            hi = (z * (o["sd"] + b_sd) / (eh * (1 - b_est))) ** 2
            assert math.floor(lo) != math.floor(hi), (g, o, lo, hi)
            _say("  count flipped at an integer boundary in round N_r=%d (%d vs %d): later rounds not compared"
                 % (nr, g["nh"], o["nh"]))
            return False
    assert len(out["rounds"]) == len(ora["rounds"])
    assert out["n_sketch"] == ora["n_sketch"] and out["n_hutch"] == ora["n_hutch"]
    assert out["capped"] == ora["capped"]
    _say("  rounds %s, kept N_r=%d N_H=%d" % ([(r["nr"], r["nh"]) for r in out["rounds"]], out["n_sketch"],
                                              out["n_hutch"]))
    return True


def test_rank_10_function_keeps_a_sketch_of_12(ctx):
    # ten eigenvalues at 1/e (f = 1/e) and 190 at 1e-6 (f = 1.4e-5): f(A) is
    # rank 10 up to 4e-5 of its norm, and a sketch of 12 keeps f(A) Omega
    # within CholeskyQR2's reach (cond ~ 3e4); with 1e-12 for the small ones
    # (the oracle's pin) the device's Cholesky of the sketch fails
    # (VNE_ENUMERIC), where the oracle's Householder QR does not
    _say("case adaptive Hutch++ diagonal n=200, f(A) of rank 10 (+1e-6), FP64")
    lam = np.array([math.exp(-1.0)] * 10 + [1e-6] * 190)
    lam = lam[np.random.default_rng(3).permutation(lam.size)]
    exact = float(np.sum(-lam * np.log(lam)))
    n = lam.size
    rp = np.arange(n + 1, dtype=np.int32)
    gid = ctx.register(rp, np.arange(n, dtype=np.int32), lam, 1.0, node_keys=np.arange(n, dtype=np.int64))
    out = ctx.hutchpp_adaptive(gid, 4, rel_eps=1e-3, delta=1e-2, mode=vne.MODE_F64, seed=5, quad_cap=64)
    A = sp.diags(lam).tocsr()
    ora = adaptive_hutchpp(A, np.arange(n), 5, 4, eps=1e-3, desing=False)
    assert _compare_rounds(out, ora, A, np.arange(n), 5, 4, True, desing=False)
    assert out["n_sketch"] == 12 and out["n_hutch"] == 16
    # what remains after the sketch is 190 eigenvalues of f = 1.4e-5
    assert abs(out["estimate"] - exact) <= 5 * out["std_error"] + 1e-12 * exact
    # the kept round is the last and asks for the pilot's count: no final run
    assert out["krylov_runs"] == ora["krylov_runs"] == sum(2 * r["nr"] + 16 for r in ora["rounds"])


@pytest.mark.parametrize("fp64", [True, False])
def test_barabasi_albert_matches_oracle(ctx, fp64):
    _say("case adaptive Hutch++ BA n=2000 rel_eps=0.05 fp64=%s" % fp64)
    n, e = synth.barabasi_albert(2000, 3, 23)
    gid, ref = _setup(ctx, n, e, fp64)
    k = 30
    mode = vne.MODE_DESING | (vne.MODE_F64 if fp64 else 0)
    out = ctx.hutchpp_adaptive(gid, k, rel_eps=0.05, delta=1e-2, mode=mode, seed=21, quad_cap=4096)
    A = ref.scipy()
    ora = adaptive_hutchpp(A, ref.node_ids, 21, k, eps=0.05, delta=1e-2, fp64_tau=fp64)
    if not _compare_rounds(out, ora, A, ref.node_ids, 21, k, fp64):
        return
    assert out["krylov_runs"] == ora["krylov_runs"]
    nr, nh = out["n_sketch"], out["n_hutch"]
    Om = oracle.rademacher_block(21, ref.node_ids, np.arange(nr))
    G = oracle.rademacher_block(21, ref.node_ids, np.arange(128, 128 + nh))
    est, det, sens = _hutchpp_oracle(A, Om, G, k, fp64)
    _check_hutchpp(dict(estimate=out["estimate"], quad=out["quad"]), est, det, sens, nr, fp64)
    assert ora["estimate"] == est
    q = det["psi"][nr:]
    assert _rel(out["std_error"], np.std(q, ddof=1) / math.sqrt(nh)) <= (1e-9 if fp64 else 1e-3)


def test_wide_first_sketch_and_absolute_tolerance(ctx):
    # r_first = r_max: one round; an absolute tolerance fixes eps_hat
    _say("case adaptive Hutch++ ER n=1500 single round, abs_eps")
    n, e = synth.erdos_renyi(1500, 8.0, 5)
    gid, ref = _setup(ctx, n, e, True)
    out = ctx.hutchpp_adaptive(gid, 25, abs_eps=0.02, delta=0.05, mode=vne.MODE_DESING | vne.MODE_F64, seed=3,
                               r_first=24, r_max=24, n_pilot=8, quad_cap=4096)
    ora = adaptive_hutchpp(ref.scipy(), ref.node_ids, 3, 25, eps_abs=0.02, delta=0.05, n_pilot=8, r_first=24,
                           r_max=24)
    assert len(out["rounds"]) == 1 and out["eps_hat"] == 0.02
    z = normal_quantile_two_sided(0.05)
    g, o = out["rounds"][0], ora["rounds"][0]
    assert g["nh"] == o["nh"] == max(8, math.ceil((z * o["sd"] / 0.02) ** 2))
    assert abs(out["estimate"] - ora["estimate"]) <= 1e-10 * abs(ora["estimate"])


def test_cap_and_errors(ctx):
    _say("case adaptive Hutch++ cap and error paths")
    n, e = synth.cycle_graph(300)
    gid, ref = _setup(ctx, n, e, True)
    mode = vne.MODE_DESING | vne.MODE_F64
    out = ctx.hutchpp_adaptive(gid, 20, rel_eps=1e-4, mode=mode, seed=1, r_first=3, r_max=3, n_h_max=32)
    assert out["capped"] and out["n_hutch"] == 32 and out["rounds"][0]["nh"] > 32
    bad = [dict(k=0), dict(k=129), dict(rel_eps=0.0), dict(rel_eps=1.0), dict(delta=0.0), dict(delta=1.0),
           dict(abs_eps=-1.0), dict(abs_eps=float("inf")), dict(n_pilot=1), dict(n_pilot=1025),
           dict(r_first=129), dict(r_first=8, r_max=4), dict(r_max=129), dict(n_pilot=16, n_h_max=8),
           dict(mode=vne.MODE_F64 | (1 << 9))]
    for b in bad:
        kw = dict(k=10, rel_eps=0.1, delta=0.01, mode=mode, seed=0)
        kw.update(b)
        k = kw.pop("k")
        with pytest.raises(vne.VneError) as ei:
            ctx.hutchpp_adaptive(gid, k, **kw)
        assert ei.value.status == -1, b
    with pytest.raises(vne.VneError):
        ctx.hutchpp_adaptive(gid + 1000, 10)
    # DESING on a matrix whose rows do not sum to zero
    rp = np.arange(11, dtype=np.int32)
    g2 = ctx.register(rp, np.arange(10, dtype=np.int32), np.ones(10), 0.1)
    with pytest.raises(vne.VneError):
        ctx.hutchpp_adaptive(g2, 5, mode=vne.MODE_DESING | vne.MODE_F64)
    # the context still works
    out = ctx.hutchpp_adaptive(gid, 10, rel_eps=0.1, mode=mode, seed=2)
    assert out["n_sketch"] >= 3 and np.isfinite(out["estimate"])
