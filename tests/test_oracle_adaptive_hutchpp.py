"""Pins of the adaptive Hutch++ oracle (oracle/adaptive_hutchpp.py): the rule
pieces on hand-worked values, composition with plain Hutch++, a matrix whose
f(A) has rank 10, and the coverage of the tail bound eq. (3.10) over seeds."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from oracle.adaptive_hutchpp import adaptive_hutchpp, hutch_count, kept_round, normal_quantile_two_sided


def test_normal_quantile_textbook_values():
    # two-sided tails of the standard normal: 1%, 5% and the one-sigma tail
    assert normal_quantile_two_sided(0.01) == pytest.approx(2.5758293035489004, abs=1e-12)
    assert normal_quantile_two_sided(0.05) == pytest.approx(1.959963984540054, abs=1e-12)
    assert normal_quantile_two_sided(0.31731050786291415) == pytest.approx(1.0, abs=1e-12)


def test_hutch_count_hand_cases():
    # (z s / eps_hat)^2 = (2 * 1 / 0.1)^2 = 400 exactly
    assert hutch_count(1.0, 0.1, 2.0, 16) == 400
    # 401.0000...: the next integer
    assert hutch_count(1.0, 0.1, 2.0 * math.sqrt(401.0001 / 400.0), 16) == 402
    assert hutch_count(0.0, 0.1, 2.0, 16) == 16             # no spread: the pilot
    assert hutch_count(1e-3, 1.0, 2.576, 16) == 16          # below the pilot
    assert hutch_count(1.0, 1e-30, 2.576, 16) == 10 ** 15   # square capped


def test_kept_round():
    assert kept_round([4102, 70, 40, 64]) == 2
    assert kept_round([30, 30]) == 0
    assert kept_round([10]) == 0


def _ba(n, seed):
    nn, e = synth.barabasi_albert(n, 3, seed)
    ref = oracle.laplacian_from_edges(nn, e)
    return ref, ref.scipy()


def test_single_round_is_plain_hutchpp():
    ref, A = _ba(300, 4)
    out = adaptive_hutchpp(A, ref.node_ids, 9, 25, eps=0.05, r_first=4, r_max=4)
    assert len(out["rounds"]) == 1 and out["n_sketch"] == 4
    nh = out["n_hutch"]
    Om = oracle.rademacher_block(9, ref.node_ids, np.arange(4))
    G = oracle.rademacher_block(9, ref.node_ids, np.arange(128, 128 + nh))
    est, det = oracle.hutchpp(A, Om, G, 25, oracle.breakdown_tau(True))
    assert out["estimate"] == est
    assert np.array_equal(out["psi"], det["psi"])
    # the round's own numbers follow the rule
    r = out["rounds"][0]
    z = normal_quantile_two_sided(1e-2)
    assert r["eps_hat"] == 0.5 * 0.05 * abs(r["estimate"])
    assert r["nh"] == hutch_count(r["sd"], r["eps_hat"], z, 16) == nh


def _rank10():
    # f(A) = -A log A with ten eigenvalues at 1/e (f = 1/e, its largest value)
    # and 190 at 1e-12 (f ~ 2.8e-11): numerically rank 10
    lam = np.array([math.exp(-1.0)] * 10 + [1e-12] * 190)
    perm = np.random.default_rng(3).permutation(lam.size)
    lam = lam[perm]
    exact = float(np.sum(-lam * np.log(lam)))
    return sp.diags(lam).tocsr(), np.arange(lam.size), exact


def test_rank_10_function_keeps_a_sketch_of_12():
    A, ids, exact = _rank10()
    out = adaptive_hutchpp(A, ids, 5, 4, eps=1e-3, desing=False)
    nr = [r["nr"] for r in out["rounds"]]
    # widths 3 and 6 leave part of the rank-10 range in the deflated matrix
    # (near a million forms asked for); 12 takes all of it (the pilot
    # suffices: effort 2 * 12 + 16 = 40); width 24 could not do better
    # (2 * 24 + 16 = 64), so the rounds end at 12
    assert nr == [3, 6, 12]
    assert out["rounds"][0]["nh"] > 10 ** 5 and out["rounds"][1]["nh"] > 10 ** 5
    assert out["n_sketch"] == 12 and out["n_hutch"] == 16 and not out["capped"]
    assert abs(out["estimate"] - exact) <= 1e-9 * exact
    # the last round is the final run: 2 * (3 + 6 + 12) + 3 * 16 Krylov runs
    assert out["krylov_runs"] == 2 * 21 + 48
    # and it is the same as running it again
    Om = oracle.rademacher_block(5, ids, np.arange(12))
    G = oracle.rademacher_block(5, ids, np.arange(128, 144))
    est, det = oracle.hutchpp(A, Om, G, 4, oracle.breakdown_tau(True), False)
    assert out["estimate"] == est


def test_capped_count_is_flagged():
    A, ids, exact = _rank10()
    out = adaptive_hutchpp(A, ids, 5, 4, eps=1e-3, desing=False, r_first=3, r_max=3, n_h_max=64)
    assert out["capped"] and out["n_hutch"] == 64 and out["n_sketch"] == 3


def test_tail_bound_coverage_over_seeds():
    """eq. (3.10) with eps_hat = eps/2 S: over 300 seeds the estimate misses
    by eps_hat or more in at most delta of the runs (plus three binomial
    standard deviations)."""
    nn, e = synth.erdos_renyi(60, 5.0, 2)
    ref = oracle.laplacian_from_edges(nn, e)
    A = ref.scipy()
    S = oracle.exact_entropy(A.toarray())
    eps, delta, runs = 0.05, 0.2, 300
    miss = 0
    for seed in range(runs):
        out = adaptive_hutchpp(A, ref.node_ids, 1000 + seed, 60, eps=eps, delta=delta)
        miss += abs(out["estimate"] - S) >= 0.5 * eps * S
    bar = delta + 3 * math.sqrt(delta * (1 - delta) / runs)
    assert miss / runs <= bar, (miss, runs, bar)
