"""Pins of the trace estimators (eq. (3.2), (3.7), (3.8), (3.9);
Proposition 3.6; Corollary 3.2)."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth
from oracle import bounds

TAU64 = oracle.breakdown_tau(True)


def _g(kind, n, seed):
    if kind == "er":
        return oracle.laplacian_from_edges(*synth.erdos_renyi(n, 5.0, seed))
    if kind == "ba":
        return oracle.laplacian_from_edges(*synth.barabasi_albert(n, 2, seed))
    return oracle.laplacian_from_edges(*synth.watts_strogatz(n, 4, 0.1, seed))


def _f_dense(rho):
    lam, U = np.linalg.eigh(rho)
    return (U * oracle.f_entropy(lam)) @ U.T


def test_probing_with_one_colour_per_node_is_exact():
    g = _g("er", 30, 1)
    rho = oracle.dense_matrix(g)
    res = oracle.quadforms(g.scipy(), np.eye(g.n), g.n, TAU64)
    assert abs(oracle.probing_sum(res["psi"]) - oracle.exact_entropy(rho)) < 1e-10


@pytest.mark.parametrize("kind", ["er", "ba", "ws"])
def test_probing_lower_bound_error_identity_and_bound(kind):
    g = _g(kind, 160, 2)
    rho = oracle.dense_matrix(g)
    S = oracle.exact_entropy(rho)
    F = _f_dense(rho)
    lam_max = np.linalg.eigvalsh(rho)[-1]
    for d in (1, 2, 3):
        col, s = oracle.greedy_distance_coloring(g.row_ptr, g.col_idx, g.n, d)
        P = oracle.indicator_block(col, s)
        Td = float(np.einsum("ij,ij->", P, F @ P))                 # exact quadforms
        assert Td <= S + 1e-13                                      # Prop. 3.6
        same = (col[:, None] == col[None, :]) & ~np.eye(g.n, dtype=bool)
        assert abs((S - Td) - (-F[same].sum())) < 1e-12             # eq. (3.7)
        if d >= 2:
            assert S - Td <= bounds.cor32(d, g.n, 0.0, lam_max)      # eq. (3.6)
        # the Krylov route reaches the same T_d
        res = oracle.quadforms(g.scipy(), P, 60, TAU64)
        assert abs(oracle.probing_sum(res["psi"]) - Td) < 1e-9 * S


def test_hutchinson_is_unbiased():
    g = _g("ba", 120, 3)
    rho = oracle.dense_matrix(g)
    S = oracle.exact_entropy(rho)
    N = 3000
    X = oracle.rademacher_block(11, g.node_ids, np.arange(N))
    res = oracle.quadforms(g.scipy(), X, 40, TAU64)
    est = oracle.hutchinson(res["psi"])
    se = np.std(res["psi"]) / np.sqrt(N)
    assert abs(est - S) < 4.5 * se
    # each quadform matches the exact form
    assert np.allclose(res["psi"][:20], oracle.exact_quadform(rho, X[:, :20]), rtol=1e-9)


def test_hutchpp_with_full_sketch_is_exact():
    g = _g("er", 24, 4)
    rho = oracle.dense_matrix(g)
    S = oracle.exact_entropy(rho)
    Om = oracle.rademacher_block(1, g.node_ids, np.arange(g.n))
    G = oracle.rademacher_block(2, g.node_ids, np.arange(8))
    est, det = oracle.hutchpp(g.scipy(), Om, G, g.n, TAU64)
    assert abs(est - S) < 1e-9
    assert np.abs(det["psi"][g.n:]).max() < 1e-12          # nothing left outside range(Q)


def test_f_times_block_matches_dense_matrix_function():
    g = _g("ws", 90, 5)
    rho = oracle.dense_matrix(g)
    B = oracle.rademacher_block(3, g.node_ids, np.arange(6))
    Y, _ = oracle.estimators.f_times_block(g.scipy(), B, 60, TAU64)
    assert np.allclose(Y, _f_dense(rho) @ B, rtol=0, atol=1e-10 * np.abs(Y).max())


def test_hutchpp_is_unbiased():
    g = _g("ba", 100, 6)
    rho = oracle.dense_matrix(g)
    S = oracle.exact_entropy(rho)
    errs = []
    for t in range(40):
        Om = oracle.rademacher_block(100 + t, g.node_ids, np.arange(10))
        G = oracle.rademacher_block(200 + t, g.node_ids, np.arange(10))
        est, det = oracle.hutchpp(g.scipy(), Om, G, 40, TAU64)
        errs.append(est - S)
        Q = det["Q"]
        assert np.abs(Q.T @ Q - np.eye(10)).max() < 1e-12
        assert np.abs(Q.T @ det["Gt"]).max() < 1e-12
    errs = np.array(errs)
    assert abs(errs.mean()) < 4 * errs.std() / np.sqrt(errs.size)
