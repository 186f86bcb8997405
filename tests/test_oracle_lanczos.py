"""Pins of the oracle's Lanczos quadrature (Section 4: eq. (4.2), Lemma 4.3,
Proposition 4.4 with Theorem 2.2)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import bounds


def _graph(kind="er", n=200, seed=1):
    if kind == "er":
        nn, e = synth.erdos_renyi(n, 6.0, seed)
    elif kind == "ba":
        nn, e = synth.barabasi_albert(n, 3, seed)
    else:
        nn, e = synth.watts_strogatz(n, 6, 0.1, seed)
    return oracle.laplacian_from_edges(nn, e)


TAU64 = oracle.breakdown_tau(True)


@pytest.mark.parametrize("kind", ["er", "ba", "ws"])
def test_moments_lemma_4_3(kind):
    g = _graph(kind, 150, 3)
    A = g.scipy()
    rng = np.random.default_rng(0)
    C = oracle.desingularize(rng.standard_normal((g.n, 3)))
    k = 5
    res = oracle.lanczos(A, C, k, TAU64)
    for p in range(0, 2 * k):
        quad = oracle.gauss_quadrature(res["alpha"], res["beta"], res["k_eff"], res["norm2"],
                                       f=lambda x, p=p: x ** p)
        X = C.copy()
        for _ in range(p // 2):
            X = A @ X
        if p % 2:
            exact = np.einsum("ij,ij->j", X, A @ X)
        else:
            exact = np.einsum("ij,ij->j", X, X)
        assert np.allclose(quad, exact, rtol=1e-10, atol=0), p
    # degree 2k is no longer exact
    quad = oracle.gauss_quadrature(res["alpha"], res["beta"], res["k_eff"], res["norm2"],
                                   f=lambda x: x ** (2 * k))
    X = C.copy()
    for _ in range(k):
        X = A @ X
    assert not np.allclose(quad, np.einsum("ij,ij->j", X, X), rtol=1e-6, atol=0)


def test_exact_at_krylov_dimension():
    g = _graph("er", 40, 7)
    rho = oracle.dense_matrix(g)
    rng = np.random.default_rng(1)
    B = rng.standard_normal((g.n, 4))
    C = oracle.desingularize(B)
    exact = oracle.exact_quadform(rho, B)
    full = oracle.lanczos_full_reorth(rho, C, g.n, TAU64)
    psi = oracle.gauss_quadrature(full["alpha"], full["beta"], full["k_eff"], full["norm2"])
    assert np.allclose(psi, exact, rtol=1e-11)
    # rounding noise along the null vector 1 is amplified by the recurrence
    # (0 lies outside [lambda_2, lambda_n]) and can add one direction, but the
    # Gauss weight it receives stays at rounding level, so psi is unaffected
    assert np.all(full["k_eff"] <= g.n)


def test_complete_graph_breaks_down_after_one_step():
    n = 25
    g = oracle.laplacian_from_edges(*synth.complete_graph(n))
    rng = np.random.default_rng(2)
    B = rng.choice([-1.0, 1.0], size=(n, 6))
    for tau in (oracle.breakdown_tau(True), oracle.breakdown_tau(False)):
        res = oracle.quadforms(g.scipy(), B, 10, tau)
        assert np.all(res["k_eff"] == 1)
        expect = np.log(n - 1) / (n - 1) * ((B * B).sum(0) - B.sum(0) ** 2 / n)
        assert np.allclose(res["psi"], expect, rtol=1e-13)


@pytest.mark.parametrize("kind", ["er", "ba"])
def test_prop_4_4_bound_and_gauss_monotonicity(kind):
    g = _graph(kind, 300, 5)
    rho = oracle.dense_matrix(g)
    lam = np.linalg.eigvalsh(rho)
    lam2, lamn = lam[1], lam[-1]
    rng = np.random.default_rng(4)
    B = rng.choice([-1.0, 1.0], size=(g.n, 5))
    exact = oracle.exact_quadform(rho, B)
    C = oracle.desingularize(B)
    norm2 = (C * C).sum(0)
    prev = np.full(5, np.inf)
    for k in range(1, 13):
        res = oracle.quadforms(g.scipy(), B, k, TAU64)
        psi = res["psi"]
        # Gauss rule overestimates: even derivatives of -x log x are negative
        assert np.all(psi >= exact - 1e-14 * np.abs(exact))
        assert np.all(psi <= prev + 1e-14 * np.abs(psi))
        prev = psi
        if k >= 2:
            assert np.all(np.abs(psi - exact) <= bounds.prop44_poly(k, norm2, lam2, lamn))


def test_plain_matches_full_reorth_before_orthogonality_loss():
    g = _graph("ws", 400, 9)
    rng = np.random.default_rng(6)
    C = oracle.desingularize(rng.choice([-1.0, 1.0], size=(g.n, 3)))
    a = oracle.lanczos(g.scipy(), C, 8, TAU64)
    b = oracle.lanczos_full_reorth(g.scipy(), C, 8, TAU64)
    assert np.allclose(a["alpha"], b["alpha"], rtol=1e-11)
    assert np.allclose(a["beta"], b["beta"], rtol=1e-11)


def test_plain_lanczos_converges_despite_orthogonality_loss():
    # many more steps than needed: ghosts appear but the quadrature stays put
    g = _graph("ba", 250, 8)
    rho = oracle.dense_matrix(g)
    rng = np.random.default_rng(7)
    B = rng.choice([-1.0, 1.0], size=(g.n, 4))
    exact = oracle.exact_quadform(rho, B)
    res = oracle.quadforms(g.scipy(), B, 120, TAU64)
    assert np.allclose(res["psi"], exact, rtol=1e-10)


def test_zero_start_vector_gives_zero():
    g = _graph("er", 50, 2)
    B = np.ones((g.n, 2))                      # desingularizes to 0
    res = oracle.quadforms(g.scipy(), B, 5, TAU64)
    assert np.all(res["k_eff"] == 0) and np.all(res["psi"] == 0)
