"""Pins of the exact entropy and exact quadratic forms against closed forms
(eq. (2.1), (2.2); spectra of circulant and product graphs)."""
import numpy as np
import pytest

import oracle
import synth


def _S_from_laplacian_eigs(lam):
    lam = np.asarray(lam, np.float64)
    rho = lam / lam.sum()
    rho = rho[rho > 1e-300]
    return float(-np.sum(rho * np.log(rho)))


def _exact(n, e):
    g = oracle.laplacian_from_edges(n, e)
    return oracle.exact_entropy(oracle.dense_matrix(g))


@pytest.mark.parametrize("n", [2, 3, 5, 17, 40])
def test_complete_graph_entropy_is_log_n_minus_1(n):
    assert abs(_exact(*synth.complete_graph(n)) - np.log(n - 1)) < 1e-13


@pytest.mark.parametrize("n", [3, 8, 31])
def test_star(n):
    lam = np.r_[0.0, np.ones(n - 2), float(n)]
    assert abs(_exact(*synth.star_graph(n)) - _S_from_laplacian_eigs(lam)) < 1e-13


@pytest.mark.parametrize("n", [3, 10, 47])
def test_cycle(n):
    j = np.arange(n)
    lam = 2 - 2 * np.cos(2 * np.pi * j / n)
    assert abs(_exact(*synth.cycle_graph(n)) - _S_from_laplacian_eigs(lam)) < 1e-13


@pytest.mark.parametrize("n", [2, 9, 40])
def test_path(n):
    j = np.arange(n)
    lam = 2 - 2 * np.cos(np.pi * j / n)
    assert abs(_exact(*synth.path_graph(n)) - _S_from_laplacian_eigs(lam)) < 1e-13


@pytest.mark.parametrize("r,c", [(3, 4), (6, 7)])
def test_grid(r, c):
    i = np.arange(r)[:, None]
    j = np.arange(c)[None, :]
    lam = (2 - 2 * np.cos(np.pi * i / r)) + (2 - 2 * np.cos(np.pi * j / c))
    assert abs(_exact(*synth.grid2d_graph(r, c)) - _S_from_laplacian_eigs(lam.ravel())) < 1e-13


@pytest.mark.parametrize("n,k", [(11, 4), (30, 6), (50, 10)])
def test_ring_lattice(n, k):
    j = np.arange(n)[:, None]
    r = np.arange(1, k // 2 + 1)[None, :]
    lam = k - 2 * np.cos(2 * np.pi * j * r / n).sum(axis=1)
    assert abs(_exact(*synth.ring_lattice(n, k)) - _S_from_laplacian_eigs(lam)) < 1e-13


def test_entropy_range_and_maximally_mixed():
    for seed in range(3):
        n, e = synth.erdos_renyi(150, 5.0, seed)
        g = oracle.laplacian_from_edges(n, e)
        S = oracle.exact_entropy(oracle.dense_matrix(g))
        assert 0.0 <= S <= np.log(g.n - 1) + 1e-12        # rank n-1 when connected
    n = 37
    assert abs(oracle.exact_entropy(np.eye(n) / n) - np.log(n)) < 1e-13
    pure = np.zeros((5, 5))
    pure[2, 2] = 1.0
    assert oracle.exact_entropy(pure) == 0.0


def test_scaling_relation_2_2():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((30, 12))
    A = X @ X.T                       # PSD, rank 12, trace not 1
    for gamma in (0.01, 0.3, 2.5):
        lhs = oracle.exact_entropy(gamma * A)
        rhs = gamma * oracle.exact_entropy(A) - gamma * np.log(gamma) * np.trace(A)
        assert abs(lhs - rhs) < 1e-9 * max(1.0, abs(rhs))


def test_f_zero_convention():
    assert oracle.f_entropy(0.0) == 0.0
    assert oracle.f_entropy(-1e-18) == 0.0
    assert abs(oracle.f_entropy(np.e ** -1) - np.e ** -1) < 1e-16


@pytest.mark.parametrize("n", [5, 23])
def test_quadform_complete_graph_closed_form(n):
    g = oracle.laplacian_from_edges(*synth.complete_graph(n))
    rng = np.random.default_rng(n)
    B = rng.standard_normal((n, 6))
    psi = oracle.exact_quadform(oracle.dense_matrix(g), B)
    expect = np.log(n - 1) / (n - 1) * ((B * B).sum(0) - B.sum(0) ** 2 / n)
    assert np.allclose(psi, expect, rtol=1e-12, atol=0)


@pytest.mark.parametrize("maker", [lambda: synth.cycle_graph(64), lambda: synth.ring_lattice(90, 8)])
def test_quadform_circulant_via_fft(maker):
    n, e = maker()
    g = oracle.laplacian_from_edges(n, e)
    first_row = g.laplacian().toarray()[0] * g.scale
    mu = np.real(np.fft.fft(first_row))          # circulant eigenvalues
    rng = np.random.default_rng(3)
    B = rng.standard_normal((n, 5))
    bh = np.fft.fft(B, axis=0)
    expect = (oracle.f_entropy(mu)[:, None] * np.abs(bh) ** 2).sum(0) / n
    psi = oracle.exact_quadform(oracle.dense_matrix(g), B)
    assert np.allclose(psi, expect, rtol=1e-11, atol=0)


def test_quadform_trace_identity_and_desing_invariance():
    n, e = synth.barabasi_albert(80, 2, 4)
    g = oracle.laplacian_from_edges(n, e)
    rho = oracle.dense_matrix(g)
    S = oracle.exact_entropy(rho)
    assert abs(oracle.exact_quadform(rho, np.eye(g.n)).sum() - S) < 1e-12
    rng = np.random.default_rng(9)
    B = rng.standard_normal((g.n, 4)) + 3.0
    assert np.allclose(oracle.exact_quadform(rho, B),
                       oracle.exact_quadform(rho, oracle.desingularize(B)), rtol=1e-11)
