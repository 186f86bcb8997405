"""Pins of the rational Krylov cross-check (eq. (4.1), (4.2), Lemma 4.3)."""
import numpy as np

import oracle
import synth
from oracle import rational


def _setup():
    g = oracle.laplacian_from_edges(*synth.barabasi_albert(120, 2, 3))
    rho = oracle.dense_matrix(g)
    lam = np.linalg.eigvalsh(rho)
    rng = np.random.default_rng(0)
    c = oracle.desingularize(rng.standard_normal((g.n, 1)))[:, 0]
    return rho, lam, c


def test_all_poles_infinite_equals_lanczos():
    rho, lam, c = _setup()
    for m in (3, 6, 10):
        psi, _ = rational.rational_quadform(rho, c, [np.inf] * (m - 1))
        res = oracle.lanczos_full_reorth(rho, c[:, None], m, oracle.breakdown_tau(True))
        q = oracle.gauss_quadrature(res["alpha"], res["beta"], res["k_eff"], res["norm2"])[0]
        assert abs(psi - q) < 1e-12 * abs(q)


def test_lemma_4_3_rational_exactness():
    rho, lam, c = _setup()
    m = 5
    poles = rational.default_poles(m, 2, lam[1], lam[-1])
    V = rational.rational_basis(rho, c, poles)
    Am = V.T @ rho @ V
    q = np.prod([1 - lam / xi if np.isfinite(xi) else np.ones_like(lam) for xi in poles], axis=0)
    th, U = np.linalg.eigh(0.5 * (Am + Am.T))
    qth = np.prod([1 - th / xi if np.isfinite(xi) else np.ones_like(th) for xi in poles], axis=0)
    lam_all, W = np.linalg.eigh(rho)
    proj = (W.T @ c) ** 2
    qa = np.prod([1 - lam_all / xi if np.isfinite(xi) else np.ones_like(lam_all) for xi in poles], axis=0)
    for p in range(2 * m):
        exact = np.sum(proj * lam_all ** p / qa ** 2)
        approx = np.dot(c, c) * np.sum(U[0] ** 2 * th ** p / qth ** 2)
        assert abs(approx - exact) < 1e-9 * abs(exact), p


def test_rational_converges_to_exact():
    rho, lam, c = _setup()
    exact = oracle.exact_quadform(rho, c[:, None])[0]
    errs = []
    for m in (4, 8, 16):
        psi, _ = rational.rational_quadform(rho, c, rational.default_poles(m, 2, lam[1], lam[-1]))
        errs.append(abs(psi - exact) / abs(exact))
    assert errs[-1] < 1e-8 and errs[-1] < errs[0]
