"""Pins of the bound functions (Theorem 2.2, Remark 2.3, Theorem 4.8,
Example 4.10)."""
import numpy as np
import pytest
from scipy.optimize import linprog

import oracle
from oracle import bounds


def _lp_minimax(k, a, b, npts=500):
    """Discrete minimax error of x log x by degree-k polynomials (a lower
    estimate of E_k on the interval)."""
    x = (a + b) / 2 + (b - a) / 2 * np.cos(np.linspace(0, np.pi, npts))
    f = np.where(x > 0, x * np.log(np.maximum(x, 1e-300)), 0.0)
    T = np.polynomial.chebyshev.chebvander((2 * x - (a + b)) / (b - a), k)
    ones = np.ones((npts, 1))
    res = linprog(np.r_[np.zeros(k + 1), 1.0],
                  A_ub=np.vstack([np.hstack([T, -ones]), np.hstack([-T, -ones])]),
                  b_ub=np.r_[f, -f], bounds=[(None, None)] * (k + 2), method="highs")
    return res.x[-1]


@pytest.mark.parametrize("a,b", [(0.0, 1.0), (1e-6, 1e-2), (1e-3, 1.0), (0.1, 1.0)])
@pytest.mark.parametrize("k", [2, 5, 12])
def test_theorem_2_2(a, b, k):
    lp = _lp_minimax(k, a, b)
    assert lp <= bounds.thm22(k, a, b) * (1 + 1e-9)
    assert bounds.thm22(k, a, b) <= bounds.thm22_proof(k, a, b) * (1 + 1e-12)
    assert abs(bounds.thm22_proof(k, a, b) / bounds.thm22_integral(k, a, b) - 1) < 1e-8
    if a == 0.0:
        assert abs(bounds.thm22(k, a, b) - bounds.rem23(k, b)) < 1e-15 * b


def test_theorem_4_8_bracket_on_example_4_10():
    # Example 4.10: diagonal A whose eigenvalues are Chebyshev points of
    # [1e-3, 1e3] (first kind), random b; f = x log x has the same |error|
    n = 2000
    j = np.arange(n)
    lam = 0.5 * (1e3 + 1e-3) + 0.5 * (1e3 - 1e-3) * np.cos((2 * j + 1) * np.pi / (2 * n))
    import scipy.sparse as sp
    A = sp.diags(lam).tocsr()
    rng = np.random.default_rng(4)
    b = rng.standard_normal((n, 1))
    exact = float(np.sum(b[:, 0] ** 2 * oracle.f_entropy(lam)))
    res = oracle.lanczos(A, b, 40, oracle.breakdown_tau(True))
    for m in (5, 10, 20, 30):
        psi = oracle.gauss_quadrature(res["alpha"][:, :m], res["beta"][:, :m], [m], res["norm2"])[0]
        err = abs(psi - exact)
        lo, hi, est = bounds.posterior_bracket(res["alpha"][0], res["beta"][0], m, res["norm2"][0],
                                               lam.min(), lam.max())
        assert lo * (1 - 1e-8) <= err <= hi * (1 + 1e-8)
        assert est / 30 < err < est * 30                     # geometric-mean estimate (4.10)


def test_entropy_divided_differences_pins():
    """The cancellation-free divided differences against their definitions
    away from theta (plain quotients in long double precision are not
    needed: |t| >= 0.1 leaves no cancellation), against the limits f'(theta)
    and f''(theta)/2 at z = theta, and continuity across the series switch."""
    th = 3.7e-4
    z = th * np.array([0.2, 0.5, 0.9, 1.1, 2.0, 7.0])
    d1, d2 = bounds.entropy_divided_differences(z, th)
    f = oracle.f_entropy
    fp = -np.log(th) - 1.0
    assert np.allclose(d1, (f(z) - f(th)) / (z - th), rtol=1e-12, atol=0)
    assert np.allclose(d2, ((f(z) - f(th)) / (z - th) - fp) / (z - th), rtol=1e-10, atol=0)
    e1, e2 = bounds.entropy_divided_differences(np.array([th]), th)
    assert np.isclose(e1[0], fp, rtol=1e-15) and np.isclose(e2[0], -0.5 / th, rtol=1e-15)
    for t in (1e-3 * (1 - 1e-9), 1e-3 * (1 + 1e-9), -1e-3 * (1 - 1e-9), -1e-3 * (1 + 1e-9)):
        a1, a2 = bounds.entropy_divided_differences(np.array([th * (1 + t)]), th)
        b1, b2 = bounds.entropy_divided_differences(np.array([th * (1 + t * (1 + 1e-7))]), th)
        assert abs(a1[0] - b1[0]) < 1e-9 * abs(a1[0]) and abs(a2[0] - b2[0]) < 1e-9 * abs(a2[0])


def test_g_m_entropy_matches_generic_away_from_ritz_values():
    rng = np.random.default_rng(2)
    n = 300
    lam = np.sort(rng.uniform(1e-4, 1e-2, n))
    import scipy.sparse as sp
    A = sp.diags(lam).tocsr()
    b = rng.standard_normal((n, 1))
    res = oracle.lanczos(A, b, 12, oracle.breakdown_tau(True))
    from scipy.linalg import eigh_tridiagonal
    m = 10
    theta, U = eigh_tridiagonal(res["alpha"][0][:m], res["beta"][0][:m - 1])
    z = np.geomspace(1e-4, 1e-2, 400)
    dist = np.min(np.abs(z[:, None] / theta[None, :] - 1.0), axis=1)
    z = z[dist > 0.05]
    g1 = bounds.g_m(z, theta, U, res["beta"][0][m - 1])
    g2 = bounds.g_m_entropy(z, theta, U, res["beta"][0][m - 1], 1e-12)
    # terms of size max|g| cancel in the sum over Ritz values: absolute bar
    assert np.allclose(g1, g2, rtol=1e-9, atol=1e-8 * np.abs(g1).max())
