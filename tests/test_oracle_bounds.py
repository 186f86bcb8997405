"""Pins of the bound functions (Theorem 2.2, Remark 2.3, Theorem 4.8,
Example 4.10)."""
import numpy as np
import pytest
from scipy.optimize import linprog

import oracle
from oracle import bounds
import synth


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


def _g48_mp(a, b, m, z, dps=60):
    """Eq. (4.8) for -x log x written out term by term in dps-digit arithmetic."""
    import mpmath as mp
    mp.mp.dps = dps
    T = mp.matrix(m, m)
    for i in range(m):
        T[i, i] = mp.mpf(a[i])
        if i < m - 1:
            T[i, i + 1] = T[i + 1, i] = mp.mpf(b[i])
    E, Q = mp.eigsy(T)
    bm = mp.mpf(b[m - 1])
    th = [E[j] for j in range(m)]
    ab = [bm * Q[m - 1, j] * Q[0, j] for j in range(m)]
    cj = [mp.fsum(ab[l] / (th[j] - th[l]) for l in range(m) if l != j) for j in range(m)]
    f = lambda x: -x * mp.log(x)
    fp = lambda x: -mp.log(x) - 1
    out = []
    for zz in z:
        zz = mp.mpf(zz)
        g = mp.mpf(0)
        for j in range(m):
            d1 = (f(zz) - f(th[j])) / (zz - th[j])
            d2 = (d1 - fp(th[j])) / (zz - th[j])
            g += ab[j] ** 2 * d2 + 2 * ab[j] * cj[j] * d1
        out.append(float(g))
    return np.array(out)


@pytest.mark.slow
def test_g_m_residue_form_against_eq_4_8_in_high_precision():
    """The bracket's g_m (residue form) equals eq. (4.8) evaluated in 60-digit
    arithmetic on Lanczos matrices of a graph Laplacian, up to m = 39, where
    eq. (4.8) in double precision has lost several digits; |g_m| decreases
    in z and g_m < 0."""
    g = oracle.laplacian_from_edges(*synth.barabasi_albert(1500, 3, 33))
    A = g.scipy()
    B = oracle.rademacher_block(3, g.node_ids, np.arange(2))
    res = oracle.lanczos(A, oracle.desingularize(B), 40, oracle.breakdown_tau(True))
    lam_hi = float(np.abs(A).sum(1).max())
    z = np.array([1e-12 * lam_hi, 1e-6 * lam_hi, 1e-3 * lam_hi, lam_hi])
    for c in range(2):
        for m in (3, 12, 25, 39):
            a, b = res["alpha"][c], res["beta"][c]
            want = _g48_mp(a, b, m, z)
            got = bounds.g_m_resolvent(z, a, b, m)
            assert np.all(want < 0) and np.all(np.diff(np.abs(want)) < 0)
            assert np.allclose(got, want, rtol=1e-10, atol=0), (c, m, got, want)


def test_g_m_residue_form_against_adaptive_quadrature():
    """The trapezoidal rule in ln t against QUADPACK on the same integral,
    with the corner entry of the resolvent from a banded solve."""
    from scipy import integrate
    from scipy.linalg import solve_banded
    g = oracle.laplacian_from_edges(*synth.watts_strogatz(800, 6, 0.1, 3))
    A = g.scipy()
    B = oracle.rademacher_block(5, g.node_ids, np.arange(1))
    res = oracle.lanczos(A, oracle.desingularize(B), 30, oracle.breakdown_tau(True))
    a, b = res["alpha"][0], res["beta"][0]
    for m in (2, 9, 30):
        def h2(t):
            ab = np.zeros((3, m))
            ab[0, 1:] = b[:m - 1]
            ab[1] = a[:m] + t
            ab[2, :-1] = b[:m - 1]
            e = np.zeros(m)
            e[-1] = 1.0
            return (b[m - 1] * solve_banded((1, 1), ab, e)[0]) ** 2
        for zz in (1e-9, 1e-5, 3e-3):
            val, _ = integrate.quad(lambda s: np.exp(2 * s) * h2(np.exp(s)) / (np.exp(s) + zz), -80, 20,
                                    limit=2000, epsabs=0, epsrel=1e-12)
            assert bounds.g_m_resolvent([zz], a, b, m)[0] == pytest.approx(-val, rel=1e-9)
