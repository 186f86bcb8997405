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
