"""Pins of the Gauss quadrature step (eq. (4.2), (4.3))."""
import numpy as np

import oracle


def _T(alpha, beta, k):
    return np.diag(alpha[:k]) + np.diag(beta[:k - 1], 1) + np.diag(beta[:k - 1], -1)


def test_quadrature_polynomials_need_no_eigendecomposition():
    rng = np.random.default_rng(0)
    for k in (1, 2, 7, 30):
        alpha = rng.uniform(0.1, 1.0, k)
        beta = rng.uniform(0.05, 0.5, k)
        T = _T(alpha, beta, k)
        e1 = np.zeros(k)
        e1[0] = 1.0
        for p in range(0, 5):
            q = oracle.gauss_quadrature(alpha, beta, k, 2.5, f=lambda x, p=p: x ** p)[0]
            assert abs(q - 2.5 * (np.linalg.matrix_power(T, p) @ e1)[0]) < 1e-12 * max(1, abs(q))
            v = oracle.f_of_T_e1(alpha, beta, k, f=lambda x, p=p: x ** p)
            assert np.allclose(v, np.linalg.matrix_power(T, p) @ e1, atol=1e-12)


def test_quadrature_entropy_matches_dense_eigh():
    rng = np.random.default_rng(1)
    k = 25
    alpha = rng.uniform(1e-4, 1e-2, k)
    beta = rng.uniform(1e-5, 1e-3, k)
    th, U = np.linalg.eigh(_T(alpha, beta, k))
    expect = 3.0 * np.sum(U[0] ** 2 * oracle.f_entropy(th))
    assert abs(oracle.gauss_quadrature(alpha, beta, k, 3.0)[0] - expect) < 1e-13 * abs(expect)


def test_first_moments_equal_lanczos_quantities():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((40, 40))
    A = A @ A.T / 40
    c = rng.standard_normal((40, 1))
    res = oracle.lanczos(A, c, 6, oracle.breakdown_tau(True))
    q1 = oracle.gauss_quadrature(res["alpha"], res["beta"], res["k_eff"], res["norm2"], f=lambda x: x)
    q2 = oracle.gauss_quadrature(res["alpha"], res["beta"], res["k_eff"], res["norm2"], f=lambda x: x * x)
    assert abs(q1[0] - res["alpha"][0, 0] * res["norm2"][0]) < 1e-12 * abs(q1[0])
    assert abs(q1[0] - (c.T @ A @ c)[0, 0]) < 1e-12 * abs(q1[0])
    assert abs(q2[0] - np.sum((A @ c) ** 2)) < 1e-12 * q2[0]
