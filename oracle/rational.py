"""Rational Krylov cross-check (paper Section 4, eq. (4.1) and (4.2)).

Rational Arnoldi with full orthogonalization: v_1 = b / ||b||, and for
j = 1, ..., m-1 the next direction is (I - A / xi_j)^{-1} A v_j
(xi_j = inf gives A v_j), orthogonalized twice against all previous basis
vectors.  The basis spans q_{m-1}(A)^{-1} K_m(A, b) with
q_{m-1}(z) = prod (1 - z / xi_j) (eq. (4.1)).  The quadratic form is
psi_m = ||b||^2 e_1^T f(A_m) e_1 with the explicit projection A_m = V^T A V
(eq. (4.2)).  Dense linear algebra; small n only.  This path is kept only as a
cross-check of the polynomial one.

The paper's EDS poles are not described in enough detail to rebuild; the
cross-check uses a few poles at infinity followed by fixed negative poles
spread logarithmically over [-lambda_max, -lambda_min].

Pinned by: exactness for r = p_{2m-1} / q_{m-1}^2 (Lemma 4.3), convergence to
the exact form, and agreement with full-reorthogonalization Lanczos when
every pole is infinite (tests).
"""
import numpy as np

from .entropy import f_entropy


def rational_basis(A, b, poles):
    A = np.asarray(A, np.float64)
    n = A.shape[0]
    V = [b / np.linalg.norm(b)]
    for xi in poles:
        w = A @ V[-1]
        if np.isfinite(xi):
            w = np.linalg.solve(np.eye(n) - A / xi, w)
        Vb = np.stack(V, axis=1)
        for _ in range(2):
            w = w - Vb @ (Vb.T @ w)
        nw = np.linalg.norm(w)
        if nw == 0:
            break
        V.append(w / nw)
    return np.stack(V, axis=1)


def rational_quadform(A, b, poles, f=f_entropy):
    V = rational_basis(A, b, poles)
    Am = V.T @ np.asarray(A, np.float64) @ V
    Am = 0.5 * (Am + Am.T)
    th, U = np.linalg.eigh(Am)
    return float(np.dot(b, b) * np.sum(U[0] ** 2 * f(th))), V


def default_poles(m, n_inf, lam_min, lam_max):
    """n_inf poles at infinity, then m-1-n_inf negative poles, log-spaced."""
    finite = -np.geomspace(lam_max, lam_min, max(m - 1 - n_inf, 0))
    return [np.inf] * min(n_inf, m - 1) + list(finite)
