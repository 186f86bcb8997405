"""Gauss quadrature from the Lanczos coefficients (paper eq. (4.2)):
psi_k = ||c||^2 e_1^T f(T_k) e_1, where T_k is the symmetric tridiagonal
matrix with diagonal alpha_1..alpha_k and off-diagonal beta_1..beta_{k-1}.
With T_k = U diag(theta) U^T this is ||c||^2 sum_i U[0,i]^2 f(theta_i)
(Golub-Welsch: nodes theta_i, weights U[0,i]^2).

f_of_T_e1 returns f(T_k) e_1, the coefficient vector of the Krylov
approximation f(A) b ~ ||b|| V_k f(T_k) e_1 (eq. (4.3)).

Nonpositive Ritz values get f = 0 (0 log 0 = 0, eq. (2.1)).

Pinned by: agreement with a dense eigendecomposition of T_k, f(x) = x and
f(x) = x^2 reproducing alpha_1 ||c||^2 and ||A c||^2 (tests).
"""
import numpy as np
from scipy.linalg import eigh_tridiagonal

from .entropy import f_entropy


def _eig(alpha, beta, k):
    if k == 1:
        return np.array([alpha[0]]), np.ones((1, 1))
    return eigh_tridiagonal(alpha[:k], beta[:k - 1])


def gauss_quadrature(alpha, beta, k_eff, norm2, f=f_entropy):
    """psi for every column; alpha, beta are [m, k] arrays."""
    alpha = np.atleast_2d(alpha)
    beta = np.atleast_2d(beta)
    k_eff = np.atleast_1d(k_eff)
    norm2 = np.atleast_1d(norm2)
    out = np.zeros(alpha.shape[0])
    for c in range(alpha.shape[0]):
        k = int(k_eff[c])
        if k == 0:
            continue
        theta, U = _eig(alpha[c], beta[c], k)
        out[c] = norm2[c] * np.sum(U[0] ** 2 * f(theta))
    return out


def f_of_T_e1(alpha, beta, k, f=f_entropy):
    """f(T_k) e_1 as a k-vector."""
    if k == 0:
        return np.zeros(0)
    theta, U = _eig(alpha, beta, k)
    return U @ (f(theta) * U[0])
