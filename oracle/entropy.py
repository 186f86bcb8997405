"""Exact von Neumann entropy and exact quadratic forms by diagonalization.

* f(x) = -x log x with the convention 0 log 0 = 0, natural logarithm
  (paper Section 2, eq. (2.1)).  Reading: f(x) = 0 for x <= 0, which only
  matters for rounding-level negative eigenvalues of a PSD matrix.
* S(rho) = sum of f over the eigenvalues (eq. (2.1)), computed with LAPACK's
  symmetric eigensolver; small n only.
* psi(b) = b^T f(A) b = sum_i f(lambda_i) (u_i^T b)^2 via A = U diag(lambda) U^T
  (the definition of a matrix function, Section 3), the limit that the Krylov
  quadrature of eq. (4.2) converges to.

Pinned by closed-form spectra (complete, star, cycle, path, grid and ring
graphs), 0 <= S <= log(rank), S(I/n) = log n and the scaling relation (2.2)
(tests).
"""
import numpy as np


def f_entropy(x):
    """f(x) = -x log x, f(x) = 0 for x <= 0."""
    x = np.asarray(x, np.float64)
    out = np.zeros_like(x)
    pos = x > 0
    out[pos] = -x[pos] * np.log(x[pos])
    return out


def entropy_from_eigenvalues(lam):
    """eq. (2.1): S = -sum lambda log lambda, 0 log 0 = 0."""
    return float(np.sum(f_entropy(lam)))


def exact_entropy(rho_dense):
    """S(rho) by dense diagonalization."""
    lam = np.linalg.eigvalsh(np.asarray(rho_dense, np.float64))
    return entropy_from_eigenvalues(lam)


def exact_quadform(rho_dense, B):
    """psi_j = b_j^T f(rho) b_j for every column b_j of B (dense eigh)."""
    lam, U = np.linalg.eigh(np.asarray(rho_dense, np.float64))
    B = np.asarray(B, np.float64)
    if B.ndim == 1:
        B = B[:, None]
    proj = U.T @ B
    return (f_entropy(lam)[:, None] * proj * proj).sum(axis=0)
