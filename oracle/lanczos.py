"""Polynomial Krylov (Lanczos) recurrence for quadratic forms b^T f(A) b.

The paper builds an orthonormal basis V_m of the Krylov space
span{b, Ab, ..., A^{m-1} b} (Section 4, polynomial case: all poles at
infinity) and approximates psi = b^T f(A) b by psi_m = ||b||^2 e_1^T f(A_m) e_1
with A_m = V_m^T A V_m (eq. (4.2)).  For symmetric A the projected matrix is
tridiagonal and the basis obeys the three-term recurrence; the paper itself
runs Arnoldi with full orthogonalization (Remark 4.2), which this module
provides as ``lanczos_full_reorth``.  ``lanczos`` is the plain short
recurrence without reorthogonalization, the variant the GPU path computes.

Order of operations within a step (the paper does not fix one):
    u = A v_j;  w = u - beta_{j-1} v_{j-1};  alpha_j = v_j . w;
    w = w - alpha_j v_j;  beta_j = ||w||;  v_{j+1} = w / beta_j.
Breakdown (not discussed in the paper): a column is frozen after step j when
beta_j <= tau (|alpha_j| + beta_{j-1}) (beta_0 = 0); its Krylov dimension
k_eff is then j, beta_j is recorded as 0 and later coefficients stay 0.
tau depends on the precision of the vectors the device keeps (see
``breakdown_tau``), so that both sides freeze the same columns.

Every column of the start block is an independent recurrence; the block
form below only evaluates the m recurrences side by side.

Pinned by: the moment identities of Lemma 4.3 (Gauss rule exact for degree
<= 2k-1), exactness once k reaches the Krylov dimension, the a-priori bound of
Proposition 4.4 with Theorem 2.2, monotone decrease of the Gauss values for
f = -x log x, and the full-reorthogonalization variant (tests).
"""
import numpy as np


def breakdown_tau(fp64_vectors):
    """Relative breakdown threshold.  FP32 vectors: 64 u_32 = 2^-18.  FP64
    vectors: 2^-23, above the sqrt(u_64) resolution of a beta obtained from
    one-pass float64 sums."""
    return 2.0 ** -23 if fp64_vectors else 2.0 ** -18


def _apply(A, X):
    return np.asarray(A @ X, np.float64)


def lanczos(A, C, k, tau, keep_basis=False):
    """Plain Lanczos on every column of the n x m start block C.

    Returns dict with alpha[m,k], beta[m,k], k_eff[m], norm2[m] (= ||c||^2)
    and, if keep_basis, V[k, n, m] (v_1..v_k).
    """
    C = np.asarray(C, np.float64)
    n, m = C.shape
    alpha = np.zeros((m, k))
    beta = np.zeros((m, k))
    k_eff = np.full(m, k, np.int64)
    norm2 = np.einsum("ij,ij->j", C, C)
    active = norm2 > 0
    k_eff[~active] = 0
    v_prev = np.zeros((n, m))
    beta_prev = np.zeros(m)
    v = np.zeros((n, m))
    v[:, active] = C[:, active] / np.sqrt(norm2[active])
    V = np.zeros((k, n, m)) if keep_basis else None
    for j in range(k):
        if not active.any():
            break
        if keep_basis:
            V[j][:, active] = v[:, active]
        u = _apply(A, v)
        w = u - beta_prev[None, :] * v_prev
        a = np.einsum("ij,ij->j", v, w)
        w = w - a[None, :] * v
        b = np.sqrt(np.einsum("ij,ij->j", w, w))
        alpha[active, j] = a[active]
        frozen_now = active & (b <= tau * (np.abs(a) + beta_prev))
        beta[active & ~frozen_now, j] = b[active & ~frozen_now]
        k_eff[frozen_now] = j + 1
        active = active & ~frozen_now
        v_prev = v
        v = np.zeros((n, m))
        v[:, active] = w[:, active] / b[active]
        beta_prev = np.where(active, b, 0.0)
    out = dict(alpha=alpha, beta=beta, k_eff=k_eff, norm2=norm2)
    if keep_basis:
        out["V"] = V
    return out


def lanczos_full_reorth(A, C, k, tau):
    """Same recurrence with full Gram-Schmidt reorthogonalization (twice)
    against all previous basis vectors: the paper's Arnoldi with full
    orthogonalization (Remark 4.2) with every pole at infinity."""
    C = np.asarray(C, np.float64)
    n, m = C.shape
    alpha = np.zeros((m, k))
    beta = np.zeros((m, k))
    k_eff = np.full(m, k, np.int64)
    norm2 = np.einsum("ij,ij->j", C, C)
    for c in range(m):
        if norm2[c] == 0:
            k_eff[c] = 0
            continue
        basis = [C[:, c] / np.sqrt(norm2[c])]
        b_prev = 0.0
        for j in range(k):
            vj = basis[-1]
            w = _apply(A, vj[:, None])[:, 0]
            if j > 0:
                w = w - b_prev * basis[-2]
            a = vj @ w
            w = w - a * vj
            Vb = np.stack(basis, axis=1)
            for _ in range(2):
                w = w - Vb @ (Vb.T @ w)
            b = np.linalg.norm(w)
            alpha[c, j] = a
            if b <= tau * (abs(a) + b_prev):
                k_eff[c] = j + 1
                break
            beta[c, j] = b
            basis.append(w / b)
            b_prev = b
    return dict(alpha=alpha, beta=beta, k_eff=k_eff, norm2=norm2)
