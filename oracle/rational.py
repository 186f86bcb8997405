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

rational_run builds the basis one vector at a time and evaluates psi_j after
every step j (the basis size), with the poles either given step by step or
chosen by the switch rule of the Krylov method implementation (Section 5):
the method starts with poles at infinity and moves to finite poles once the
error estimate err_j = |psi_j - psi_{j-1}| has not dropped by the factor c^ell
over the last ell steps.  Readings where the paper leaves a choice: err_j is
the difference of consecutive forms; the rule is checked after each step j
with j - ell >= 2 (both estimates defined), and fires at the first j with
err_j >= c^ell err_{j-ell}; from that step on the finite poles are taken in
the caller's order (infinity again past the list).  A new direction that
keeps no more than 1e-12 of its norm after the orthogonalization counts as an
invariant subspace: the basis stops growing and later steps repeat psi.

Pinned by: exactness for r = p_{2m-1} / q_{m-1}^2 (Lemma 4.3), convergence to
the exact form, and agreement with full-reorthogonalization Lanczos when
every pole is infinite; the switch step on sequences whose errors decay
geometrically (it fires at the first checked step exactly when the ratio
is at least c), rational_run against rational_quadform for the pole
sequence the rule chose, and the invariant-subspace case against the exact
form (tests).
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


def switch_step(psi, ell, c):
    """The step j (1-based; psi[j-1] = psi_j) at which the switch rule first
    fires on the sequence psi, or 0 when it does not."""
    for j in range(ell + 2, len(psi) + 1):
        e_j = abs(psi[j - 1] - psi[j - 2])
        e_0 = abs(psi[j - ell - 1] - psi[j - ell - 2])
        if e_j >= c ** ell * e_0:
            return j
    return 0


def rational_run(A, b, steps, poles=None, finite_poles=(), ell=3, c=0.75, f=f_entropy, drop=1e-12):
    """psi_1..psi_steps of the rational Krylov method for one start vector b.
    poles: the pole of each of the steps - 1 steps (np.inf for infinity), or
    None for the switch rule with finite_poles.  Returns dict(psi, switch
    (step of the switch, 0: none), basis (vectors built), poles (the pole
    each step used))."""
    A = np.asarray(A, np.float64)
    n = A.shape[0]
    nb2 = float(np.dot(b, b))
    psi, used = [], []
    if nb2 == 0.0:
        return dict(psi=[0.0] * steps, switch=0, basis=0, poles=[np.inf] * (steps - 1))
    V = [b / np.sqrt(nb2)]
    growing = True
    switched = 0
    for j in range(1, steps + 1):
        Vb = np.stack(V, axis=1)
        Am = Vb.T @ A @ Vb
        th, U = np.linalg.eigh(0.5 * (Am + Am.T))
        psi.append(float(nb2 * np.sum(U[0] ** 2 * f(th))))
        if j == steps:
            break
        if poles is not None:
            xi = poles[j - 1]
        else:
            if switched == 0 and switch_step(psi, ell, c) == j:
                switched = j
            t = j - switched if switched else -1
            xi = finite_poles[t] if 0 <= t < len(finite_poles) else np.inf
        used.append(xi)
        if not growing:
            continue
        w = A @ V[-1]
        if np.isfinite(xi):
            w = np.linalg.solve(np.eye(n) - A / xi, w)
        w0 = np.linalg.norm(w)
        for _ in range(2):
            w = w - Vb @ (Vb.T @ w)
        nw = np.linalg.norm(w)
        if not nw > drop * w0:
            growing = False
            continue
        V.append(w / nw)
    return dict(psi=psi, switch=switched, basis=len(V), poles=used)
