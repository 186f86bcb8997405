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
poles at infinity first, then finite poles once the error bound err_j
(Theorem 4.8's upper bound, eq. (4.9), or the geometric-mean estimate of
eq. (4.10), over the caller's interval [lam_lo, lam_hi]) fails to drop by
c^ell between steps j - ell - 1 and j: err_j / err_{j-ell-1} >= c^ell,
checked after every polynomial step j >= ell + 2.  While every pole so far
is infinite the projection V_j^T A V_j is Lanczos's T_j, so the bound is
the polynomial one: alpha and beta_1..beta_{j-1} from the projection and
beta_j the norm of A v_j orthogonalized against V_j.  The pole of the switch
step and of the steps after it are the caller's finite poles in order
(infinity again past the list).  Readings where the paper leaves a choice:
the finite poles themselves (the EDS poles are not described in enough
detail to rebuild), and a new direction that keeps no more than 1e-12 of its
norm after the orthogonalization counts as an invariant subspace: the basis
stops growing, beta_j is 0 and later steps repeat psi.

Pinned by: exactness for r = p_{2m-1} / q_{m-1}^2 (Lemma 4.3), convergence to
the exact form, and agreement with full-reorthogonalization Lanczos when
every pole is infinite; the switch step on error sequences that decay
geometrically (it fires at the first checked step exactly when the ratio
per step is at least c^(ell / (ell + 1))) and on a hand-worked sequence;
the bounds of a switch-rule run against Theorem 4.8 evaluated on the
Lanczos coefficients of the same start vector; rational_run against
rational_quadform for the pole sequence the rule chose; and the
invariant-subspace case against the exact form (tests).
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


def switch_step(err, ell, c):
    """The step j (1-based; err[j-1] = err_j) at which the switch rule first
    fires on the error bounds err: err_j >= c^ell err_{j-ell-1}, or 0."""
    for j in range(ell + 2, len(err) + 1):
        if err[j - 1] >= c ** ell * err[j - ell - 2]:
            return j
    return 0


def rational_run(A, b, steps, poles=None, finite_poles=(), ell=3, c=0.75, lam_lo=None, lam_hi=None,
                 estimate=False, f=f_entropy, drop=1e-12):
    """psi_1..psi_steps of the rational Krylov method for one start vector b.
    poles: the pole of each of the steps - 1 steps (np.inf for infinity), or
    None for the switch rule with finite_poles, whose error bounds need the
    interval [lam_lo, lam_hi] (0 < lam_lo) holding A's spectrum on the Krylov
    space; estimate: the eq. (4.10) estimate instead of the upper bound.
    Returns dict(psi, switch (step of the switch, 0: none), basis (vectors
    built), poles (the pole each step used), err (the bounds of the
    polynomial steps up to the switch))."""
    from .bounds import posterior_bracket
    A = np.asarray(A, np.float64)
    n = A.shape[0]
    nb2 = float(np.dot(b, b))
    psi, used, errs = [], [], []
    if nb2 == 0.0:
        return dict(psi=[0.0] * steps, switch=0, basis=0, poles=[np.inf] * (steps - 1), err=[])
    V = [b / np.sqrt(nb2)]
    growing = True
    switched = 0
    for j in range(1, steps + 1):
        Vb = np.stack(V, axis=1)
        Am = 0.5 * ((Vb.T @ A @ Vb) + (Vb.T @ A @ Vb).T)
        th, U = np.linalg.eigh(Am)
        psi.append(float(nb2 * np.sum(U[0] ** 2 * f(th))))
        if j == steps:
            break
        # the polynomial direction: A v_j orthogonalized against V_j
        w = A @ V[-1]
        w0 = np.linalg.norm(w)
        wp = w.copy()
        for _ in range(2):
            wp = wp - Vb @ (Vb.T @ wp)
        keep = growing and np.linalg.norm(wp) > drop * w0
        if poles is not None:
            xi = poles[j - 1]
        else:
            if switched == 0:
                kk = Vb.shape[1]
                alpha = np.diag(Am).copy()
                beta = np.zeros(kk)
                beta[:kk - 1] = np.abs(np.diag(Am, -1))
                beta[kk - 1] = np.linalg.norm(wp) if keep else 0.0
                lo, hi, est = posterior_bracket(alpha, beta, kk, nb2, lam_lo, lam_hi)
                errs.append(est if estimate else hi)
                if switch_step(errs, ell, c) == j:
                    switched = j
            t = j - switched if switched else -1
            xi = finite_poles[t] if 0 <= t < len(finite_poles) else np.inf
        used.append(xi)
        if not growing:
            continue
        # the direction of the step's pole; one that keeps no more than drop
        # of its norm after the orthogonalization ends the basis
        if np.isfinite(xi):
            w = np.linalg.solve(np.eye(n) - A / xi, w)
            w0 = np.linalg.norm(w)
            for _ in range(2):
                w = w - Vb @ (Vb.T @ w)
        else:
            w = wp
        if not np.linalg.norm(w) > drop * w0:
            growing = False
            continue
        V.append(w / np.linalg.norm(w))
    return dict(psi=psi, switch=switched, basis=len(V), poles=used, err=errs)
