"""Probing method for S(A) with a relative accuracy target (Section 5,
probing method implementation; Algorithm 2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* fit_heuristic(T1, T2, T3): the error model of eq. (5.1),
  |tr f(A) - T_d| ~ C q^d / d^kappa, fitted for kappa = 2 and kappa = 3 from
  the consecutive differences e_d = |T_{d+1} - T_d|, d = 1, 2, taken as the
  errors of T_1 and T_2: e_1 = C q and e_2 = C q^2 / 2^kappa, so
  q = 2^kappa e_2 / e_1 and C = e_1 / q.
* heuristic_error(d, fits): the larger of the two model values at d (the
  paper keeps the maximum of the kappa = 2 and kappa = 3 estimates).  The
  model value is written e_1 q^(d-1) / d^kappa, which equals C q^d / d^kappa
  and stays defined at q = 0.
* bound_d(n, b, eps_hat, d_max): the smallest d >= 2 for which Corollary
  3.2's bound with a = 0, n b / (2 (d^2 - 1)), is within eps_hat (d_max,
  flagged capped, when none up to d_max is).
* select_d(T, eps_hat, n, b, d_max): the smallest d >= 1 whose heuristic
  error is within eps_hat; the bound's d when the fit has no decay (q >= 1
  for either kappa, or e_1 = 0 < e_2).  Both T_d differences zero: d = 1.
* adaptive_quadforms: psi_l ~ v_l^T f(A) v_l by Lanczos and Gauss quadrature
  (eq. (4.2)) stopped, column by column, at the first check step m (m = 3, 5,
  7, ...) where the stopping quantity is within that column's tolerance; a
  column that never meets it ends at k_max.  The quantity is the upper bound
  of Theorem 4.8, eq. (4.9) (rule="bound"), or the geometric mean of the
  lower and upper bounds, eq. (4.10) (rule="estimate": a heuristic with no
  guarantee, Remark 4.11).  The bounds are the polynomial-case g_m of
  eq. (4.8) over [lam_lo, lam_hi].
* probing_entropy: Algorithm 2.  Readings where the paper leaves a choice:
  - the rough entropy of Remark 5.1 is S0 = -log tr(A^2) (a lower bound of S
    for a density matrix) while T_1..T_3 are computed, then
    S_hat = max(S0, T_1, T_2, T_3): for an M-matrix every T_d is a lower bound
    of S (Proposition 3.6), so S_hat stays a lower bound up to the Krylov
    error, and eps_hat = eps S_hat / 2 never exceeds the split of Remark 5.2;
  - per-column Krylov tolerance eps_hat |V_l| / n (eq. (5.3)); T_1..T_3 use
    eps_hat0 = eps S0 / 2, which is no larger;
  - when the selected d is 1, 2 or 3 its preprocessing run is the result;
  - the Krylov method is the polynomial one (every pole at infinity) and the
    stopping rule the upper bound of Theorem 4.8 on the interval
    [lam_lo, lam_hi] given by the caller;
  - Corollary 3.2 is applied with a = 0 (a graph Laplacian is singular) and
    b the caller's upper bound of lambda_max.

Pinned by: the fit recovering (C, q) from sequences that follow the model
exactly and the selected d being the first at which the generating model
meets the target; the bound's d against Corollary 3.2 as evaluated by
``bounds.cor32``; every adaptive quadratic form within its tolerance of the
exact one (dense eigendecomposition); T_d <= S for graph Laplacians
(Proposition 3.6); the whole estimate within eps S of the exact entropy on
small graphs (tests).
"""
import numpy as np

from .coloring import greedy_distance_coloring
from .lanczos import lanczos
from .probes import desingularize, indicator_block
from .quadrature import gauss_quadrature
from .bounds import posterior_bracket

KAPPAS = (2, 3)


def fit_heuristic(T1, T2, T3):
    """[(kappa, e1, q)] for kappa = 2, 3; q is None when e1 = 0 (no fit)."""
    e1 = abs(T2 - T1)
    e2 = abs(T3 - T2)
    fits = []
    for kappa in KAPPAS:
        q = (2.0 ** kappa) * e2 / e1 if e1 > 0 else None
        fits.append((kappa, e1, q))
    return fits


def heuristic_error(d, fits):
    return max(e1 * q ** (d - 1) / float(d) ** kappa for kappa, e1, q in fits)


def bound_d(n, b, eps_hat, d_max):
    """Smallest d in [2, d_max] with n b / (2 (d^2 - 1)) <= eps_hat, else d_max
    (with capped=True).  Corollary 3.2 covers d >= 2 only: with d_max = 1 the
    result is d = 1, capped."""
    for d in range(2, d_max + 1):
        if n * b / (2.0 * (d * d - 1)) <= eps_hat:
            return d, False
    return d_max, True


def select_d(T, eps_hat, n, b, d_max):
    """Returns (d, fits, fallback, capped)."""
    T1, T2, T3 = T
    fits = fit_heuristic(T1, T2, T3)
    e1 = fits[0][1]
    e2 = abs(T3 - T2)
    if e1 == 0 and e2 == 0:
        return 1, fits, False, False
    if e1 == 0 or any(q >= 1.0 for _, _, q in fits):
        d, capped = bound_d(n, b, eps_hat, d_max)
        return d, fits, True, capped
    for d in range(1, d_max + 1):
        if heuristic_error(d, fits) <= eps_hat:
            return d, fits, False, False
    return d_max, fits, False, True


def adaptive_quadforms(A, B, k_max, tau, tol, lam_lo, lam_hi, grid=256, desing=True, rule="bound"):
    """psi[c] at the first check step whose stopping quantity (Theorem 4.8's
    upper bound, or the eq. (4.10) estimate) is within tol[c]; returns (psi,
    steps, converged, lanczos result)."""
    if rule not in ("bound", "estimate"):
        raise ValueError("rule must be 'bound' or 'estimate'")
    C = desingularize(B) if desing else np.asarray(B, np.float64)
    res = lanczos(A, C, k_max, tau)
    m = C.shape[1]
    steps = np.full(m, k_max, np.int64)
    converged = np.zeros(m, bool)
    for c in range(m):
        for s in range(3, k_max + 1, 2):
            mm = min(int(res["k_eff"][c]), s)
            if mm <= 0 or res["beta"][c, mm - 1] == 0.0:
                q = 0.0                        # invariant Krylov space: exact
            else:
                lo, hi, _ = posterior_bracket(res["alpha"][c], res["beta"][c], mm, res["norm2"][c],
                                              lam_lo, lam_hi, grid=grid)
                q = hi if rule == "bound" else np.sqrt(lo * hi)
            if q <= tol[c]:
                steps[c] = s
                converged[c] = True
                break
    k_use = np.minimum(res["k_eff"], steps)
    psi = gauss_quadrature(res["alpha"], res["beta"], k_use, res["norm2"])
    return psi, steps, converged, res


def probing_run(A, row_ptr, col_idx, d, eps_hat, k_max, tau, lam_lo, lam_hi, grid=256, desing=True,
                rule="bound"):
    """One distance-d probing pass with the tolerances of eq. (5.3)."""
    n = A.shape[0]
    colors, s = greedy_distance_coloring(row_ptr, col_idx, n, d)
    sizes = np.bincount(colors, minlength=s).astype(np.float64)
    tol = eps_hat * sizes / n
    psi, steps, conv, _ = adaptive_quadforms(A, indicator_block(colors, s), k_max, tau, tol, lam_lo, lam_hi,
                                             grid, desing, rule)
    return dict(d=d, colors=colors, n_colors=s, psi=psi, steps=steps, converged=conv, tol=tol,
                T=float(np.sum(psi)))


def probing_entropy(g, eps, d_max=12, k_max=128, tau=None, lam_lo_fraction=1e-12, grid=256,
                    select="heuristic", desing=True, stop="bound"):
    """Algorithm 2 on a GraphCSR density matrix g (A = g.scipy()); stop is the
    Krylov stopping rule of step 3 ("bound", eq. (4.9); "estimate",
    eq. (4.10))."""
    from .lanczos import breakdown_tau
    if tau is None:
        tau = breakdown_tau(False)
    A = g.scipy()
    n = g.n
    lam_hi = float(np.abs(A).sum(axis=1).max())          # Gershgorin bound of lambda_max
    lam_lo = lam_lo_fraction * lam_hi
    s0 = float(-np.log(np.sum(A.data ** 2)))             # -log tr(A^2), A symmetric
    eps_hat0 = 0.5 * eps * s0
    runs = {}
    out = dict(s0=s0, lam_hi=lam_hi)
    if select == "heuristic":
        for d in (1, 2, 3):
            runs[d] = probing_run(A, g.row_ptr, g.col_idx, d, eps_hat0, k_max, tau, lam_lo, lam_hi, grid, desing,
                                  stop)
        T = tuple(runs[d]["T"] for d in (1, 2, 3))
        s_hat = max(s0, *T)
        eps_hat = 0.5 * eps * s_hat
        d, fits, fallback, capped = select_d(T, eps_hat, n, lam_hi, d_max)
        out.update(T_pre=T, fits=fits)
    elif select == "bound":
        s_hat, eps_hat = s0, eps_hat0
        d, capped = bound_d(n, lam_hi, eps_hat, d_max)
        fallback = True
    else:
        raise ValueError("select must be 'heuristic' or 'bound'")
    final = runs.get(d)
    if final is None:
        final = probing_run(A, g.row_ptr, g.col_idx, d, eps_hat, k_max, tau, lam_lo, lam_hi, grid, desing, stop)
    out.update(estimate=final["T"], d=d, s_hat=s_hat, eps_hat=eps_hat, fallback=fallback, capped=capped,
               final=final, runs=runs)
    return out
