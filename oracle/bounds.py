"""A-priori and a-posteriori error bounds used as test assertions.

* thm22: Theorem 2.2 as stated, bound on the best uniform polynomial
  approximation error E_k(x log x, [a, b]) for k >= 2 with gamma = a / b.
* thm22_proof: the value the proof of Theorem 2.2 actually establishes.  The
  proof reduces E_k to b / (2 (1-gamma)^(k-1)) times an integral whose closed
  form is (1-sqrt(gamma))^(2k) (1+gamma+2k sqrt(gamma)) / (2 (k^2-1)); the last
  display of the printed proof shows twice that.  Carried through, the bound is
  b (1-gamma) (1+gamma+2k sqrt(gamma)) / (4 (k^2-1)) rho^k, rho =
  (1-sqrt(gamma)) / (1+sqrt(gamma)), which exceeds the stated form by the
  factor 1 + sqrt(gamma) (the two agree for gamma = 0, Remark 2.3).  Assertions
  that must be rigorous use thm22_proof; tests check both against a minimax
  linear program and thm22_proof against numerical quadrature of the integral.
* rem23: Remark 2.3, the gamma = 0 case b / (4 (k^2 - 1)).
* cor32: Corollary 3.2, |S(A) - T_d| bound for a distance-d colouring (d >= 2).
* prop44_poly: Proposition 4.4 in the polynomial case (q = 1):
  |psi - psi_k| <= 2 ||b||^2 E_{2k-1}(f, [lambda_min, lambda_max]), bounded
  with thm22_proof at degree 2k - 1.
* g_m and the a-posteriori bracket of Theorem 4.8 for the polynomial Krylov
  method (K_m = I, h_{m+1} = beta_m e_m), and the geometric-mean estimate
  (4.10) of Example 4.10; g_m_entropy evaluates eq. (4.8) for -x log x with
  divided differences free of cancellation near the Ritz values (pinned
  against the generic g_m away from them and against its own limits);
  g_m_resolvent evaluates the same g_m through its residue form (pinned
  against eq. (4.8) written out in 60-digit arithmetic and against an
  adaptive quadrature of the same integral), which the bracket uses.

Pinned by: thm22 against the integral of its proof; every bound checked to
hold on exact errors computed by diagonalization (tests).
"""
import numpy as np
from scipy import integrate

from .entropy import f_entropy


def thm22(k, a, b):
    k = np.asarray(k, np.float64)
    g = a / b
    sg = np.sqrt(g)
    return b * (1 - sg) * (1 + g + 2 * k * sg) / (4 * (k * k - 1)) * ((1 - sg) / (1 + sg)) ** k


def thm22_proof(k, a, b):
    k = np.asarray(k, np.float64)
    g = a / b
    sg = np.sqrt(g)
    return b * (1 - g) * (1 + g + 2 * k * sg) / (4 * (k * k - 1)) * ((1 - sg) / (1 + sg)) ** k


def thm22_integral(k, a, b):
    """b / (2 (1-gamma)^(k-1)) * int_0^inf (sqrt(1+t) - sqrt(gamma+t))^(2k) dt,
    the quantity the proof of Theorem 2.2 bounds in closed form."""
    g = a / b

    def integrand(t):
        # sqrt(1+t) - sqrt(g+t) = (1-g) / (sqrt(1+t) + sqrt(g+t)), cancellation-free
        return ((1 - g) / (np.sqrt(1 + t) + np.sqrt(g + t))) ** (2 * k)

    val, _ = integrate.quad(integrand, 0, np.inf, limit=400, epsabs=0, epsrel=1e-12)
    return b * val / (2 * (1 - g) ** (k - 1))


def rem23(k, b):
    k = np.asarray(k, np.float64)
    return b / (4 * (k * k - 1))


def cor32(d, n, a, b):
    """Corollary 3.2 (2 n E_d with Theorem 2.2 as stated)."""
    d = np.asarray(d, np.float64)
    g = a / b
    sg = np.sqrt(g)
    return n * b * (1 - sg) * (1 + g + 2 * d * sg) / (2 * (d * d - 1)) * ((1 - sg) / (1 + sg)) ** d


def prop44_poly(k, norm2, a, b):
    """Bound on |psi - psi_k| after k polynomial Krylov steps (k >= 2)."""
    return 2 * norm2 * thm22_proof(2 * k - 1, a, b)


def _fprime(x):
    return -np.log(x) - 1.0


def _fsecond(x):
    return -1.0 / x


def g_m(z, theta, U, beta_m, f=f_entropy, fp=_fprime, fpp=_fsecond):
    """eq. (4.8) for the polynomial Krylov method, for f = -x log x.

    T_m = U diag(theta) U^T; K_m = I and h_{m+1}^T = beta_m e_m^T, so the
    coefficients are a*_j = beta_m U[m-1, j], b*_j = U[0, j] and
    c*_j = sum_{l != j} a*_l b*_l / (theta_j - theta_l).
    """
    z = np.atleast_1d(np.asarray(z, np.float64))
    a = beta_m * U[-1, :]
    bb = U[0, :]
    ab = a * bb
    diff = theta[:, None] - theta[None, :]
    np.fill_diagonal(diff, np.inf)
    c = (ab[None, :] / diff).sum(axis=1)
    out = np.zeros_like(z)
    fth = f(theta)
    for j in range(theta.size):
        dz = z - theta[j]
        near = np.abs(dz) <= 1e-12 * max(1.0, abs(theta[j]))
        term = np.empty_like(z)
        zz = z[~near]
        d = dz[~near]
        term[~near] = (ab[j] ** 2 * ((f(zz) - fth[j]) / d ** 2 - fp(theta[j]) / d)
                       + 2 * ab[j] * c[j] * (f(zz) - fth[j]) / d)
        term[near] = 0.5 * ab[j] ** 2 * fpp(theta[j]) + 2 * ab[j] * c[j] * fp(theta[j])
        out += term
    return out


def entropy_divided_differences(z, theta):
    """D1 = (f(z) - f(theta)) / (z - theta) and
    D2 = (D1 - f'(theta)) / (z - theta) for f(x) = -x log x, z, theta > 0,
    with their limits f'(theta) and f''(theta) / 2 at z = theta (the limits
    eq. (4.8) takes).  Written with r = z / theta, t = r - 1:
    f(z) - f(theta) = -theta (t log theta + r log r), so
    D1 = -log theta - (1 + t) log1p(t) / t and D2 = q(t) / theta,
    q(t) = (t - (1 + t) log1p(t)) / t^2; both by their Taylor series for
    |t| < 1e-3, where the quotients would cancel."""
    z = np.asarray(z, np.float64)
    t = z / theta - 1.0
    small = np.abs(t) < 1e-3
    ts = np.where(small, 1.0, t)
    l1 = np.log1p(ts)
    h = np.where(small, 1.0 + t / 2 - t * t / 6 + t ** 3 / 12 - t ** 4 / 20, (1.0 + ts) * l1 / ts)
    q = np.where(small, -0.5 + t / 6 - t * t / 12 + t ** 3 / 20 - t ** 4 / 30, (ts - (1.0 + ts) * l1) / (ts * ts))
    return -np.log(theta) - h, q / theta


def g_m_entropy(z, theta, U, beta_m, theta_floor):
    """eq. (4.8) for f = -x log x in the polynomial case, evaluated with the
    cancellation-free divided differences above.  Ritz values below
    theta_floor (rounding-level ones, possible only along a null direction)
    are raised to it."""
    z = np.atleast_1d(np.asarray(z, np.float64))
    a = beta_m * U[-1, :]
    bb = U[0, :]
    ab = a * bb
    diff = theta[:, None] - theta[None, :]
    np.fill_diagonal(diff, np.inf)
    c = (ab[None, :] / diff).sum(axis=1)
    th = np.maximum(theta, theta_floor)
    out = np.zeros_like(z)
    for j in range(theta.size):
        d1, d2 = entropy_divided_differences(z, th[j])
        out += ab[j] ** 2 * d2 + 2 * ab[j] * c[j] * d1
    return out


def corner_resolvent_sq(alpha, beta, m, t):
    """(e_1^T (T_m + t I)^{-1} e_m)^2 for an array of t >= 0 with T_m + t I
    positive definite: the corner entry of the inverse of a symmetric
    tridiagonal matrix is (-1)^(m-1) prod_{i<m} beta_i / det(T_m + t I), and
    det = prod of the pivots p_1 = alpha_1 + t, p_{i+1} = alpha_{i+1} + t -
    beta_i^2 / p_i (kept in logarithms against overflow)."""
    t = np.asarray(t, np.float64)
    p = alpha[0] + t
    logsq = np.zeros_like(t)
    for i in range(1, m):
        logsq += 2.0 * (np.log(np.abs(beta[i - 1])) - np.log(p))
        p = alpha[i] + t - beta[i - 1] ** 2 / p
    logsq -= 2.0 * np.log(p)
    return np.exp(logsq)


def g_m_resolvent(z, alpha, beta, m, nodes_per_unit=20, span=60.0):
    """g_m(z) of eq. (4.8) for f = -x log x, through its residue form.

    With h(w) = sum_j a_j b_j / (w - theta_j) = beta_m e_1^T (w I - T_m)^{-1}
    e_m, the terms of eq. (4.8) are the residues of f(w) h(w)^2 / (w - z) at
    the Ritz values (double poles: the D2 terms; cross terms of h^2: the c_j
    D1 terms) and at z.  Writing -x log x = int_0^inf x (1 - x) / ((x + t)(1
    + t)) dt (x > 0), each integrand x (1 - x) h(x)^2 / ((x + t)(1 + t)(x -
    z)) is rational with residues summing to zero (it decays like x^-2), so
    the residues above sum to minus the one at x = -t:
        g_m(z) = - int_0^inf t h(-t)^2 / (t + z) dt,
        h(-t)^2 = beta_m^2 (e_1^T (T_m + t I)^{-1} e_m)^2.
    Valid when T_m is positive definite.  The integral is taken in s = ln t
    by the trapezoidal rule, nodes_per_unit points per unit of s over
    [ln(sigma) - span, ln(sigma) + span], sigma the largest |alpha|.
    Consequences used by posterior_bracket: g_m < 0, and |g_m| decreases in
    z (the integrand does)."""
    z = np.atleast_1d(np.asarray(z, np.float64))
    a = np.asarray(alpha[:m], np.float64)
    b = np.asarray(beta[:m], np.float64)
    sigma = float(np.max(np.abs(a)))
    s = np.linspace(np.log(sigma) - span, np.log(sigma) + span, int(2 * span * nodes_per_unit) + 1)
    ds = s[1] - s[0]
    t = np.exp(s)
    h2 = b[m - 1] ** 2 * corner_resolvent_sq(a, b, m, t)
    w = np.full(t.size, ds)
    w[0] = w[-1] = 0.5 * ds
    return np.array([-np.sum(w * t * t * h2 / (t + zz)) for zz in z])


def posterior_bracket(alpha, beta, m, norm2, lam_min, lam_max, grid=2000):
    """Theorem 4.8: (lower, upper) bounds on |psi - psi_m| and the estimate
    (4.10), the extremes of |g_m| over [lam_min, lam_max] (lam_min > 0).

    When T_m is positive definite, g_m comes from its residue form
    (g_m_resolvent): |g_m| decreases in z, so the extremes are its values at
    the ends of the interval.  (Eq. (4.8) evaluated term by term in double
    precision loses accuracy to cancellation as m grows: 7e-7 at m = 25 and
    4e-2 at m = 39 against a 60-digit evaluation on a graph Laplacian, where
    the residue form stays within 2e-12.)  Otherwise (a Ritz value <= 0
    from rounding) eq. (4.8) is evaluated term by term on a log-spaced grid of
    grid points plus the Ritz values inside the interval, Ritz values below
    lam_min raised to it."""
    from scipy.linalg import eigh_tridiagonal
    theta, U = eigh_tridiagonal(alpha[:m], beta[:m - 1])
    if theta.min() > 0.0:
        g = np.abs(g_m_resolvent(np.array([lam_min, lam_max]), alpha, beta, m))
        lo, hi = norm2 * g[1], norm2 * g[0]
        return lo, hi, np.sqrt(lo * hi)
    z = np.geomspace(lam_min, lam_max, grid)
    z = np.concatenate([z, theta[(theta > lam_min) & (theta < lam_max)]])
    g = np.abs(g_m_entropy(z, theta, U, beta[m - 1], lam_min))
    lo, hi = norm2 * g.min(), norm2 * g.max()
    return lo, hi, np.sqrt(lo * hi)
