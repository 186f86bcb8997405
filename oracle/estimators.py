"""Trace estimators built from quadratic forms (paper Section 3).

* quadforms: psi_j ~ b_j^T f(A) b_j for each column of a probe block, by
  optional implicit desingularization (Remark 4.6), plain Lanczos and Gauss
  quadrature (eq. (4.2)).
* hutchinson: (1/N) sum psi_j (eq. (3.8)).
* probing_sum: T_d = sum over colours of psi_l (eq. (3.2)).
* hutchpp: tr(Q^T B Q) + Hutchinson on (I - QQ^T) B (I - QQ^T) with Q an
  orthonormal basis of range(B Omega) (eq. (3.9)); B Omega is approximated
  column by column with f(A) b ~ ||b|| V_k f(T_k) e_1 (eq. (4.3)).  The
  orthonormal basis comes from numpy's Householder QR; the projected test
  vectors are G - Q (Q^T G), which gives (I - QQ^T) B (I - QQ^T) the same
  quadratic forms.  The basis V_k is not stored: a second pass repeats the
  identical recurrence and accumulates the combination.

Pinned by: Hutchinson mean over many seeds within its confidence interval of
the exact entropy, probing with one colour per node being exact, Hutch++ with
N_r = n being exact (tests).
"""
import numpy as np

from .lanczos import lanczos
from .probes import desingularize
from .quadrature import gauss_quadrature, f_of_T_e1


def quadforms(A, B, k, tau, desing=True):
    C = desingularize(B) if desing else np.asarray(B, np.float64)
    res = lanczos(A, C, k, tau)
    res["psi"] = gauss_quadrature(res["alpha"], res["beta"], res["k_eff"], res["norm2"])
    return res


def hutchinson(psi):
    return float(np.mean(psi))


def probing_sum(psi):
    return float(np.sum(psi))


def f_times_block(A, B, k, tau, desing=True):
    """Y[:, j] ~ f(A) b_j by eq. (4.3), with the basis regenerated in a second
    pass of the same recurrence instead of being stored."""
    C = desingularize(B) if desing else np.asarray(B, np.float64)
    res = lanczos(A, C, k, tau)
    n, m = C.shape
    S = np.zeros((m, k))
    for c in range(m):
        ke = int(res["k_eff"][c])
        S[c, :ke] = f_of_T_e1(res["alpha"][c], res["beta"][c], ke)
    # second pass: identical recurrence, accumulating sum_j s_j v_j
    norm2 = res["norm2"]
    active = norm2 > 0
    v = np.zeros((n, m))
    v[:, active] = C[:, active] / np.sqrt(norm2[active])
    v_prev = np.zeros((n, m))
    Y = np.zeros((n, m))
    for j in range(k):
        live = res["k_eff"] > j
        if not live.any():
            break
        Y[:, live] += S[live, j][None, :] * v[:, live]
        a = res["alpha"][:, j]
        b = res["beta"][:, j]
        b_prev = res["beta"][:, j - 1] if j > 0 else np.zeros(m)
        w = np.asarray(A @ v, np.float64) - b_prev[None, :] * v_prev
        w = w - a[None, :] * v
        v_prev = v
        v = np.zeros((n, m))
        ok = live & (b > 0)
        v[:, ok] = w[:, ok] / b[ok]
    Y *= np.sqrt(norm2)[None, :]
    return Y, res


def hutchpp(A, Omega, G, k, tau, desing=True):
    """Hutch++ estimate of tr f(A) (eq. (3.9)).  Returns (estimate, detail)."""
    Y, sketch = f_times_block(A, Omega, k, tau, desing)
    Q, _ = np.linalg.qr(Y)
    Gt = np.asarray(G, np.float64) - Q @ (Q.T @ np.asarray(G, np.float64))
    block = np.concatenate([Q, Gt], axis=1)
    res = quadforms(A, block, k, tau, desing)
    nr = Q.shape[1]
    psi = res["psi"]
    est = float(np.sum(psi[:nr]) + (np.mean(psi[nr:]) if psi.size > nr else 0.0))
    return est, dict(Y=Y, Q=Q, Gt=Gt, psi=psi, quad=res, sketch=sketch)
