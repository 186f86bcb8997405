"""Adaptive Hutch++ (Section 3.2, the tail bound eq. (3.10); the adaptive
Hutch++ implementation of Section 5).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper runs the adaptive variant of Hutch++ of Persson, Cortinovis and
Kressner without printing it.  What the paper fixes: the target (eq. (3.10):
the estimate misses tr f(A) by eps_hat or more with probability at most
delta), the tolerance eps_hat ~ eps/2 tr f(A) for a relative target eps,
taken from a rough value of the trace, a smallest sketch of three products
with f(A), and that the algorithm picks N_r and N_H for the least effort,
counted as N_r products and N_r + N_H quadratic forms.  This module is a
reading of those facts, not that algorithm: parity unpinned against it.

* Rounds i = 0, 1, ...: sketch width N_r = r_first 2^i (at most r_max).
  Omega holds the first N_r Rademacher columns of the seed (nested across
  rounds), Q is an orthonormal basis of f(A) Omega (eq. (4.3)), and the
  round takes n_pilot deflated quadratic forms g^T (I - QQ^T) f(A)
  (I - QQ^T) g on Rademacher columns that do not depend on N_r (hash
  columns g_col0, g_col0 + 1, ...).
* Round estimate t = sum of the Q forms + mean of the deflated forms (eq.
  (3.9)); tolerance eps_hat = eps_abs, or eps/2 |t| for a relative target.
* Hutchinson count from a normal approximation of the deflated forms'
  mean: N_H = ceil((z s / eps_hat)^2) (the square capped at 1e15), s the
  forms' sample standard deviation, z the two-sided normal quantile of
  delta, and at least n_pilot.
* Effort 2 N_r + N_H.  A next round (width 2 N_r, at most r_max) runs
  only while it could still lower the least effort found so far: its
  effort is at least 2 N_r' + n_pilot.  The round of least effort is kept
  (the earlier on ties).  (Stopping at the first round whose effort rose
  instead would end on the noise of a 16-form standard deviation.)
* Final estimate: Hutch++ with the kept N_r and min(N_H, n_h_max) deflated
  forms, whose first n_pilot columns are the pilot's (when the count is the
  pilot's, the kept round itself); `capped` says that n_h_max cut the count
  (the target of eq. (3.10) is then not met by the rule).  `krylov_runs`
  counts the Krylov runs: 2 N_r + n_pilot per round (N_r products, N_r +
  n_pilot forms) and N_r + N_H forms for a final run, whose Q is the kept
  round's (an implementation keeps it; this module forms it again, the same
  Q).

Pinned by (tests/test_oracle_adaptive_hutchpp.py): the normal quantile
against its textbook values, the count and round rules on hand-worked
cases, a single round against plain Hutch++ on the same columns, a matrix
whose f(A) has rank 10 (the rule must keep a sketch of 12 and return the
exact trace), and the coverage of eq. (3.10) over many seeds on a small
graph with a diagonalised exact value.
"""
import math

import numpy as np

from .estimators import hutchpp
from .lanczos import breakdown_tau
from .probes import rademacher_block


def normal_quantile_two_sided(delta):
    """z with P(|N(0, 1)| >= z) = delta."""
    from scipy.stats import norm
    return float(norm.isf(delta / 2.0))


def hutch_count(s, eps_hat, z, n_pilot):
    """Deflated forms a round asks for (the normal-approximation rule)."""
    if s <= 0.0:
        return int(n_pilot)
    x = (z * s / eps_hat) ** 2 if eps_hat > 0.0 else 1e15
    return int(max(math.ceil(min(x, 1e15)), n_pilot))


def kept_round(efforts):
    """Index of the round of least effort among those run (earliest on ties)."""
    return min(range(len(efforts)), key=lambda i: (efforts[i], i))


def _run(A, node_ids, seed, nr, g_col0, nh, k, tau, desing):
    Om = rademacher_block(seed, node_ids, np.arange(nr))
    G = rademacher_block(seed, node_ids, np.arange(g_col0, g_col0 + nh))
    est, det = hutchpp(A, Om, G, k, tau, desing)
    return est, np.asarray(det["psi"])


def run_rule(round_stats, eps=1e-2, eps_abs=0.0, delta=1e-2, n_pilot=16, r_first=3, r_max=96, n_h_max=4096):
    """The rule's decisions from the rounds' statistics: round_stats(nr)
    returns (estimate, sd) of the round of sketch width nr.  Returns
    dict(rounds=[dict(nr, estimate, sd, eps_hat, nh, effort)], kept,
    n_hutch, capped, reuse, krylov_runs); reuse: the final run is the kept
    round itself."""
    z = normal_quantile_two_sided(delta)
    rounds = []
    nr = r_first
    while True:
        est, sd = round_stats(nr)
        eh = eps_abs if eps_abs > 0 else 0.5 * eps * abs(est)
        nh = hutch_count(sd, eh, z, n_pilot)
        rounds.append(dict(nr=nr, estimate=est, sd=sd, eps_hat=eh, nh=nh, effort=2 * nr + nh))
        nxt = min(2 * nr, r_max)
        if nr >= r_max or 2 * nxt + n_pilot >= min(r["effort"] for r in rounds):
            break
        nr = nxt
    ib = kept_round([r["effort"] for r in rounds])
    nh = min(rounds[ib]["nh"], n_h_max)
    reuse = nh == n_pilot
    runs = sum(2 * r["nr"] + n_pilot for r in rounds) + (0 if reuse else rounds[ib]["nr"] + nh)
    return dict(rounds=rounds, kept=ib, n_hutch=nh, capped=rounds[ib]["nh"] > n_h_max, reuse=reuse,
                krylov_runs=runs)


def adaptive_hutchpp(A, node_ids, seed, k, eps=1e-2, eps_abs=0.0, delta=1e-2, n_pilot=16, r_first=3,
                     r_max=96, n_h_max=4096, g_col0=128, fp64_tau=True, desing=True):
    """Adaptive Hutch++ estimate of tr f(A) by the reading above.

    Returns dict(estimate, n_sketch, n_hutch, std_error, eps_hat, capped,
    krylov_runs, rounds=[dict(nr, estimate, sd, eps_hat, nh, effort)], psi)."""
    tau = breakdown_tau(fp64_tau)
    runs = {}

    def round_stats(nr):
        est, psi = _run(A, node_ids, seed, nr, g_col0, n_pilot, k, tau, desing)
        runs[nr] = (est, psi)
        return est, float(np.std(psi[nr:], ddof=1))

    rule = run_rule(round_stats, eps, eps_abs, delta, n_pilot, r_first, r_max, n_h_max)
    best = rule["rounds"][rule["kept"]]
    nr, nh = best["nr"], rule["n_hutch"]
    if rule["reuse"]:
        est, psi = runs[nr]
    else:
        est, psi = _run(A, node_ids, seed, nr, g_col0, nh, k, tau, desing)
    q = psi[nr:]
    return dict(estimate=est, n_sketch=nr, n_hutch=nh, std_error=float(np.std(q, ddof=1) / math.sqrt(nh)),
                eps_hat=best["eps_hat"], capped=rule["capped"], krylov_runs=rule["krylov_runs"],
                rounds=rule["rounds"], psi=psi)
