"""Pins of the rational Krylov cross-check (eq. (4.1), (4.2), Lemma 4.3)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import rational


def _setup():
    g = oracle.laplacian_from_edges(*synth.barabasi_albert(120, 2, 3))
    rho = oracle.dense_matrix(g)
    lam = np.linalg.eigvalsh(rho)
    rng = np.random.default_rng(0)
    c = oracle.desingularize(rng.standard_normal((g.n, 1)))[:, 0]
    return rho, lam, c


def test_all_poles_infinite_equals_lanczos():
    rho, lam, c = _setup()
    for m in (3, 6, 10):
        psi, _ = rational.rational_quadform(rho, c, [np.inf] * (m - 1))
        res = oracle.lanczos_full_reorth(rho, c[:, None], m, oracle.breakdown_tau(True))
        q = oracle.gauss_quadrature(res["alpha"], res["beta"], res["k_eff"], res["norm2"])[0]
        assert abs(psi - q) < 1e-12 * abs(q)


def test_lemma_4_3_rational_exactness():
    rho, lam, c = _setup()
    m = 5
    poles = rational.default_poles(m, 2, lam[1], lam[-1])
    V = rational.rational_basis(rho, c, poles)
    Am = V.T @ rho @ V
    q = np.prod([1 - lam / xi if np.isfinite(xi) else np.ones_like(lam) for xi in poles], axis=0)
    th, U = np.linalg.eigh(0.5 * (Am + Am.T))
    qth = np.prod([1 - th / xi if np.isfinite(xi) else np.ones_like(th) for xi in poles], axis=0)
    lam_all, W = np.linalg.eigh(rho)
    proj = (W.T @ c) ** 2
    qa = np.prod([1 - lam_all / xi if np.isfinite(xi) else np.ones_like(lam_all) for xi in poles], axis=0)
    for p in range(2 * m):
        exact = np.sum(proj * lam_all ** p / qa ** 2)
        approx = np.dot(c, c) * np.sum(U[0] ** 2 * th ** p / qth ** 2)
        assert abs(approx - exact) < 1e-9 * abs(exact), p


def test_rational_converges_to_exact():
    rho, lam, c = _setup()
    exact = oracle.exact_quadform(rho, c[:, None])[0]
    errs = []
    for m in (4, 8, 16):
        psi, _ = rational.rational_quadform(rho, c, rational.default_poles(m, 2, lam[1], lam[-1]))
        errs.append(abs(psi - exact) / abs(exact))
    assert errs[-1] < 1e-8 and errs[-1] < errs[0]


def test_switch_step_on_geometric_errors():
    # err_j = r^j: err_j / err_(j-ell-1) = r^(ell+1), so the rule fires at
    # the first checked step j = ell + 2 exactly when r^(ell+1) >= c^ell
    for r, want in ((0.81, 5), (0.8, 0), (0.9, 5), (0.3, 0)):
        err = [r ** j for j in range(1, 30)]
        assert rational.switch_step(err, 3, 0.75) == want, r
    # equality (powers of two, exact in binary): r^(ell+1) = c^ell fires
    assert rational.switch_step([0.5 ** j for j in range(1, 10)], 1, 0.25) == 3
    assert rational.switch_step([0.125 ** j for j in range(1, 10)], 3, 0.0625) == 5
    assert rational.switch_step([1.0, 0.5, 0.25, 0.125], 3, 0.75) == 0          # too short to check
    # by hand, ell = 3, c^3 = 0.421875: e5/e1 = 0.1, e6/e2 = 0.18, e7/e3 = 0.34,
    # e8/e4 = 0.48, so the rule fires at j = 8
    err = [1.0, 0.5, 0.25, 0.125, 0.1, 0.09, 0.085, 0.06, 0.05]
    assert rational.switch_step(err, 3, 0.75) == 8
    # ell = 1, c = 0.5: e3/e1 = 0.25, e4/e2 = 0.25, e5/e3 = 0.4, e6/e4 = 0.72
    assert rational.switch_step(err, 1, 0.5) == 6


def test_stepwise_run_matches_the_one_shot_form():
    rho, lam, c = _setup()
    steps = 9
    poles = rational.default_poles(steps, 3, lam[1], lam[-1])
    run = rational.rational_run(rho, c, steps, poles=poles)
    for j in range(1, steps + 1):
        q, _ = rational.rational_quadform(rho, c, poles[: j - 1])
        assert abs(run["psi"][j - 1] - q) < 1e-12 * abs(q), j
    assert run["basis"] == steps and run["poles"] == poles


@pytest.mark.parametrize("estimate", [False, True])
def test_switch_rule_run_on_an_ill_conditioned_path(estimate):
    n, e = synth.path_graph(300)
    A = oracle.laplacian_from_edges(n, e).scipy().toarray()
    lam = np.linalg.eigvalsh(A)
    lo, hi = 0.999 * lam[1], 1.001 * lam[-1]
    b = oracle.rademacher_block(5, np.arange(n), np.arange(1))[:, 0]
    c = oracle.desingularize(b[:, None])[:, 0]
    exact = float(oracle.exact_quadform(A, c)[0])
    steps = 24
    fin = list(-np.geomspace(lam[-1], lam[1], 12))
    run = rational.rational_run(A, c, steps, finite_poles=fin, ell=3, c=0.75, lam_lo=lo, lam_hi=hi,
                                estimate=estimate)
    s = run["switch"]
    # Lanczos on a path graph stalls early: the rule fires, at the step that
    # the rule gives on the run's own bounds
    assert 5 <= s < steps and len(run["err"]) == s
    assert rational.switch_step(run["err"], 3, 0.75) == s
    # the bounds are Theorem 4.8's (eq. (4.9), or (4.10)) on the Lanczos
    # coefficients of the same start vector: the polynomial phase spans the
    # same Krylov spaces
    res = oracle.lanczos_full_reorth(A, c[:, None], s + 1, oracle.breakdown_tau(True))
    for j in range(1, s + 1):
        blo, bhi, best = oracle.bounds.posterior_bracket(res["alpha"][0], res["beta"][0], j, res["norm2"][0], lo, hi)
        want = best if estimate else bhi
        assert abs(run["err"][j - 1] - want) <= 1e-6 * want, j
    # poles: infinity before the switch, then (from the switch step on) the
    # finite list in order, then infinity again past its end
    k = min(len(fin), steps - s)
    assert run["poles"] == [np.inf] * (s - 1) + fin[:k] + [np.inf] * (steps - s - k)
    # the same basis rebuilt in one shot from those poles gives the same form
    q, _ = rational.rational_quadform(A, c, run["poles"])
    assert abs(q - run["psi"][-1]) < 1e-11 * abs(q)
    # and the finite poles beat poles at infinity at the same dimension
    poly, _ = rational.rational_quadform(A, c, [np.inf] * (steps - 1))
    assert abs(run["psi"][-1] - exact) < 0.1 * abs(poly - exact)


def test_invariant_subspace_stops_the_basis():
    g = oracle.laplacian_from_edges(*synth.path_graph(6))
    rho = oracle.dense_matrix(g)
    c = oracle.desingularize(np.arange(6, dtype=np.float64)[:, None] ** 2)[:, 0]
    exact = float(oracle.exact_quadform(rho, c)[0])
    run = rational.rational_run(rho, c, 10, poles=[np.inf] * 9)
    # the centred vector lives in the 5-dimensional range of the Laplacian
    assert run["basis"] == 5
    assert all(abs(p - exact) < 1e-12 * abs(exact) for p in run["psi"][4:])
    zero = rational.rational_run(rho, np.zeros(6), 4, poles=[np.inf] * 3)
    assert zero["psi"] == [0.0] * 4 and zero["basis"] == 0
