"""Host logic of the serving loop (no GPU): the arena allocator and the error
rule, through the C++ sources and through the library's exported planner,
pinned against the oracle's bound functions and against exact quadratic
forms on small graphs."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
import paper_2212_09642_amd as vne

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_arena_and_rule_host_program(tmp_path):
    exe = str(tmp_path / "test_serve_host")
    csrc = os.path.join(ROOT, "paper_2212_09642_amd", "csrc")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                    "-I", os.path.join(ROOT, "include"), "-I", csrc,
                    os.path.join(ROOT, "tests", "cpp", "test_serve_host.cpp"),
                    os.path.join(csrc, "serve_host.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0 and "serve host ok" in r.stdout, r.stdout + r.stderr


def test_plan_steps_matches_oracle_bound():
    # Proposition 4.4 (polynomial case) with Remark 2.3: the oracle's
    # prop44_poly at gamma = 0 is 2 norm2 rem23(2k - 1, lambda_max)
    rng = np.random.default_rng(5)
    for _ in range(300):
        n = float(np.exp(rng.uniform(np.log(10), np.log(1e7))))
        lam = float(np.exp(rng.uniform(np.log(1e-8), 0.0)))
        s = float(rng.uniform(0.1, 16.0))
        eps = float(np.exp(rng.uniform(np.log(1e-5), np.log(1e-1))))
        kmax = int(rng.integers(2, 129))
        k = vne.plan_steps(n, lam, s, eps, 0.5, kmax)
        target = 0.5 * eps * s
        bound = lambda kk: 2 * n * float(oracle.bounds.rem23(2 * kk - 1, lam))
        assert 2 <= k <= kmax
        if k < kmax:
            assert bound(k) <= target
        if k > 2:
            assert bound(k - 1) > target
        # gamma = 0 makes Theorem 2.2 (as proved) equal to Remark 2.3
        assert np.isclose(float(oracle.bounds.prop44_poly(k, n, 0.0, lam)), bound(k), rtol=1e-12)


def test_plan_probes_closed_form():
    for s_hat, sd, eps in ((10.0, 0.01, 1e-3), (3.0, 0.2, 1e-2), (12.0, 1.5, 1e-3), (5.0, 0.0, 1e-3)):
        want = int(np.ceil((2.576 * sd / (0.5 * eps * s_hat)) ** 2))
        assert vne.plan_probes(s_hat, sd, eps, 0.5, 2.576, 16, 4096) == min(max(want, 16), 4096)


@pytest.mark.parametrize("maker", [lambda: synth.erdos_renyi(400, 6.0, 3),
                                   lambda: synth.barabasi_albert(500, 2, 4),
                                   lambda: synth.watts_strogatz(600, 6, 0.1, 5)])
def test_error_rule_premises_and_guarantee(maker):
    """The rule's inputs bound the truth (Gershgorin >= lambda_max,
    -log tr(rho^2) <= S), and its k meets the quadrature target on every
    probe against the exact quadratic form (dense eigendecomposition)."""
    n, e = maker()
    g = oracle.laplacian_from_edges(n, e)
    rho = oracle.dense_matrix(g)
    lam = np.linalg.eigvalsh(rho)
    lam_ub = np.abs(rho).sum(1).max()
    S = oracle.exact_entropy(rho)
    s_low = -np.log((rho * rho).sum())
    assert lam_ub >= lam[-1] and s_low <= S
    eps = 1e-3
    k = vne.plan_steps(float(g.n), lam_ub, s_low, eps, 0.5, 128)
    B = oracle.rademacher_block(7, g.node_ids, np.arange(16))
    got = oracle.quadforms(g.scipy(), B, k, oracle.breakdown_tau(True))["psi"]
    exact = oracle.exact_quadform(rho, oracle.desingularize(B))
    assert np.all(np.abs(got - exact) <= 0.5 * eps * S)
