"""The distance choice of Algorithm 2 in the library (host code, no GPU)
against the oracle's reading of eq. (5.1) and Corollary 3.2."""
import numpy as np
import pytest

from oracle import probing
import paper_2212_09642_amd as vne


def test_heuristic_choice_matches_oracle():
    rng = np.random.default_rng(7)
    for _ in range(2000):
        T1 = float(rng.uniform(1, 12))
        e1 = float(np.exp(rng.uniform(-12, 0)))
        ratio = float(np.exp(rng.uniform(-6, 1)))       # e2 / e1, sometimes large (fallback)
        T = (T1, T1 + e1 * rng.choice([-1, 1]), 0.0)
        T = (T[0], T[1], T[1] + e1 * ratio * rng.choice([-1, 1]))
        eps_hat = float(np.exp(rng.uniform(-14, -2)))
        n = float(rng.integers(100, 10 ** 7))
        b = float(np.exp(rng.uniform(-8, -1)))
        d_max = int(rng.integers(1, 65))
        got = vne.probing_select(T, eps_hat, n, b, d_max)
        d, fits, fallback, capped = probing.select_d(T, eps_hat, n, b, d_max)
        assert (got["d"], got["fallback"], got["capped"]) == (d, int(fallback), int(capped))
        assert got["e1"] == pytest.approx(fits[0][1], rel=1e-15)
        if fits[0][2] is not None:
            assert got["q"] == pytest.approx([fits[0][2], fits[1][2]], rel=1e-14)


def test_bound_choice_matches_oracle():
    rng = np.random.default_rng(8)
    for _ in range(500):
        eps_hat = float(np.exp(rng.uniform(-10, -1)))
        n = float(rng.integers(100, 10 ** 7))
        b = float(np.exp(rng.uniform(-8, -1)))
        d_max = int(rng.integers(1, 65))
        got = vne.probing_select(None, eps_hat, n, b, d_max, use_bound=True)
        d, capped = probing.bound_d(n, b, eps_hat, d_max)
        assert (got["d"], got["capped"], got["fallback"]) == (d, int(capped), 1)


def test_choice_edge_cases():
    # converged differences, no-decay fits, invalid arguments
    assert vne.probing_select([2.0, 2.0, 2.0], 1e-3, 1e4, 1e-3, 8)["d"] == 1
    r = vne.probing_select([2.0, 2.0, 2.1], 1e-3, 1e4, 1e-3, 8)
    assert r["fallback"] == 1 and r["capped"] == 1 and r["d"] == 8
    # Corollary 3.2 starts at d = 2: with d_max = 1 the choice stays at 1, capped
    for use_bound in (False, True):
        r = vne.probing_select([2.0, 2.0, 2.1], 1e3, 1e4, 1e-3, 1, use_bound=use_bound)
        assert (r["d"], r["fallback"], r["capped"]) == (1, 1, 1)
    for bad in [dict(eps_hat=0.0), dict(n=0.0), dict(lambda_ub=-1.0), dict(d_max=0), dict(d_max=65)]:
        args = dict(T=[1.0, 1.1, 1.15], eps_hat=1e-3, n=1e4, lambda_ub=1e-3, d_max=8)
        args.update(bad)
        with pytest.raises(vne.VneError):
            vne.probing_select(**args)
