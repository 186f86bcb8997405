"""GPU parity of the a-posteriori bracket of Theorem 4.8 (vne_error_bounds)
against the oracle's posterior_bracket on the same Lanczos coefficients, and
its validity against exact errors (dense eigendecomposition)."""
import numpy as np
import pytest

import oracle
import synth
import paper_2212_09642_amd as vne
from gpu_common import ctx, _say  # noqa: F401

pytestmark = pytest.mark.gpu


def _gq(res, m):
    M = res["quad"].size
    return oracle.gauss_quadrature(res["alpha"][:, :m], res["beta"][:, :m], np.full(M, m), res["norm2"])


def test_bounds_example_4_10(ctx):
    # diagonal matrix, Chebyshev points of [1e-3, 1e3], N(0,1) probes (Example 4.10)
    _say("case Theorem 4.8 bracket, Example 4.10")
    n = 2000
    j = np.arange(n)
    lam = 0.5 * (1e3 + 1e-3) + 0.5 * (1e3 - 1e-3) * np.cos((2 * j + 1) * np.pi / (2 * n))
    gid = ctx.register(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), lam, 1.0)
    B = np.random.default_rng(4).standard_normal((n, 3))
    res = ctx.estimate(gid, vne.PROBE_DENSE, 3, 40, vne.MODE_F64, dense=B)
    exact = (B * B * oracle.f_entropy(lam)[:, None]).sum(0)
    for m in (5, 10, 20, 30):
        lo, hi = ctx.error_bounds(res["alpha"], res["beta"], res["k_eff"], res["norm2"], m, lam.min(), lam.max(),
                                  n_grid=2000)
        psi_m = np.array([oracle.gauss_quadrature(res["alpha"][c:c + 1, :m], res["beta"][c:c + 1, :m], [m],
                                                  res["norm2"][c:c + 1])[0] for c in range(3)])
        err = np.abs(psi_m - exact)
        for c in range(3):
            olo, ohi, _ = oracle.bounds.posterior_bracket(res["alpha"][c], res["beta"][c], m, res["norm2"][c],
                                                           lam.min(), lam.max(), grid=2000)
            assert abs(hi[c] - ohi) <= 1e-6 * ohi, (m, c, hi[c], ohi)
            assert abs(lo[c] - olo) <= 1e-6 * ohi
        _say("   m=%d err %s hi %s" % (m, np.array2string(err, precision=2), np.array2string(hi, precision=2)))
        assert np.all(lo * (1 - 1e-6) <= err) and np.all(err <= hi * (1 + 1e-6))


def test_bounds_graph_conservative_interval(ctx):
    """On a Laplacian density matrix with desingularization, the bracket over
    [lambda_2, lambda_n] holds, and the conservative interval the serving loop
    uses ([1e-12 lambda_ub, lambda_ub], Gershgorin lambda_ub) still gives an
    upper bound."""
    _say("case Theorem 4.8 bracket, BA n=1500")
    n, e = synth.barabasi_albert(1500, 3, 33)
    g = vne.laplacian_from_edges(n, e, np.float64)
    ref = oracle.laplacian_from_edges(n, e)
    gid = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
    res = ctx.estimate(gid, vne.PROBE_RADEMACHER, 8, 30, vne.MODE_F64 | vne.MODE_DESING, seed=3)
    rho = oracle.dense_matrix(ref)
    lam = np.linalg.eigvalsh(rho)
    B = oracle.rademacher_block(3, ref.node_ids, np.arange(8))
    exact = oracle.exact_quadform(rho, oracle.desingularize(B))
    lam_ub = np.abs(rho).sum(1).max()
    for m in (3, 6, 10, 16):
        psi_m = _gq(res, m)
        err = np.abs(psi_m - exact)
        lo, hi = ctx.error_bounds(res["alpha"], res["beta"], res["k_eff"], res["norm2"], m, lam[1], lam[-1])
        assert np.all(err <= hi * (1 + 1e-6) + 1e-15) and np.all(lo * (1 - 1e-6) <= err + 1e-15)
        lo2, hi2 = ctx.error_bounds(res["alpha"], res["beta"], res["k_eff"], res["norm2"], m, 1e-12 * lam_ub,
                                    lam_ub, n_grid=256)
        _say("   m=%d max err %.2e  hi [l2,ln] %.2e  hi conservative %.2e" % (m, err.max(), hi.max(), hi2.max()))
        assert np.all(err <= hi2 * (1 + 1e-6) + 1e-15)


def test_bounds_errors(ctx):
    a = np.zeros((2, 5))
    with pytest.raises(vne.VneError):
        ctx.error_bounds(a, a, np.array([5, 5]), np.ones(2), 6, 1e-3, 1.0)
    with pytest.raises(vne.VneError):
        ctx.error_bounds(a, a, np.array([5, 5]), np.ones(2), 3, 0.0, 1.0)
    with pytest.raises(vne.VneError):
        ctx.error_bounds(a, a, np.array([5, 5]), np.ones(2), 3, 1e-3, 1.0, n_grid=1)
