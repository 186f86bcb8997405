"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances (per quadratic form, relative): FP64 vectors 1e-12, FP32 vectors
1e-5.  Integer results (Krylov dimension, graph structure) are compared
exactly.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import workloads
import paper_2212_09642_amd as vne

pytestmark = pytest.mark.gpu

from gpu_common import (TOL, ctx, _say, _setup, _rel, _order_sensitivity, _check_quad, _bar,  # noqa: F401
                        _assert_within, _hutchpp_oracle, _check_hutchpp, _model_tile)


@pytest.mark.parametrize("fp64", [True, False])
def test_tiny_er_hutchinson(ctx, fp64):
    w = workloads.tiny()
    _say("case tiny ER n=2000 m=30 k=40 fp64=%s" % fp64)
    gid, ref = _setup(ctx, w["n_nodes"], w["edges"], fp64)
    mode = vne.MODE_DESING | (vne.MODE_F64 if fp64 else 0)
    out = ctx.estimate(gid, vne.PROBE_RADEMACHER, w["m"], w["k"], mode, seed=w["probe_seed"])
    B = oracle.rademacher_block(w["probe_seed"], ref.node_ids, np.arange(w["m"]))
    want = oracle.quadforms(ref.scipy(), B, w["k"], oracle.breakdown_tau(fp64))
    _check_quad(out, want, fp64, n=ref.n)
    # the first Lanczos coefficients agree before orthogonality is lost
    j = 8
    assert np.allclose(out["alpha"][:, :j], want["alpha"][:, :j], rtol=1e-10 if fp64 else 1e-5, atol=0)
    assert np.allclose(out["beta"][:, :j], want["beta"][:, :j], rtol=1e-10 if fp64 else 1e-5, atol=0)
    assert abs(out["estimate"] - want["psi"].mean()) < TOL[fp64] * abs(out["estimate"])
    # the Hutchinson estimate is within its statistical error of the exact entropy
    S = oracle.exact_entropy(oracle.dense_matrix(ref))
    se = want["psi"].std() / np.sqrt(w["m"])
    assert abs(out["estimate"] - S) < 5 * se


@pytest.mark.parametrize("fp64", [True, False])
def test_complete_graph_breakdown(ctx, fp64):
    n = 64
    _say("case K_64 breakdown fp64=%s" % fp64)
    gid, ref = _setup(ctx, *synth.complete_graph(n), fp64=fp64)
    mode = vne.MODE_DESING | (vne.MODE_F64 if fp64 else 0)
    out = ctx.estimate(gid, vne.PROBE_RADEMACHER, 8, 10, mode, seed=3)
    B = oracle.rademacher_block(3, ref.node_ids, np.arange(8))
    expect = np.log(n - 1) / (n - 1) * ((B * B).sum(0) - B.sum(0) ** 2 / n)
    assert np.all(out["k_eff"] == 1)
    assert np.all(_rel(out["quad"], expect) < TOL[fp64])


@pytest.mark.parametrize("fp64", [True, False])
def test_example_4_10_diagonal(ctx, fp64):
    # diagonal matrix with Chebyshev-point eigenvalues in [1e-3, 1e3], dense N(0,1) probe
    n = 2000
    _say("case Example 4.10 fp64=%s" % fp64)
    j = np.arange(n)
    lam = 0.5 * (1e3 + 1e-3) + 0.5 * (1e3 - 1e-3) * np.cos((2 * j + 1) * np.pi / (2 * n))
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    gid = ctx.register(rp, ci, lam.astype(np.float64 if fp64 else np.float32), 1.0)
    rng = np.random.default_rng(4)
    B = rng.standard_normal((n, 3))
    if not fp64:
        B = B.astype(np.float32).astype(np.float64)
    mode = vne.MODE_F64 if fp64 else 0
    out = ctx.estimate(gid, vne.PROBE_DENSE, 3, 30, mode, dense=B)
    import scipy.sparse as sp
    lam_dev = lam if fp64 else lam.astype(np.float32).astype(np.float64)
    want = oracle.quadforms(sp.diags(lam_dev).tocsr(), B, 30, oracle.breakdown_tau(fp64), desing=False)
    _check_quad(out, want, fp64, n=n)


@pytest.mark.parametrize("fp64", [True, False])
def test_hub_rows_use_segments(ctx, fp64):
    # star: one row with n-1 off-diagonal entries, split across many segments
    _say("case star n=3001 + BA hubs fp64=%s" % fp64)
    for n, e in (synth.star_graph(3001), synth.barabasi_albert(20000, 3, 5)):
        gid, ref = _setup(ctx, n, e, fp64)
        mode = vne.MODE_DESING | (vne.MODE_F64 if fp64 else 0)
        out = ctx.estimate(gid, vne.PROBE_RADEMACHER, 40, 25, mode, seed=8)
        B = oracle.rademacher_block(8, ref.node_ids, np.arange(40))
        want = oracle.quadforms(ref.scipy(), B, 25, oracle.breakdown_tau(fp64))
        _check_quad(out, want, fp64, sens=_order_sensitivity(ref.scipy(), B, 25, fp64), n=ref.n)


@pytest.mark.parametrize("m,k", [(1, 1), (1, 7), (37, 3), (257, 5), (64, 50)])
def test_ragged_shapes(ctx, m, k, monkeypatch):
    """Ragged widths with the autotuner off, so that the byte model's tile
    runs (padded three-column tiles for FP32 m = 37, 257; the one-lane tile
    for m = 1) and the test asserts which one did."""
    _say("case ragged m=%d k=%d" % (m, k))
    monkeypatch.setenv("VNE_AUTOTUNE", "0")
    n, e = synth.watts_strogatz(1237, 6, 0.2, 9)
    with vne.Context(0) as c:
        for fp64 in (True, False):
            gid, ref = _setup(c, n, e, fp64)
            mode = vne.MODE_DESING | (vne.MODE_F64 if fp64 else 0)
            out = c.estimate(gid, vne.PROBE_RADEMACHER, m, k, mode, seed=21)
            plan = c.last_plan()
            tile = _model_tile(m, fp64, ref.n, ref.nnz)
            _say("   fp64=%s tile %d, m_pad %d" % (fp64, plan["tile"], plan["m_pad"]))
            assert plan == dict(tile=tile, m_pad=-(-m // tile) * tile)
            if not fp64 and m in (37, 257):
                assert tile % 3 == 0 and plan["m_pad"] > m      # a padded three-column tile ran
            if m == 1:
                assert tile == (2 if fp64 else 4)               # one lane per row
            B = oracle.rademacher_block(21, ref.node_ids, np.arange(m))
            want = oracle.quadforms(ref.scipy(), B, k, oracle.breakdown_tau(fp64))
            _check_quad(out, want, fp64, n=ref.n)


def test_coloring_probes(ctx):
    _say("case colouring probes WS n=5000 d=2")
    n, e = synth.watts_strogatz(5000, 10, 0.1, 4)
    gid, ref = _setup(ctx, n, e, False)
    col, s = vne.color_greedy(ref.row_ptr.astype(np.int32), ref.col_idx.astype(np.int32), ref.values, 2)
    out = ctx.estimate(gid, vne.PROBE_COLORING, s, 40, vne.MODE_DESING, colors=col)
    P = oracle.indicator_block(col, s)
    want = oracle.quadforms(ref.scipy(), P, 40, oracle.breakdown_tau(False))
    _check_quad(out, want, False, n=ref.n)
    assert abs(out["estimate"] - want["psi"].sum()) < 1e-5 * abs(out["estimate"])


def test_dense_probes_device_tensor(ctx):
    import torch
    _say("case dense probes from a device tensor")
    n, e = synth.barabasi_albert(3000, 2, 6)
    gid, ref = _setup(ctx, n, e, True)
    rng = np.random.default_rng(1)
    B = rng.standard_normal((ref.n, 12))
    Bt = torch.tensor(B, dtype=torch.float64, device="cuda")
    out = ctx.estimate(gid, vne.PROBE_DENSE, 12, 30, vne.MODE_F64 | vne.MODE_DESING, dense=Bt)
    want = oracle.quadforms(ref.scipy(), B, 30, oracle.breakdown_tau(True))
    _check_quad(out, want, True, sens=_order_sensitivity(ref.scipy(), B, 30, True), n=ref.n)
    # the binding refuses device tensors the library would misread
    with pytest.raises(ValueError):
        ctx.estimate(gid, vne.PROBE_DENSE, 12, 30, vne.MODE_F64 | vne.MODE_DESING,
                     dense=Bt.t().contiguous().t())        # (n, 12) view with column-major strides
    with pytest.raises(ValueError):
        ctx.estimate(gid, vne.PROBE_DENSE, 12, 30, vne.MODE_F64 | vne.MODE_DESING, dense=Bt.float())


def test_deterministic(ctx):
    _say("case run-twice bitwise")
    n, e = synth.barabasi_albert(30000, 3, 2)
    gid, ref = _setup(ctx, n, e, False)
    a = ctx.estimate(gid, vne.PROBE_RADEMACHER, 64, 30, vne.MODE_DESING, seed=5)
    b = ctx.estimate(gid, vne.PROBE_RADEMACHER, 64, 30, vne.MODE_DESING, seed=5)
    for key in ("quad", "alpha", "beta", "k_eff", "norm2"):
        assert np.array_equal(a[key], b[key]), key
    assert a["estimate"] == b["estimate"]


@pytest.mark.parametrize("fp64", [True, False])
def test_narrow_tiles(ctx, fp64, monkeypatch):
    """Tiles of one and two lanes per row (4 and 8 FP32 columns, 2 and 4
    FP64): the byte model's choice for blocks of a few columns, forced tiles
    (two tiles of a block run as concurrent chains), the long rows of a hub
    graph in segments, and a Hutch++ whose three-column sketch takes a
    narrow tile; each against the oracle at the usual bar."""
    cpl = 2 if fp64 else 4
    monkeypatch.setenv("VNE_AUTOTUNE", "0")
    n, e = synth.barabasi_albert(6000, 3, 31)
    mode = vne.MODE_DESING | (vne.MODE_F64 if fp64 else 0)
    with vne.Context(0) as c:
        gid, ref = _setup(c, n, e, fp64)
        A = ref.scipy()
        for m, forced in ((1, 0), (3, 0), (cpl, 0), (2 * cpl, cpl), (2 * cpl, 2 * cpl), (5, cpl)):
            monkeypatch.setenv("VNE_TILE", str(forced))
            _say("case narrow tile fp64=%s m=%d forced=%d" % (fp64, m, forced))
            out = c.estimate(gid, vne.PROBE_RADEMACHER, m, 20, mode, seed=40 + m)
            plan = c.last_plan()
            tile = forced if forced else _model_tile(m, fp64, ref.n, ref.nnz)
            _say("   tile %d, m_pad %d" % (plan["tile"], plan["m_pad"]))
            assert tile <= 2 * cpl and plan == dict(tile=tile, m_pad=-(-m // tile) * tile)
            B = oracle.rademacher_block(40 + m, ref.node_ids, np.arange(m))
            want = oracle.quadforms(A, B, 20, oracle.breakdown_tau(fp64))
            _check_quad(out, want, fp64, sens=_order_sensitivity(A, B, 20, fp64), n=ref.n)
        monkeypatch.setenv("VNE_TILE", "0")
        _say("case narrow tile fp64=%s: Hutch++ 3 + 13" % fp64)
        out = c.estimate(gid, vne.PROBE_HUTCHPP, 16, 20, mode, seed=5, n_sketch=3)
        Om = oracle.rademacher_block(5, ref.node_ids, np.arange(3))
        G = oracle.rademacher_block(5, ref.node_ids, np.arange(3, 16))
        est, det, sens = _hutchpp_oracle(A, Om, G, 20, fp64)
        _check_hutchpp(out, est, det, sens, 3, fp64)


@pytest.mark.parametrize("fp64", [True, False])
def test_hutchpp_small(ctx, fp64):
    _say("case Hutch++ BA n=3000 16+16 fp64=%s" % fp64)
    n, e = synth.barabasi_albert(3000, 3, 7)
    gid, ref = _setup(ctx, n, e, fp64)
    nr, nh, k = 16, 16, 30
    mode = vne.MODE_DESING | (vne.MODE_F64 if fp64 else 0)
    out = ctx.estimate(gid, vne.PROBE_HUTCHPP, nr + nh, k, mode, seed=13, n_sketch=nr)
    Om = oracle.rademacher_block(13, ref.node_ids, np.arange(nr))
    G = oracle.rademacher_block(13, ref.node_ids, np.arange(nr, nr + nh))
    est, det, sens = _hutchpp_oracle(ref.scipy(), Om, G, k, fp64)
    _check_hutchpp(out, est, det, sens, nr, fp64)


def test_error_paths(ctx):
    _say("case error paths")
    n, e = synth.cycle_graph(50)
    gid, ref = _setup(ctx, n, e, False)
    with pytest.raises(vne.VneError) as ei:
        ctx.estimate(gid, vne.PROBE_RADEMACHER, 4, 0, vne.MODE_DESING)
    assert ei.value.status == -1
    with pytest.raises(vne.VneError):
        ctx.estimate(gid, vne.PROBE_RADEMACHER, 4, 129, vne.MODE_DESING)
    with pytest.raises(vne.VneError):
        ctx.estimate(gid, vne.PROBE_RADEMACHER, 0, 5, vne.MODE_DESING)
    with pytest.raises(vne.VneError):
        ctx.estimate(gid + 100, vne.PROBE_RADEMACHER, 4, 5, vne.MODE_DESING)
    with pytest.raises(vne.VneError):
        ctx.estimate(gid, vne.PROBE_COLORING, 3, 5, vne.MODE_DESING, colors=np.full(ref.n, 7))
    # desingularization needs zero row sums
    rp = np.arange(11, dtype=np.int32)
    gid2 = ctx.register(rp, np.arange(10, dtype=np.int32), np.ones(10, np.float32), 0.1)
    with pytest.raises(vne.VneError):
        ctx.estimate(gid2, vne.PROBE_RADEMACHER, 4, 5, vne.MODE_DESING)
    # malformed matrix rejected at registration (row 0 repeats column 1)
    rp_bad = np.array([0, 2] + [2] * 9, np.int32)
    with pytest.raises(vne.VneError):
        ctx.register(rp_bad, np.array([1, 1], np.int32), np.ones(2, np.float32), 0.1)
    # a budget too small for the workspace
    with vne.Context(0, hbm_budget_bytes=1 << 16) as small:
        with pytest.raises(vne.VneError) as ei:
            g2 = small.register(ref.row_ptr.astype(np.int32), ref.col_idx.astype(np.int32),
                                ref.values.astype(np.float32), ref.scale)
            small.estimate(g2, vne.PROBE_RADEMACHER, 64, 10, vne.MODE_DESING)
        assert ei.value.status == -2


@pytest.mark.parametrize("fp64", [True, False])
def test_numerical_failures_are_reported(ctx, fp64):
    """A NaN in a dense probe block makes the Lanczos coefficients non-finite
    and the call fails with VNE_ENUMERIC; a Hutch++ sketch whose Gram matrix
    is singular (single edge: rho has eigenvalues 0 and 1 and f(1) = 0, so
    f(A) Omega is exactly zero) fails with VNE_ENUMERIC in its Cholesky
    factorisation; the context stays usable after both."""
    _say("case VNE_ENUMERIC: NaN probe, singular sketch Gram, fp64=%s" % fp64)
    n, e = synth.erdos_renyi(500, 6.0, 51)
    gid, ref = _setup(ctx, n, e, fp64)
    mode = vne.MODE_DESING | (vne.MODE_F64 if fp64 else 0)
    B = np.random.default_rng(2).standard_normal((ref.n, 6))
    bad = B.copy()
    bad[17, 3] = np.nan
    with pytest.raises(vne.VneError) as ei:
        ctx.estimate(gid, vne.PROBE_DENSE, 6, 12, mode, dense=bad)
    assert ei.value.status == -6 and "non-finite" in str(ei.value)
    if not fp64:
        B = B.astype(np.float32).astype(np.float64)
    good = ctx.estimate(gid, vne.PROBE_DENSE, 6, 12, mode, dense=B)
    want = oracle.quadforms(ref.scipy(), B, 12, oracle.breakdown_tau(fp64))
    _check_quad(good, want, fp64, n=ref.n)
    g1, _ = _setup(ctx, 2, np.array([[0, 1]]), fp64)
    with pytest.raises(vne.VneError) as ei:
        ctx.estimate(g1, vne.PROBE_HUTCHPP, 8, 5, mode, seed=3, n_sketch=4)
    assert ei.value.status == -6 and "Cholesky" in str(ei.value)
    again = ctx.estimate(gid, vne.PROBE_DENSE, 6, 12, mode, dense=B)
    assert np.array_equal(again["quad"], good["quad"])
    ctx.release(g1)
    ctx.release(gid)


@pytest.mark.parametrize("fp64", [True, False])
def test_schedules_bitwise_identical(ctx, fp64, monkeypatch):
    # lazy one-pass and normalize + single-stream schedules evaluate every
    # entry of v_j with the same expression and sum in the same order
    _say("case lazy vs two-pass schedule fp64=%s" % fp64)
    n, e = synth.barabasi_albert(20000, 3, 11)
    gid, ref = _setup(ctx, n, e, fp64)
    mode = vne.MODE_DESING | (vne.MODE_F64 if fp64 else 0)
    outs = []
    for sched in ("0", "1"):
        monkeypatch.setenv("VNE_SCHED", sched)
        outs.append(ctx.estimate(gid, vne.PROBE_RADEMACHER, 48, 20, mode, seed=17))
    for key in ("quad", "alpha", "beta", "k_eff", "norm2"):
        assert np.array_equal(outs[0][key], outs[1][key]), key


@pytest.mark.parametrize("fp64", [True, False])
def test_tile_chains_bitwise_identical(ctx, fp64, monkeypatch):
    # the tiles of a block split into concurrent chains on streams of their
    # own touch only their own columns: every result is the same to the bit
    # as one chain, with captured graphs, with direct launches under kernel
    # timing, and for the stored basis of the Hutch++ sketch
    _say("case tile chains fp64=%s" % fp64)
    n, e = synth.barabasi_albert(20000, 3, 12)
    gid, ref = _setup(ctx, n, e, fp64)
    mode = vne.MODE_DESING | (vne.MODE_F64 if fp64 else 0)
    monkeypatch.setenv("VNE_AUTOTUNE", "0")
    monkeypatch.setenv("VNE_TILE", "16" if fp64 else "32")
    outs = []
    for chains, timing in (("1", False), ("2", False), ("4", False), ("3", True)):
        monkeypatch.setenv("VNE_CHAINS", chains)
        ctx.enable_kernel_timing(timing)
        r = ctx.estimate(gid, vne.PROBE_RADEMACHER, 100, 25, mode, seed=31)
        h = ctx.estimate(gid, vne.PROBE_HUTCHPP, 96, 20, mode, seed=32, n_sketch=64)
        assert ctx.last_plan()["tile"] == (16 if fp64 else 32)
        outs.append((r, h))
        ctx.enable_kernel_timing(False)
    for r, h in outs[1:]:
        for key in ("quad", "alpha", "beta", "k_eff", "norm2"):
            assert np.array_equal(r[key], outs[0][0][key]), key
            assert np.array_equal(h[key], outs[0][1][key]), key
        assert h["estimate"] == outs[0][1]["estimate"]
    # the chains against the oracle at 12 steps (at 25, some columns of this
    # graph have lost orthogonality and their forms move by ~1e-7 under any
    # change of rounding, as the tile width alone shows)
    monkeypatch.setenv("VNE_CHAINS", "4")
    out = ctx.estimate(gid, vne.PROBE_RADEMACHER, 100, 12, mode, seed=31)
    B = oracle.rademacher_block(31, ref.node_ids, np.arange(100))
    want = oracle.quadforms(ref.scipy(), B, 12, oracle.breakdown_tau(fp64))
    _check_quad(out, want, fp64, sens=_order_sensitivity(ref.scipy(), B, 12, fp64), n=ref.n)


def test_graph_and_timing_paths_agree(ctx, monkeypatch):
    # captured graph, per-part graphs with kernel timing, and direct launches
    # run the same kernels in the same order
    _say("case graph / timing / direct launch paths")
    n, e = synth.barabasi_albert(8000, 3, 12)
    gid, ref = _setup(ctx, n, e, False)
    base = ctx.estimate(gid, vne.PROBE_HUTCHPP, 48, 15, vne.MODE_DESING, seed=3, n_sketch=16)
    ctx.enable_kernel_timing(True)
    ctx.kernel_timing(reset=True)
    timed = ctx.estimate(gid, vne.PROBE_HUTCHPP, 48, 15, vne.MODE_DESING, seed=3, n_sketch=16)
    t = ctx.kernel_timing(reset=True)
    ctx.enable_kernel_timing(False)
    assert t["launches"] == 30 and t["total_ms"] > 0 and t["bytes"] > 0
    monkeypatch.setenv("VNE_GRAPH", "0")
    direct = ctx.estimate(gid, vne.PROBE_HUTCHPP, 48, 15, vne.MODE_DESING, seed=3, n_sketch=16)
    for other in (timed, direct):
        for key in ("quad", "alpha", "beta", "k_eff", "norm2"):
            assert np.array_equal(base[key], other[key]), key


@pytest.mark.parametrize("fp64", [True, False])
def test_max_steps_and_wide_block(ctx, fp64):
    # k = 128 (the largest the kernels take; the QR runs with two register
    # halves) and m = 1000 (eight column tiles with a ragged last one)
    _say("case k=128 and m=1000 fp64=%s" % fp64)
    n, e = synth.watts_strogatz(3000, 8, 0.1, 41)
    gid, ref = _setup(ctx, n, e, fp64)
    mode = vne.MODE_DESING | (vne.MODE_F64 if fp64 else 0)
    A = ref.scipy()
    out = ctx.estimate(gid, vne.PROBE_RADEMACHER, 6, 128, mode, seed=12)
    B = oracle.rademacher_block(12, ref.node_ids, np.arange(6))
    want = oracle.quadforms(A, B, 128, oracle.breakdown_tau(fp64))
    _check_quad(out, want, fp64, k_exact=False, sens=_order_sensitivity(A, B, 128, fp64), n=ref.n)
    out = ctx.estimate(gid, vne.PROBE_RADEMACHER, 1000, 12, mode, seed=13, want_coeffs=False)
    cols = np.array([0, 511, 999])
    B = oracle.rademacher_block(13, ref.node_ids, cols)
    want = oracle.quadforms(A, B, 12, oracle.breakdown_tau(fp64))
    rel = _rel(out["quad"][cols], want["psi"])
    assert np.all(rel < TOL[fp64]), rel
    assert abs(out["estimate"] - out["quad"].mean()) <= 1e-13 * abs(out["estimate"])


def test_single_edge_graph(ctx):
    # two nodes: rho = [[.5, -.5], [-.5, .5]] has eigenvalues 0 and 1, S = 0;
    # the desingularized probe lies in the eigenvalue-1 direction
    _say("case single edge")
    gid, ref = _setup(ctx, 2, np.array([[0, 1]]), True)
    out = ctx.estimate(gid, vne.PROBE_RADEMACHER, 4, 5, vne.MODE_DESING | vne.MODE_F64, seed=2)
    assert np.all(out["k_eff"] <= 1)
    assert np.all(np.abs(out["quad"]) < 1e-15)


def test_hutchpp_wide_g_block(ctx):
    # N_H = 200 > 128: the projection G - Q (Q^T G) runs in column slices
    _say("case Hutch++ BA n=3000 24+200 fp32")
    n, e = synth.barabasi_albert(3000, 3, 17)
    gid, ref = _setup(ctx, n, e, False)
    nr, nh, k = 24, 200, 25
    out = ctx.estimate(gid, vne.PROBE_HUTCHPP, nr + nh, k, vne.MODE_DESING, seed=19, n_sketch=nr)
    Om = oracle.rademacher_block(19, ref.node_ids, np.arange(nr))
    G = oracle.rademacher_block(19, ref.node_ids, np.arange(nr, nr + nh))
    est, det, sens = _hutchpp_oracle(ref.scipy(), Om, G, k, False)
    _check_hutchpp(out, est, det, sens, nr, False)


@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("neg", [-0.3, -1e-10, -1e-14])
def test_quadrature_negative_and_near_null_spectrum(ctx, fp64, neg):
    """The quadrature's integral route needs T + tI positive definite down to
    its lower limit: a clearly negative eigenvalue (f = 0 there, eq. (2.1))
    sends the column to the QR route; a tiny negative one moves the lower
    limit (FP32 coefficients) or also takes the QR route (FP64, where the
    moved limit would cost accuracy).  Every case against the oracle's
    diagonalisation at the usual bar."""
    n = 400
    _say("case quadrature with a negative eigenvalue %g, fp64=%s" % (neg, fp64))
    lam = np.linspace(1e-3, 1.0, n)
    lam[0] = neg
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    gid = ctx.register(rp, ci, lam.astype(np.float64 if fp64 else np.float32), 1.0)
    rng = np.random.default_rng(9)
    B = rng.standard_normal((n, 4))
    B[0, :] = [1.0, 1e-3, 1e-6, 0.0]                 # weight on the negative eigenvalue
    if not fp64:
        B = B.astype(np.float32).astype(np.float64)
    mode = vne.MODE_F64 if fp64 else 0
    import scipy.sparse as sp
    lam_dev = lam if fp64 else lam.astype(np.float32).astype(np.float64)
    A = sp.diags(lam_dev).tocsr()
    for k in (5, 40, 100):
        out = ctx.estimate(gid, vne.PROBE_DENSE, 4, k, mode, dense=B)
        want = oracle.quadforms(A, B, k, oracle.breakdown_tau(fp64), desing=False)
        # past the first Ritz convergences plain Lanczos is rounding-sensitive
        _check_quad(out, want, fp64, sens=_order_sensitivity(A, B, k, fp64, desing=False), n=n)
    ctx.release(gid)


def test_hutchpp_changing_sketch_width(ctx):
    """The same (m, k) with a different N_r on each call: the workspace sized
    for N_r = 8 must grow for N_r = 96 and still serve N_r = 8 afterwards;
    each estimate against the oracle's."""
    _say("case Hutch++ with N_r = 8, 96, 8 at the same m, k")
    n, e = synth.erdos_renyi(2500, 6.0, 17)
    gid, ref = _setup(ctx, n, e, True)
    m, k = 128, 20
    mode = vne.MODE_DESING | vne.MODE_F64
    for nr in (8, 96, 8):
        out = ctx.estimate(gid, vne.PROBE_HUTCHPP, m, k, mode, seed=5, n_sketch=nr, want_coeffs=False)
        Om = oracle.rademacher_block(5, ref.node_ids, np.arange(nr))
        G = oracle.rademacher_block(5, ref.node_ids, np.arange(nr, m))
        est, det, sens = _hutchpp_oracle(ref.scipy(), Om, G, k, True)
        _say("   N_r=%d" % nr)
        _check_hutchpp(out, est, det, sens, nr, True)
    ctx.release(gid)


@pytest.mark.parametrize("nr,nh", [(8, 0), (1, 7), (128, 8)])
def test_hutchpp_sketch_width_edges(ctx, nr, nh):
    """Hutch++ with no Hutchinson part (N_H = 0: the estimate is the sum over
    Q), a one-column sketch, and the widest sketch (N_r = 128), FP64 vectors,
    against the oracle (eq. (3.9))."""
    _say("case Hutch++ N_r=%d N_H=%d" % (nr, nh))
    n, e = synth.erdos_renyi(1500, 8.0, 29)
    gid, ref = _setup(ctx, n, e, True)
    k = 20
    out = ctx.estimate(gid, vne.PROBE_HUTCHPP, nr + nh, k, vne.MODE_DESING | vne.MODE_F64, seed=31,
                       n_sketch=nr, want_coeffs=False)
    Om = oracle.rademacher_block(31, ref.node_ids, np.arange(nr))
    G = oracle.rademacher_block(31, ref.node_ids, np.arange(nr, nr + nh))
    est, det, sens = _hutchpp_oracle(ref.scipy(), Om, G, k, True)
    _check_hutchpp(out, est, det, sens, nr, True)
    if nh == 0:
        assert abs(out["estimate"] - out["quad"].sum()) <= 1e-13 * abs(out["estimate"])
    ctx.release(gid)


def test_device_csr_and_device_colours(ctx):
    """A matrix registered from device tensors (borrowed row_ptr and col_idx)
    and colour indicators given as a device tensor give the same bits as the
    host registration and host colours."""
    import torch
    _say("case device-resident CSR and colours, WS n=4000")
    n, e = synth.watts_strogatz(4000, 8, 0.1, 33)
    g = vne.laplacian_from_edges(n, e, np.float32)
    gid_h = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
    rp = torch.tensor(g["row_ptr"], dtype=torch.int32, device="cuda")
    ci = torch.tensor(g["col_idx"], dtype=torch.int32, device="cuda")
    va = torch.tensor(g["values"], dtype=torch.float32, device="cuda")
    gid_d = ctx.register(rp, ci, va, g["scale"], node_keys=g["node_ids"])
    mode = vne.MODE_DESING
    a = ctx.estimate(gid_h, vne.PROBE_RADEMACHER, 24, 30, mode, seed=4)
    b = ctx.estimate(gid_d, vne.PROBE_RADEMACHER, 24, 30, mode, seed=4)
    assert np.array_equal(a["quad"], b["quad"]) and a["estimate"] == b["estimate"]
    col, s = vne.color_greedy(g["row_ptr"], g["col_idx"], g["values"], 2)
    colt = torch.tensor(col, dtype=torch.int32, device="cuda")
    c1 = ctx.estimate(gid_h, vne.PROBE_COLORING, s, 30, mode, colors=col)
    c2 = ctx.estimate(gid_d, vne.PROBE_COLORING, s, 30, mode, colors=colt)
    assert np.array_equal(c1["quad"], c2["quad"]) and c1["estimate"] == c2["estimate"]
    # arrays of the wrong length are refused before the library reads them
    with pytest.raises(ValueError):
        ctx.estimate(gid_h, vne.PROBE_COLORING, s, 30, mode, colors=col[:-1])
    with pytest.raises(ValueError):
        ctx.estimate(gid_h, vne.PROBE_DENSE, 4, 30, mode, dense=np.ones((g["n"], 5), np.float32))
    with pytest.raises(ValueError):
        ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"][:-1])
    ctx.release(gid_d)
    ctx.release(gid_h)
    del rp, ci, va, colt


def test_stream_memory_and_budget(monkeypatch):
    """A context on a stream of its own gives the bits of the default stream
    (with the autotuner off, so that both contexts run the same column tile:
    a timed choice may differ between contexts and change the summation
    order); vne_ctx_memory follows registration and release; an estimate
    whose workspace exceeds the HBM budget fails with VNE_ENOMEM and leaves
    the context usable."""
    import torch
    _say("case stream, memory accounting and HBM budget")
    monkeypatch.setenv("VNE_AUTOTUNE", "0")
    n, e = synth.erdos_renyi(6000, 8.0, 35)
    g = vne.laplacian_from_edges(n, e, np.float32)
    mode = vne.MODE_DESING
    with vne.Context(0) as c0:
        gid = c0.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
        want = c0.estimate(gid, vne.PROBE_RADEMACHER, 32, 25, mode, seed=8)
    st = torch.cuda.Stream()                      # default priority
    with vne.Context(0, stream=st.cuda_stream) as c1:
        before = c1.memory()
        gid = c1.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
        after_reg = c1.memory()
        got = c1.estimate(gid, vne.PROBE_RADEMACHER, 32, 25, mode, seed=8)
        c1.set_stream(torch.cuda.current_stream().cuda_stream)
        got2 = c1.estimate(gid, vne.PROBE_RADEMACHER, 32, 25, mode, seed=8)
        c1.release(gid)
        assert after_reg > before and c1.memory() < after_reg
    assert np.array_equal(want["quad"], got["quad"]) and np.array_equal(want["quad"], got2["quad"])
    # a budget that holds the matrix but not a 256-column workspace
    with vne.Context(0, hbm_budget_bytes=4 << 20) as c2:
        gid = c2.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
        with pytest.raises(vne.VneError) as ex:
            c2.estimate(gid, vne.PROBE_RADEMACHER, 256, 25, mode, seed=8)
        assert ex.value.status == -2
        small = c2.estimate(gid, vne.PROBE_RADEMACHER, 4, 10, mode, seed=8)
        assert np.isfinite(small["estimate"])
        c2.release(gid)


@pytest.mark.parametrize("m", [12, 24, 48, 96, 192])
def test_three_column_tiles(ctx, m, monkeypatch):
    """FP32 widths 3 * 2^j run in tiles of three columns per lane (no padding
    to the next power of two): Rademacher forms on a BA graph with hub rows
    (long rows in segments) against the oracle."""
    _say("case three-column tiles m=%d" % m)
    # a context of its own with the autotuner off, so that the three-column
    # tile is the one that runs
    monkeypatch.setenv("VNE_AUTOTUNE", "0")
    n, e = synth.barabasi_albert(6000, 3, 41)
    with vne.Context(0) as c:
        gid, ref = _setup(c, n, e, False)
        k = 25
        out = c.estimate(gid, vne.PROBE_RADEMACHER, m, k, vne.MODE_DESING, seed=43)
    B = oracle.rademacher_block(43, ref.node_ids, np.arange(m))
    want = oracle.quadforms(ref.scipy(), B, k, oracle.breakdown_tau(False))
    _check_quad(out, want, False, sens=_order_sensitivity(ref.scipy(), B, k, False), n=ref.n)


def test_padded_three_column_tile_colouring(monkeypatch):
    """37 colour indicators (not a width 3 * 2^j) with the autotuner off: the
    byte model pads them to a three-column tile of 48; every colour's form
    against the oracle."""
    _say("case colouring with 37 colours in a padded three-column tile")
    monkeypatch.setenv("VNE_AUTOTUNE", "0")
    n, e = synth.watts_strogatz(6000, 8, 0.1, 46)
    with vne.Context(0) as c:
        gid, ref = _setup(c, n, e, False)
        col = (np.arange(ref.n) % 37).astype(np.int32)
        out = c.estimate(gid, vne.PROBE_COLORING, 37, 30, vne.MODE_DESING, colors=col)
        plan = c.last_plan()
    tile = _model_tile(37, False, ref.n, ref.nnz)
    _say("   tile %d, m_pad %d" % (plan["tile"], plan["m_pad"]))
    assert tile % 3 == 0 and plan == dict(tile=tile, m_pad=-(-37 // tile) * tile) and plan["m_pad"] > 37
    P = oracle.indicator_block(col, 37)
    want = oracle.quadforms(ref.scipy(), P, 30, oracle.breakdown_tau(False))
    _check_quad(out, want, False, sens=_order_sensitivity(ref.scipy(), P, 30, False), n=ref.n)


def test_three_column_tiles_colouring_and_sketch(ctx, monkeypatch):
    """Colour indicators with 24 colours and a Hutch++ sketch of 24 columns in
    three-column tiles, against the oracle; the padded power-of-two tile
    gives the same forms within the bar."""
    _say("case three-column tiles: 24 colours, Hutch++ sketch of 24")
    n, e = synth.watts_strogatz(9000, 6, 0.1, 44)
    gid, ref = _setup(ctx, n, e, False)
    # a colouring with exactly 24 colours: rows coloured round robin
    col = (np.arange(ref.n) % 24).astype(np.int32)
    out = ctx.estimate(gid, vne.PROBE_COLORING, 24, 30, vne.MODE_DESING, colors=col)
    P = oracle.indicator_block(col, 24)
    want = oracle.quadforms(ref.scipy(), P, 30, oracle.breakdown_tau(False))
    _check_quad(out, want, False, sens=_order_sensitivity(ref.scipy(), P, 30, False), n=ref.n)
    nr, nh, k = 24, 40, 20
    hp = ctx.estimate(gid, vne.PROBE_HUTCHPP, nr + nh, k, vne.MODE_DESING, seed=45, n_sketch=nr,
                      want_coeffs=False)
    Om = oracle.rademacher_block(45, ref.node_ids, np.arange(nr))
    G = oracle.rademacher_block(45, ref.node_ids, np.arange(nr, nr + nh))
    est, det, sens = _hutchpp_oracle(ref.scipy(), Om, G, k, False)
    _check_hutchpp(hp, est, det, sens, nr, False)
    ctx.release(gid)
    # the padded power-of-two tile (VNE_TILE3=0) gives the same forms within the bar
    monkeypatch.setenv("VNE_TILE3", "0")
    with vne.Context(0) as c2:
        g2 = vne.laplacian_from_edges(n, e, np.float32)
        gid2 = c2.register(g2["row_ptr"], g2["col_idx"], g2["values"], g2["scale"], node_keys=g2["node_ids"])
        out2 = c2.estimate(gid2, vne.PROBE_COLORING, 24, 30, vne.MODE_DESING, colors=col)
    rel = np.abs(out2["quad"] - out["quad"]) / np.abs(out["quad"])
    assert rel.max() < TOL[False], rel.max()
