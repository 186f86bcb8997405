"""GPU parity of the multi-graph batch entry point (several graphs stacked
block-diagonally, one launch per Lanczos step): every query of a batch
against the FP64 oracle at the per-quadratic-form bar, against the same
query run alone, and the batch-specific error paths.
"""
import numpy as np
import pytest

import oracle
import synth
import paper_2212_09642_amd as vne
from gpu_common import TOL, ctx, _say, _rel, _order_sensitivity, _check_quad, _bar, _assert_within  # noqa: F401

pytestmark = pytest.mark.gpu


def _graphs():
    # (name, (n, edges), m, k): uneven sizes, hub rows, breakdown cases
    return [
        ("er300", synth.erdos_renyi(300, 6.0, 11), 12, 20),
        ("ba1500", synth.barabasi_albert(1500, 3, 12), 20, 30),
        ("star500", synth.star_graph(500), 8, 10),
        ("k40", synth.complete_graph(40), 5, 6),
        ("path200", synth.path_graph(200), 16, 25),
        ("grid20", synth.grid2d_graph(20, 20), 33, 15),
        ("ws3000", synth.watts_strogatz(3000, 8, 0.1, 13), 1, 40),
        ("er2000", synth.erdos_renyi(2000, 8.0, 14), 40, 1),
    ]


def _register_all(ctx, cases, fp64):
    out = []
    for name, (n, e), m, k in cases:
        g = vne.laplacian_from_edges(n, e, np.float64 if fp64 else np.float32)
        ref = oracle.laplacian_from_edges(n, e)
        gid = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
        out.append((name, gid, ref, m, k))
    return out


@pytest.mark.parametrize("fp64", [True, False])
def test_batch_rademacher_vs_oracle_and_solo(ctx, fp64):
    _say("case batch of 8 graphs, Rademacher, per-graph m and k, fp64=%s" % fp64)
    regs = _register_all(ctx, _graphs(), fp64)
    mode = vne.MODE_DESING | (vne.MODE_F64 if fp64 else 0)
    queries = [dict(gid=gid, kind=vne.PROBE_RADEMACHER, m=m, k=k, seed=100 + i)
               for i, (name, gid, ref, m, k) in enumerate(regs)]
    outs = ctx.estimate_batch(queries, mode, want_coeffs=True)
    for i, ((name, gid, ref, m, k), out) in enumerate(zip(regs, outs)):
        _say("  query %d %s n=%d m=%d k=%d" % (i, name, ref.n, m, k))
        B = oracle.rademacher_block(100 + i, ref.node_ids, np.arange(m))
        A = ref.scipy()
        want = oracle.quadforms(A, B, k, oracle.breakdown_tau(fp64))
        sens = _order_sensitivity(A, B, k, fp64)
        _check_quad(out, want, fp64, sens=sens, n=ref.n)
        assert out["alpha"].shape == (m, k)
        assert abs(out["estimate"] - out["quad"].mean()) <= 1e-13 * abs(out["estimate"])
        solo = ctx.estimate(gid, vne.PROBE_RADEMACHER, m, k, mode, seed=100 + i)
        assert np.array_equal(solo["k_eff"], out["k_eff"])
        _assert_within(_rel(out["quad"], solo["quad"]), _bar(fp64, sens), "batch vs solo")
        # the first steps agree closely (before any loss of orthogonality)
        j = min(k, 4)
        live = out["k_eff"] >= j
        assert np.allclose(out["alpha"][live, :j], solo["alpha"][live, :j], rtol=1e-12 if fp64 else 1e-5)


def test_batch_repeated_graph_is_bitwise_identical(ctx):
    # the same graph twice in one batch, same seed: the two copies run the
    # same blocks in the same order
    _say("case batch with a repeated graph")
    n, e = synth.barabasi_albert(5000, 3, 21)
    g = vne.laplacian_from_edges(n, e, np.float32)
    gid = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
    q = dict(gid=gid, kind=vne.PROBE_RADEMACHER, m=24, k=30, seed=5)
    a, b = ctx.estimate_batch([q, dict(q)], vne.MODE_DESING, want_coeffs=True)
    for key in ("quad", "alpha", "beta", "k_eff", "norm2"):
        assert np.array_equal(a[key], b[key]), key
    assert a["estimate"] == b["estimate"]


def test_batch_coloring_and_dense(ctx):
    _say("case batch of colouring probes and of dense probes")
    cases = [synth.watts_strogatz(2000, 10, 0.1, 31), synth.erdos_renyi(800, 5.0, 32),
             synth.grid2d_graph(30, 17)]
    regs, qs, refs = [], [], []
    for n, e in cases:
        g = vne.laplacian_from_edges(n, e, np.float32)
        ref = oracle.laplacian_from_edges(n, e)
        gid = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
        col, s = vne.color_greedy(g["row_ptr"], g["col_idx"], g["values"], 2)
        want_col, want_s = oracle.greedy_distance_coloring(ref.row_ptr, ref.col_idx, ref.n, 2)
        assert np.array_equal(col, want_col) and s == want_s
        qs.append(dict(gid=gid, kind=vne.PROBE_COLORING, m=s, k=30, colors=col))
        regs.append(gid)
        refs.append((ref, col, s))
    outs = ctx.estimate_batch(qs, vne.MODE_DESING)
    for (ref, col, s), out in zip(refs, outs):
        P = oracle.indicator_block(col, s)
        want = oracle.quadforms(ref.scipy(), P, 30, oracle.breakdown_tau(False))
        _check_quad(out, want, False, sens=_order_sensitivity(ref.scipy(), P, 30, False), n=ref.n)
        assert abs(out["estimate"] - out["quad"].sum()) <= 1e-13 * abs(out["estimate"])
    # dense N(0,1) blocks of different widths, FP64, no centring
    rng = np.random.default_rng(3)
    dq, blocks = [], []
    for gid, (ref, _, _), m in zip(regs, refs, (3, 17, 9)):
        B = rng.standard_normal((ref.n, m))
        blocks.append(B)
        dq.append(dict(gid=gid, kind=vne.PROBE_DENSE, m=m, k=25, dense=B))
    # FP64 vectors need FP64 matrices: register FP64 copies
    dq64 = []
    for (n, e), q in zip(cases, dq):
        g = vne.laplacian_from_edges(n, e, np.float64)
        gid = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
        dq64.append(dict(q, gid=gid))
    outs = ctx.estimate_batch(dq64, vne.MODE_F64)
    for (ref, _, _), B, out in zip(refs, blocks, outs):
        want = oracle.quadforms(ref.scipy(), B, 25, oracle.breakdown_tau(True), desing=False)
        _check_quad(out, want, True, sens=_order_sensitivity(ref.scipy(), B, 25, True, desing=False),
                    n=ref.n)


def test_batch_tile_choice_within_tolerance(ctx, monkeypatch):
    # the autotuned column tile and a forced one sum in different orders only
    _say("case batch autotuned tile vs forced tiles")
    cases = _graphs()[:4]
    regs = _register_all(ctx, cases, False)
    qs = [dict(gid=gid, kind=vne.PROBE_RADEMACHER, m=64, k=12, seed=7 + i)
          for i, (_, gid, _, _, _) in enumerate(regs)]
    base = ctx.estimate_batch(qs, vne.MODE_DESING)
    for tile in ("16", "64"):
        monkeypatch.setenv("VNE_TILE", tile)
        other = ctx.estimate_batch(qs, vne.MODE_DESING)
        for i, ((name, gid, ref, _, _), a, b) in enumerate(zip(regs, base, other)):
            B = oracle.rademacher_block(7 + i, ref.node_ids, np.arange(64))
            sens = _order_sensitivity(ref.scipy(), B, 12, False)
            assert np.array_equal(a["k_eff"], b["k_eff"])
            _assert_within(_rel(a["quad"], b["quad"]), _bar(False, sens), "tile %s vs autotuned" % tile)


def test_batch_errors_and_release(ctx, monkeypatch):
    _say("case batch error paths and release")
    # one column tile for every set: a graph's work blocks and per-graph sums
    # do not depend on the other graphs of the batch, so its results are
    # bitwise the same in any batch that runs the same tile
    monkeypatch.setenv("VNE_TILE", "16")
    regs = _register_all(ctx, _graphs()[:3], False)
    ids = [r[1] for r in regs]
    q = [dict(gid=g, kind=vne.PROBE_RADEMACHER, m=4, k=5, seed=1) for g in ids]
    with pytest.raises(vne.VneError) as ei:
        ctx.estimate_batch([dict(q[0], kind=vne.PROBE_HUTCHPP)] + q[1:], vne.MODE_DESING)
    assert ei.value.status == -4
    with pytest.raises(vne.VneError) as ei:
        ctx.estimate_batch([q[0], dict(q[1], kind=vne.PROBE_DENSE, dense=np.zeros((regs[1][2].n, 4)))],
                           vne.MODE_DESING)
    assert ei.value.status == -4
    with pytest.raises(vne.VneError) as ei:
        ctx.estimate_batch([q[0], dict(q[1], gid=10 ** 6)], vne.MODE_DESING)
    assert ei.value.status == -1
    with pytest.raises(vne.VneError) as ei:
        ctx.estimate_batch([q[0], dict(q[1], k=0)], vne.MODE_DESING)
    assert ei.value.status == -1
    with pytest.raises(vne.VneError) as ei:
        ctx.estimate_batch(q, 1 << 5)
    assert ei.value.status == -1
    before = ctx.estimate_batch(q, vne.MODE_DESING)
    ctx.release(ids[0])
    with pytest.raises(vne.VneError):
        ctx.estimate_batch(q, vne.MODE_DESING)
    after = ctx.estimate_batch(q[1:], vne.MODE_DESING)
    for a, b in zip(before[1:], after):
        for key in ("quad", "k_eff", "norm2"):
            assert np.array_equal(a[key], b[key]), key
        assert a["estimate"] == b["estimate"]
