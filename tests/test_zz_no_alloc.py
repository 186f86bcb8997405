"""The allocation-free estimate (vne_entropy_estimate_noalloc) against the
allocating one (vne_entropy_estimate), through the C ABI: two calls in a row,
the second on a smaller input, each bitwise equal to the allocating entry
point with the same column tile (autotuner off) and within the per-form bar;
colour indicators from a host array; requests beyond the static scratch
array fail with VNE_ENOMEM and leave the context usable."""
import numpy as np
import pytest

import synth
import paper_2212_09642_amd as vne
from gpu_common import TOL, _say, _rel, _assert_within

pytestmark = pytest.mark.gpu


def _reg(c, n, e, fp64):
    g = vne.laplacian_from_edges(n, e, np.float64 if fp64 else np.float32)
    return c.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"]), g


def _same(a, b, fp64, what):
    _assert_within(_rel(a["quad"], b["quad"]), TOL[fp64], what)
    for key in ("quad", "alpha", "beta", "k_eff", "norm2"):
        assert np.array_equal(a[key], b[key]), (what, key)
    assert a["estimate"] == b["estimate"], what


@pytest.mark.parametrize("fp64", [False, True])
def test_noalloc_matches_allocating_estimate(fp64, monkeypatch):
    monkeypatch.setenv("VNE_AUTOTUNE", "0")
    mode = vne.MODE_DESING | (vne.MODE_F64 if fp64 else 0)
    with vne.Context(0) as c:
        big, _ = _reg(c, *synth.barabasi_albert(20000, 3, 91), fp64)
        small, gs = _reg(c, *synth.watts_strogatz(3000, 8, 0.1, 92), fp64)
        cases = [(big, 64, 30, 5), (small, 20, 17, 6)]           # the second call is smaller
        before = c.memory()
        for gid, m, k, seed in cases:
            _say("case no-alloc fp64=%s gid=%d m=%d k=%d" % (fp64, gid, m, k))
            na = c.estimate_noalloc(gid, vne.PROBE_RADEMACHER, m, k, mode, seed=seed)
            assert c.memory() == before                              # the context allocated nothing
            ref = c.estimate(gid, vne.PROBE_RADEMACHER, m, k, mode, seed=seed)
            _same(na, ref, fp64, "rademacher m=%d" % m)
            before = c.memory()
        # colour indicators from a host array, after the runs above left the
        # scratch array dirty
        col, s = vne.color_greedy(gs["row_ptr"], gs["col_idx"], gs["values"], 2)
        na = c.estimate_noalloc(small, vne.PROBE_COLORING, s, 25, mode, colors=col)
        ref = c.estimate(small, vne.PROBE_COLORING, s, 25, mode, colors=col)
        _same(na, ref, fp64, "colouring s=%d" % s)
        # beyond the scratch array: VNE_ENOMEM with the bytes it needed, then usable
        with pytest.raises(vne.VneError) as ei:
            c.estimate_noalloc(big, vne.PROBE_RADEMACHER, 1024, 10, mode, seed=1)
        assert ei.value.status == -2 and "scratch" in str(ei.value)
        with pytest.raises(vne.VneError) as ei:
            c.estimate_noalloc(big, vne.PROBE_HUTCHPP, 16, 10, mode, seed=1)
        assert ei.value.status == -4
        again = c.estimate_noalloc(small, vne.PROBE_RADEMACHER, 20, 17, mode, seed=6)
        ref = c.estimate(small, vne.PROBE_RADEMACHER, 20, 17, mode, seed=6)
        _same(again, ref, fp64, "after the refusals")
