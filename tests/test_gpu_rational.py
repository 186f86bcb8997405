"""GPU parity of the rational Krylov cross-check (vne_rational_quadforms;
Section 4, eq. (4.1) and (4.2); the switch rule of the Krylov method
implementation, Section 5) against the oracle's rational_run, through the C
ABI.  FP64 only.

Bar: 1e-10 relative per form and step.  The shifted systems are solved by
conjugate gradients to a relative residual of 1e-12 (the oracle solves them
directly); the Rayleigh-Ritz form depends on the basis only through the
space it spans and moved by less than 4e-14 between the two solvers on the
path, grid and Barabasi-Albert cases below in an FP64 CPU emulation, so the
bar leaves the rest to the GPU's reduction order.  Integer results (basis
size, switch step, applications of A with poles at infinity) are compared
exactly.
"""
import numpy as np
import pytest

import oracle
import synth
import paper_2212_09642_amd as vne
from oracle.rational import default_poles, rational_run, switch_step

pytestmark = pytest.mark.gpu

from gpu_common import ctx, _say, _setup  # noqa: F401

RTOL = 1e-10
CG_TOL = 1e-12
MODE = vne.MODE_F64 | vne.MODE_DESING


def _start(ref, seed, m):
    B = oracle.rademacher_block(seed, ref.node_ids, np.arange(m))
    return oracle.desingularize(B)


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(np.abs(b), 1e-300)


def _check_steps(out, runs, steps, skip=()):
    worst = 0.0
    for c, r in enumerate(runs):
        if c in skip:
            continue
        want = np.array(r["psi"])
        err = _rel(out["psi_steps"][c], want)
        worst = max(worst, float(err.max()))
        assert np.all(err <= RTOL), (c, err.max())
        assert out["basis"][c] == r["basis"], c
        assert _rel(out["quad"][c], want[-1]) <= RTOL
    _say("  worst rel err %.2e (bar %.0e) over %d columns x %d steps" % (worst, RTOL, len(runs), steps))


def test_explicit_poles_barabasi_albert(ctx):
    n, e = synth.barabasi_albert(400, 3, 11)
    _say("case rational explicit poles BA n=400 m=5 steps=12")
    gid, ref = _setup(ctx, n, e)
    A = ref.scipy().toarray()
    lam = np.linalg.eigvalsh(A)
    steps, m = 12, 5
    poles = default_poles(steps, 3, lam[1], lam[-1])
    out = ctx.rational(gid, vne.PROBE_RADEMACHER, m, MODE, steps, poles=poles, cg_tol=CG_TOL, seed=3)
    C = _start(ref, 3, m)
    assert np.allclose(out["norm2"], np.sum(C * C, axis=0), rtol=1e-13, atol=0)
    runs = [rational_run(A, C[:, c], steps, poles=poles) for c in range(m)]
    _check_steps(out, runs, steps)
    # applications of A: one per basis vector, plus every CG iteration of
    # the finite-pole steps; the poles at infinity of steps 1-3 add none
    ap = out["apps_steps"]
    assert np.array_equal(ap[:, :4], np.tile(np.arange(1, 5), (m, 1)))
    assert np.all(np.diff(ap, axis=1) >= 1)
    assert int((ap[:, -1] - steps).sum()) == out["cg_iterations"] > 0
    assert np.all(out["switch_step"] == 0)


def test_all_poles_at_infinity_is_the_polynomial_path(ctx):
    n, e = synth.erdos_renyi(500, 6.0, 21)
    _say("case rational all poles at infinity ER n=500 m=6 steps=10")
    gid, ref = _setup(ctx, n, e)
    A = ref.scipy().toarray()
    steps, m = 10, 6
    out = ctx.rational(gid, vne.PROBE_RADEMACHER, m, MODE, steps, poles=[np.inf] * (steps - 1), seed=8)
    C = _start(ref, 8, m)
    runs = [rational_run(A, C[:, c], steps, poles=[np.inf] * (steps - 1)) for c in range(m)]
    _check_steps(out, runs, steps)
    assert np.array_equal(out["apps_steps"], np.tile(np.arange(1, steps + 1), (m, 1)))
    assert out["cg_iterations"] == 0
    # the same forms from the Lanczos path (no reorthogonalization needed
    # this early on a well-conditioned graph)
    poly = ctx.estimate(gid, vne.PROBE_RADEMACHER, m, steps, MODE, seed=8)
    assert np.all(_rel(out["quad"], poly["quad"]) <= 1e-11)


@pytest.mark.parametrize("estimate", [False, True])
def test_switch_rule_on_a_path(ctx, estimate):
    n, e = synth.path_graph(300)
    _say("case rational switch rule path n=300 m=4 steps=24 ell=3 c=0.75 estimate=%s" % estimate)
    gid, ref = _setup(ctx, n, e)
    A = ref.scipy().toarray()
    lam = np.linalg.eigvalsh(A)
    lo, hi = 0.999 * lam[1], 1.001 * lam[-1]
    steps, m = 24, 4
    fin = list(-np.geomspace(lam[-1], lam[1], 12))
    out = ctx.rational(gid, vne.PROBE_RADEMACHER, m, MODE, steps, finite_poles=fin, ell=3, c=0.75,
                       cg_tol=CG_TOL, seed=5, lam_lo=lo, lam_hi=hi, estimate=estimate)
    C = _start(ref, 5, m)
    runs = [rational_run(A, C[:, c], steps, finite_poles=fin, ell=3, c=0.75, lam_lo=lo, lam_hi=hi,
                         estimate=estimate) for c in range(m)]
    flipped = set()
    worst = 0.0
    for c, r in enumerate(runs):
        s_gpu, s_ora = int(out["switch_step"][c]), r["switch"]
        # the bounds of the polynomial steps: Theorem 4.8 on both sides (the
        # device's integral route against the oracle's residue form)
        j_max = min(s_gpu, s_ora) if s_gpu and s_ora else len(r["err"])
        err = _rel(out["err_steps"][c, :j_max], np.array(r["err"][:j_max]))
        worst = max(worst, float(err.max()))
        assert np.all(err <= 1e-6), (c, err.max())
        _say("  column %d: switch at step %d (oracle %d)" % (c, s_gpu, s_ora))
        if s_gpu != s_ora:
            # a decision on bounds that agree to 1e-6 may flip only where the
            # oracle's ratio is within 1e-5 of the threshold
            j = min(v for v in (s_gpu, s_ora) if v > 0)
            ratio = r["err"][j - 1] / (0.75 ** 3 * r["err"][j - 5])
            assert abs(ratio - 1.0) < 1e-5, (c, s_gpu, s_ora, ratio)
            flipped.add(c)
    _say("  worst bound rel err %.2e" % worst)
    assert len(flipped) < m and np.all(out["switch_step"] > 0)
    _check_steps(out, runs, steps, skip=flipped)
    # the GPU's own bounds give its switch step under the rule
    for c in range(m):
        if c not in flipped:
            s = int(out["switch_step"][c])
            assert switch_step(list(out["err_steps"][c, :s]), 3, 0.75) == s
            assert np.all(out["err_steps"][c, s:] == 0.0)


@pytest.mark.parametrize("m", [1, 37, 128])
def test_column_counts_and_colouring(ctx, m):
    n, e = synth.grid2d_graph(12, 15)
    _say("case rational grid 12x15 colouring-free m=%d steps=7" % m)
    gid, ref = _setup(ctx, n, e)
    A = ref.scipy().toarray()
    lam = np.linalg.eigvalsh(A)
    steps = 7
    poles = default_poles(steps, 2, lam[1], lam[-1])
    out = ctx.rational(gid, vne.PROBE_RADEMACHER, m, MODE, steps, poles=poles, cg_tol=CG_TOL, seed=m)
    C = _start(ref, m, m)
    cols = sorted(set([0, m // 2, m - 1]))
    runs = [rational_run(A, C[:, c], steps, poles=poles) for c in cols]
    sub = {k: (v[cols] if isinstance(v, np.ndarray) else v) for k, v in out.items()}
    _check_steps(sub, runs, steps)


def test_colouring_probes_and_invariant_subspace(ctx):
    # a 6-node path: centred indicator vectors live in the 5-dimensional
    # range of the Laplacian, so the basis stops at <= 5 vectors and the
    # later forms are exact
    n, e = synth.path_graph(6)
    _say("case rational path n=6 colouring probes steps=9")
    gid, ref = _setup(ctx, n, e)
    A = ref.scipy().toarray()
    colors = np.array([0, 1, 2, 0, 1, 2], np.int32)
    steps = 9
    out = ctx.rational(gid, vne.PROBE_COLORING, 3, MODE, steps, poles=[np.inf] * (steps - 1), colors=colors)
    C = oracle.desingularize(oracle.indicator_block(colors, 3))
    runs = [rational_run(A, C[:, c], steps, poles=[np.inf] * (steps - 1)) for c in range(3)]
    _check_steps(out, runs, steps)
    exact = oracle.exact_quadform(A, C)
    assert np.all(out["basis"] <= 5)
    assert np.all(_rel(out["quad"], exact) <= 1e-11)


def test_rational_errors(ctx):
    n, e = synth.cycle_graph(40)
    _say("case rational error paths")
    gid, ref = _setup(ctx, n, e)
    bad = [dict(mode=vne.MODE_DESING, status=-4),                       # FP32
           dict(m=129, status=-1), dict(steps=65, status=-1), dict(steps=0, status=-1),
           dict(poles=[1.0, np.inf], steps=3, status=-1),               # positive pole
           dict(poles=[np.nan, -1.0], steps=3, status=-1),
           dict(c=1.0, status=-1), dict(ell=0, status=-1),             # switch rule arguments
           dict(lam_lo=0.0, status=-1), dict(lam_lo=2.0, lam_hi=1.0, status=-1),
           dict(kind=vne.PROBE_HUTCHPP, status=-4)]
    for b in bad:
        kw = dict(kind=vne.PROBE_RADEMACHER, m=4, mode=MODE, steps=5, poles=None, c=0.75, ell=3, lam_lo=1e-3,
                  lam_hi=4.0)
        kw.update(b)
        st = kw.pop("status")
        with pytest.raises(vne.VneError) as ei:
            ctx.rational(gid, kw["kind"], kw["m"], kw["mode"], kw["steps"], poles=kw["poles"],
                         finite_poles=[-1.0], ell=kw["ell"], c=kw["c"], lam_lo=kw["lam_lo"], lam_hi=kw["lam_hi"])
        assert ei.value.status == st, b
    # the context still works
    out = ctx.rational(gid, vne.PROBE_RADEMACHER, 4, MODE, 5, poles=[np.inf] * 4)
    assert np.all(out["basis"] == 5)
