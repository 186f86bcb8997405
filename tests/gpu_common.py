"""Helpers of the GPU parity tests: context fixture, registration of a
graph on both sides, the per-quadratic-form bar and the oracle's own
rounding-order sensitivity."""
import numpy as np
import pytest

import oracle
import paper_2212_09642_amd as vne

TOL = {True: 1e-12, False: 1e-5}
# A column whose oracle value is itself rounding-sensitive gets the bar
# C_SENS times its own spread over the oracle's row orders (per column).
C_SENS = 5.0


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = vne.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True)


def _setup(ctx, n, e, fp64=True):
    g = vne.laplacian_from_edges(n, e, np.float64 if fp64 else np.float32)
    ref = oracle.laplacian_from_edges(n, e)
    gid = ctx.register(g["row_ptr"], g["col_idx"], g["values"], g["scale"], node_keys=g["node_ids"])
    return gid, ref


def _rel(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def _orders(n):
    """Row orders of the sensitivity runs besides the identity: reversed and
    two seeded random permutations."""
    return [np.arange(n)[::-1].copy(), np.random.default_rng(1001).permutation(n),
            np.random.default_rng(1002).permutation(n)]


def _spread(values, ref):
    """Per-entry relative spread (largest minus smallest) of the oracle's
    values over its row orders."""
    v = np.array(values, dtype=np.float64)
    return (v.max(axis=0) - v.min(axis=0)) / np.maximum(np.abs(ref), 1e-300)


def _order_sensitivity(A, B, k, fp64, desing=True):
    """Relative spread of the oracle's own psi_k over four row orders (the
    identity, reversed, two random permutations: the same problem with a
    different rounding order only).  After a Ritz value converges, plain
    Lanczos loses orthogonality and psi_k becomes sensitive to rounding at
    the level of its remaining quadrature error; no implementation can then
    agree with the oracle more closely than the oracle agrees with itself.
    Returns one value per column."""
    import scipy.sparse as sp
    n = A.shape[0]
    A = sp.csr_matrix(A)
    B = np.asarray(B)
    tau = oracle.breakdown_tau(fp64)
    base = oracle.quadforms(A, B, k, tau, desing)["psi"]
    runs = [base] + [oracle.quadforms(A[P][:, P], B[P], k, tau, desing)["psi"] for P in _orders(n)]
    return _spread(runs, base)


def _bar(fp64, sens=None):
    """Per-column bar: TOL, or C_SENS times the column's own spread where
    that is larger."""
    if sens is None:
        return TOL[fp64]
    return np.maximum(TOL[fp64], C_SENS * np.asarray(sens, dtype=np.float64))


def _assert_within(rel, bar, what=""):
    rel = np.atleast_1d(np.asarray(rel, dtype=np.float64))
    bar = np.broadcast_to(np.asarray(bar, dtype=np.float64), rel.shape)
    margin = float(np.max(rel / bar)) if rel.size else 0.0
    _say("   %smax rel err %.3e, worst err/bar %.3f (bar %.1e..%.1e)"
         % (what + ": " if what else "", rel.max() if rel.size else 0.0, margin, bar.min(), bar.max()))
    assert np.all(rel < bar), (what, rel.max(), margin)


def _check_quad(out, want, fp64, k_exact=True, sens=None, n=0):
    """Per-quadratic-form bar: 1e-12 (FP64 vectors) or 1e-5 (FP32 vectors),
    per column widened to C_SENS times that column's rounding-order spread
    where given."""
    rel = _rel(out["quad"], want["psi"])
    _assert_within(rel, _bar(fp64, sens), "quad")
    if k_exact:
        assert np.array_equal(out["k_eff"], want["k_eff"])
    # ||c||^2 sums n terms: either side may carry up to about n u of rounding
    rt = max(1e-13, 4 * n * 2.0 ** -53) if fp64 else 1e-6
    assert np.allclose(out["norm2"], want["norm2"], rtol=rt, atol=0)


def _hutchpp_oracle(A, Om, G, k, fp64, desing=True):
    """oracle.hutchpp in the graph's own row order, plus the relative spread
    of its estimate, of each quadratic form and of the sum over Q across the
    four row orders of _order_sensitivity."""
    import scipy.sparse as sp
    A = sp.csr_matrix(A)
    Om, G = np.asarray(Om), np.asarray(G)
    tau = oracle.breakdown_tau(fp64)
    est, det = oracle.hutchpp(A, Om, G, k, tau, desing)
    nr = Om.shape[1]
    ests, psis = [est], [det["psi"]]
    for P in _orders(A.shape[0]):
        e, d = oracle.hutchpp(A[P][:, P], Om[P], G[P], k, tau, desing)
        ests.append(e)
        psis.append(d["psi"])
    sq = [p[:nr].sum() for p in psis]
    sens = dict(estimate=float(_spread(ests, est)[()]), psi=_spread(psis, det["psi"]),
                sum_q=float(_spread(sq, sq[0])[()]))
    return est, det, sens


def _check_hutchpp(out, est, det, sens, nr, fp64):
    """Hutch++ parity: the estimate, the sum of the Q forms (it depends only
    on span(Q)), and each G~ form, each within TOL or C_SENS times its own
    spread.  With FP64 vectors also the Q forms one by one (Q is unique up
    to column signs, and psi(-q) = psi(q)); with FP32 vectors the sketch
    Y = f(A) Omega carries FP32 rounding into the individual columns of Q
    (amplified by the conditioning of Y), which the sum over Q does not
    see, so those are printed only."""
    _assert_within(abs(out["estimate"] - est) / abs(est), _bar(fp64, sens["estimate"]), "estimate")
    sq = det["psi"][:nr].sum()
    _assert_within(abs(out["quad"][:nr].sum() - sq) / abs(sq), _bar(fp64, sens["sum_q"]), "sum over Q")
    rq = _rel(out["quad"][:nr], det["psi"][:nr])
    if fp64:
        _assert_within(rq, _bar(fp64, sens["psi"][:nr]), "Q forms")
    else:
        _say("   Q forms one by one (not asserted with FP32 vectors): max rel err %.3e" % rq.max())
    if det["psi"].size > nr:
        _assert_within(_rel(out["quad"][nr:], det["psi"][nr:]), _bar(fp64, sens["psi"][nr:]), "G~ forms")


def _model_tile(m, fp64, n, nnz):
    """The column tile a plan takes without the autotuner: the cheapest, under
    a byte model of one step (six streams of the padded block, and per tile
    the CSR and one gather of at least a 128-byte line per entry), among the
    power-of-two tiles (from one lane per row: 4 FP32 / 2 FP64 columns) and,
    for FP32, the three-column tiles 12..96 (192 for m = 192); ties go to the
    wider tile."""
    es, cpl = (8, 2) if fp64 else (4, 4)
    cands = []
    t = cpl
    while t <= (64 if fp64 else 128):
        cands.append(t)
        t *= 2
    if not fp64:
        cands += [12, 24, 48, 96] + ([192] if m == 192 else [])
    best, best_cost = 0, 0.0
    for t in cands:
        mp = -(-m // t) * t
        cost = 6.0 * n * mp * es + (mp // t) * float(nnz) * (8.0 + max(t * es, 128))
        if best == 0 or cost < best_cost or (cost == best_cost and t > best):
            best, best_cost = t, cost
    return best
