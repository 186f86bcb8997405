"""Helpers of the GPU parity tests: context fixture, registration of a
graph on both sides, the per-quadratic-form bar and the oracle's own
rounding-order sensitivity."""
import numpy as np
import pytest

import oracle
import paper_2212_09642_amd as vne

TOL = {True: 1e-12, False: 1e-5}


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


def _order_sensitivity(A, B, k, fp64, desing=True):
    """Relative change of the oracle's own psi_k when the same problem is
    computed with the rows and columns in reverse order (a different rounding
    order only).  After a Ritz value converges, plain Lanczos loses
    orthogonality and psi_k becomes sensitive to rounding at the level of its
    remaining quadrature error; no implementation can then agree with the
    oracle more closely than the oracle agrees with itself."""
    import scipy.sparse as sp
    n = A.shape[0]
    P = np.arange(n)[::-1]
    Ap = sp.csr_matrix(A)[P][:, P]
    a = oracle.quadforms(A, B, k, oracle.breakdown_tau(fp64), desing)["psi"]
    b = oracle.quadforms(Ap, np.asarray(B)[P], k, oracle.breakdown_tau(fp64), desing)["psi"]
    return _rel(b, a)


def _check_quad(out, want, fp64, k_exact=True, sens=None, n=0):
    """Per-quadratic-form bar: 1e-12 (FP64 vectors) or 1e-5 (FP32 vectors),
    widened to 20x the oracle's own rounding-order sensitivity where given."""
    tol = TOL[fp64] if sens is None else max(TOL[fp64], 20 * float(np.max(sens)))
    rel = _rel(out["quad"], want["psi"])
    _say("   max rel err %.3e (bar %.1e, oracle order sensitivity %.1e)"
         % (rel.max(), TOL[fp64], 0.0 if sens is None else np.max(sens)))
    assert np.all(rel < tol), rel.max()
    if k_exact:
        assert np.array_equal(out["k_eff"], want["k_eff"])
    # ||c||^2 sums n terms: either side may carry up to about n u of rounding
    rt = max(1e-13, 4 * n * 2.0 ** -53) if fp64 else 1e-6
    assert np.allclose(out["norm2"], want["norm2"], rtol=rt, atol=0)
