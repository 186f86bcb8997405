"""Writes hutchpp_large.json: the oracle's Hutch++ estimate (eq. (3.9), with
f(A) Omega by eq. (4.3)) of the large workload (Barabasi-Albert n = 2e5,
3 edges per new node, 128 sketch + 128 Hutchinson Rademacher vectors,
60 Lanczos steps, desingularized start vectors).

The same problem is computed in four row orders: the graph's own, reversed,
and two seeded random permutations (rows and columns of A and the rows of
the probes permuted alike, so only the rounding order changes).  The values
stored are those of the graph's own order; the spread (largest minus
smallest) of each value over the four orders is its rounding-order
sensitivity.  Once Ritz values converge, plain Lanczos loses orthogonality
and its quadratic forms become sensitive to rounding at the level of their
remaining quadrature error; no implementation of the same recurrence can be
held closer to the oracle than that.

Calls only the oracle and the seeded input generators.  Run from the repo
root:  python tests/golden/make_hutchpp_large.py   (about five minutes; the
four orders run in parallel processes, one core each).
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hutchpp_large.json")
ORDERS = ("own", "reversed", "perm1", "perm2")


def _problem():
    import oracle
    from synth import workloads
    w = workloads.large()
    ref = oracle.laplacian_from_edges(w["n_nodes"], w["edges"])
    return w, ref


def _perm(name, n):
    if name == "own":
        return np.arange(n)
    if name == "reversed":
        return np.arange(n)[::-1].copy()
    return np.random.default_rng(1000 + int(name[-1])).permutation(n)


def run_order(name):
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import scipy.sparse as sp
    import oracle
    w, ref = _problem()
    nr, nh, k, seed = w["n_sketch"], w["n_hutch"], w["k"], w["probe_seed"]
    P = _perm(name, ref.n)
    A = sp.csr_matrix(ref.scipy())[P][:, P]
    keys = ref.node_ids[P]
    Om = oracle.rademacher_block(seed, keys, np.arange(nr))
    G = oracle.rademacher_block(seed, keys, np.arange(nr, nr + nh))
    t0 = time.perf_counter()
    est, det = oracle.hutchpp(A, Om, G, k, oracle.breakdown_tau(False))
    Q = det["Q"]
    orth = float(np.abs(Q.T @ Q - np.eye(nr)).max())
    print("  order %-8s %.1f s, estimate %.15g" % (name, time.perf_counter() - t0, est), flush=True)
    return dict(estimate=est, psi=det["psi"].tolist(), k_eff=det["quad"]["k_eff"].tolist(), orth=orth)


def main():
    w, ref = _problem()
    print("BA n=%d nnz=%d, Hutch++ %d + %d, k=%d, orders %s"
          % (ref.n, ref.nnz, w["n_sketch"], w["n_hutch"], w["k"], ", ".join(ORDERS)), flush=True)
    with mp.get_context("spawn").Pool(len(ORDERS)) as pool:
        runs = dict(zip(ORDERS, pool.map(run_order, ORDERS)))
    nr = w["n_sketch"]
    own = runs["own"]
    psi = np.array([runs[o]["psi"] for o in ORDERS])
    est = np.array([runs[o]["estimate"] for o in ORDERS])
    sum_q = psi[:, :nr].sum(axis=1)
    out = dict(
        workload=w["name"], n=int(ref.n), nnz=int(ref.nnz), n_sketch=nr, n_hutch=w["n_hutch"], k=w["k"],
        probe_seed=w["probe_seed"], graph_seed=w["graph_seed"], orders=list(ORDERS),
        estimate=own["estimate"], estimate_spread=float(est.max() - est.min()),
        sum_q=float(sum_q[0]), sum_q_spread=float(sum_q.max() - sum_q.min()),
        psi=own["psi"], psi_spread=(psi.max(axis=0) - psi.min(axis=0)).tolist(),
        k_eff=own["k_eff"], q_orthogonality=max(runs[o]["orth"] for o in ORDERS),
        made_by="tests/golden/make_hutchpp_large.py (oracle.hutchpp in four row orders)")
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote %s: estimate %.15g, spread %.1e; max psi spread %.1e"
          % (OUT, out["estimate"], out["estimate_spread"], max(out["psi_spread"])), flush=True)


if __name__ == "__main__":
    main()
