"""Writes hutchpp_adaptive_large.json: the oracle's adaptive Hutch++
(oracle/adaptive_hutchpp.py: the target of eq. (3.10), the adaptive Hutch++
implementation of Section 5, as that module reads them) on the large
workload's graph (Barabasi-Albert n = 2e5, 3 edges per new node, 60 Lanczos
steps, desingularized start vectors, the FP32 breakdown threshold) at a
relative target of 1e-2 and delta = 1e-2.

Every round and the final run are computed in four row orders (the graph's
own, reversed, two seeded random permutations; rows and columns of A and
the rows of the probes permuted alike, so only the rounding order changes).
The values stored are those of the graph's own order, each with its spread
over the four orders (its rounding-order sensitivity), as in
make_hutchpp_large.py.

Calls only the oracle and the seeded input generators.  Run from the repo
root:  python tests/golden/make_hutchpp_adaptive_large.py   (about a
minute; the four orders run in parallel processes, one core each).
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hutchpp_adaptive_large.json")
ORDERS = ("own", "reversed", "perm1", "perm2")
REL_EPS, DELTA = 1e-2, 1e-2


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
    from oracle.adaptive_hutchpp import adaptive_hutchpp
    w, ref = _problem()
    P = _perm(name, ref.n)
    A = sp.csr_matrix(ref.scipy())[P][:, P]
    keys = ref.node_ids[P]
    t0 = time.perf_counter()
    out = adaptive_hutchpp(A, keys, w["probe_seed"], w["k"], eps=REL_EPS, delta=DELTA, fp64_tau=False)
    # the pilot forms of every round (the oracle keeps only the final run's)
    pilots = []
    for r in out["rounds"]:
        Om = oracle.rademacher_block(w["probe_seed"], keys, np.arange(r["nr"]))
        G = oracle.rademacher_block(w["probe_seed"], keys, np.arange(128, 144))
        est, det = oracle.hutchpp(A, Om, G, w["k"], oracle.breakdown_tau(False))
        assert est == r["estimate"]
        pilots.append(det["psi"][r["nr"]:].tolist())
    print("  order %-8s %.1f s, estimate %.15g, rounds %s" % (
        name, time.perf_counter() - t0, out["estimate"], [(r["nr"], r["nh"]) for r in out["rounds"]]), flush=True)
    return dict(estimate=out["estimate"], n_sketch=out["n_sketch"], n_hutch=out["n_hutch"],
                psi=out["psi"].tolist(), rounds=out["rounds"], pilots=pilots, krylov_runs=out["krylov_runs"])


def main():
    w, ref = _problem()
    print("BA n=%d nnz=%d, adaptive Hutch++ rel_eps %g delta %g, k=%d, orders %s"
          % (ref.n, ref.nnz, REL_EPS, DELTA, w["k"], ", ".join(ORDERS)), flush=True)
    with mp.get_context("spawn").Pool(len(ORDERS)) as pool:
        runs = dict(zip(ORDERS, pool.map(run_order, ORDERS)))
    own = runs["own"]
    for o in ORDERS:
        # the decisions must not depend on the rounding order
        assert [(r["nr"], r["nh"]) for r in runs[o]["rounds"]] == [(r["nr"], r["nh"]) for r in own["rounds"]], o
    rounds = []
    for i, r in enumerate(own["rounds"]):
        est = np.array([runs[o]["rounds"][i]["estimate"] for o in ORDERS])
        sd = np.array([runs[o]["rounds"][i]["sd"] for o in ORDERS])
        pil = np.array([runs[o]["pilots"][i] for o in ORDERS])
        rounds.append(dict(nr=r["nr"], nh=r["nh"], eps_hat=r["eps_hat"], estimate=r["estimate"],
                           estimate_spread=float(est.max() - est.min()), sd=r["sd"],
                           sd_spread=float(sd.max() - sd.min()), pilot=own["pilots"][i],
                           pilot_spread=(pil.max(axis=0) - pil.min(axis=0)).tolist()))
    psi = np.array([runs[o]["psi"] for o in ORDERS])
    est = np.array([runs[o]["estimate"] for o in ORDERS])
    sum_q = psi[:, :own["n_sketch"]].sum(axis=1)
    out = dict(
        workload=w["name"].replace("hutchpp256", "hutchpp_adaptive"), n=int(ref.n), nnz=int(ref.nnz), k=w["k"],
        probe_seed=w["probe_seed"], graph_seed=w["graph_seed"], rel_eps=REL_EPS, delta=DELTA, orders=list(ORDERS),
        rounds=rounds, n_sketch=own["n_sketch"], n_hutch=own["n_hutch"], krylov_runs=own["krylov_runs"],
        estimate=own["estimate"], estimate_spread=float(est.max() - est.min()),
        sum_q=float(sum_q[0]), sum_q_spread=float(sum_q.max() - sum_q.min()),
        psi=own["psi"], psi_spread=(psi.max(axis=0) - psi.min(axis=0)).tolist(),
        made_by="tests/golden/make_hutchpp_adaptive_large.py (oracle.adaptive_hutchpp in four row orders)")
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote %s: estimate %.15g, spread %.1e, N_r %d, N_H %d"
          % (OUT, out["estimate"], out["estimate_spread"], out["n_sketch"], out["n_hutch"]), flush=True)


if __name__ == "__main__":
    main()
