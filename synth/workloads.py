"""Seeds and sizes of the synthetic workloads.

The paper measures on SuiteSparse networks (its Table 1) that are not
available here; these seeded random graphs of the same families and size
range stand in for them: Erdos-Renyi and Barabasi-Albert for small-world
networks, Watts-Strogatz for a rewired ring, ring lattices and 2D grids for
large-world (road-like) networks.
"""
import numpy as np
from . import graphs

GRAPH_SEED_TINY = 2212
GRAPH_SEED_LARGE = 2213
GRAPH_SEED_PROBING = 2214
GRAPH_SEED_BATCH = 2215
GRAPH_SEED_SERVE = 2216
PROBE_SEED = 9642


def tiny():
    """ER n=2000, mean degree 8; 30 Rademacher probes, 40 steps, FP64."""
    n, e = graphs.erdos_renyi(2000, 8.0, GRAPH_SEED_TINY)
    return dict(name="er2000_d8_hutchinson30_k40_f64", n_nodes=n, edges=e, graph_seed=GRAPH_SEED_TINY,
                m=30, k=40, probe_seed=PROBE_SEED, fp64=True)


def large():
    """BA n=2e5, 3 edges per new node; Hutch++ 128 sketch + 128 Hutchinson
    Rademacher vectors (256 in one block), 60 steps, FP32 vectors."""
    n, e = graphs.barabasi_albert(200_000, 3, GRAPH_SEED_LARGE)
    return dict(name="ba200k_m3_hutchpp256_k60_f32", n_nodes=n, edges=e, graph_seed=GRAPH_SEED_LARGE,
                n_sketch=128, n_hutch=128, k=60, probe_seed=PROBE_SEED,
                fp64=False)


def probing_eps(graph="ws", n=1_000_000, rel_eps=1e-3):
    """Algorithm 2 (probing with a relative target): the probing graph (WS
    n=1e6, k=10, p=0.1; small-world) or the same ring without rewiring (a
    large-world lattice whose entropy has a closed form), FP32 vectors."""
    if graph == "ring":
        n, e = graphs.ring_lattice(n, 10)
        seed = None
    else:
        n, e = graphs.watts_strogatz(n, 10, 0.1, GRAPH_SEED_PROBING)
        seed = GRAPH_SEED_PROBING
    name = "%s%d_k10%s_alg2_eps%g_f32" % (graph, n, "_p0.1" if graph == "ws" else "", rel_eps)
    return dict(name=name, n_nodes=n, edges=e, graph_seed=seed, rel_eps=rel_eps, graph=graph, fp64=False)


def probing(n=1_000_000):
    """WS n=1e6, k=10, p=0.1; greedy distance-2 coloring, 80 steps, FP32."""
    n, e = graphs.watts_strogatz(n, 10, 0.1, GRAPH_SEED_PROBING)
    return dict(name="ws%d_k10_p0.1_probing_d2_k80_f32" % n, n_nodes=n, graph_seed=GRAPH_SEED_PROBING,
                edges=e, d=2, k=80, fp64=False)


def batch_specs(count=512, seed=GRAPH_SEED_BATCH):
    """Sizes and families of the multi-graph batch: n log-uniform in
    [1e3, 5e4], half ER (mean degree U[4,16]), half BA (2..5 edges/node)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for g in range(count):
        n = int(round(np.exp(rng.uniform(np.log(1e3), np.log(5e4)))))
        if g % 2 == 0:
            specs.append(("er", n, float(rng.uniform(4.0, 16.0)), seed * 1000 + g))
        else:
            specs.append(("ba", n, int(rng.integers(2, 6)), seed * 1000 + g))
    return specs


def batch_graph(spec):
    fam, n, par, s = spec
    if fam == "er":
        return graphs.erdos_renyi(n, par, s)
    return graphs.barabasi_albert(n, par, s)


def serve_pool_specs(count, n_min=1000, n_max=2_000_000, seed=GRAPH_SEED_SERVE):
    """Graph pool for the serving workload: family uniform in {ER, BA, WS},
    n log-uniform in [n_min, n_max], mean degree U[4, 20]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for g in range(count):
        fam = ("er", "ba", "ws")[int(rng.integers(0, 3))]
        n = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
        deg = float(rng.uniform(4.0, 20.0))
        specs.append((fam, n, deg, seed * 1000 + g))
    return specs


def serve_graph(spec):
    fam, n, deg, s = spec
    if fam == "er":
        return graphs.erdos_renyi(n, deg, s)
    if fam == "ba":
        return graphs.barabasi_albert(n, max(1, int(round(deg / 2))), s)
    k = max(2, 2 * int(round(deg / 2)))
    return graphs.watts_strogatz(n, k, 0.1, s)
