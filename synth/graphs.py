"""Edge-list generators for simple undirected graphs.

Every generator returns ``(n_nodes, edges)`` where ``edges`` is an int64 array
of shape (E, 2).  Edges may come in any order; self loops and duplicates are
possible only where a docstring says so (the Laplacian builders on both sides
drop them).  Random generators take an integer seed and use numpy's PCG64.
"""
import numpy as np


def _pairs(u, v):
    return np.stack([np.asarray(u, np.int64), np.asarray(v, np.int64)], axis=1)


def complete_graph(n):
    """K_n: every pair of distinct nodes is joined."""
    iu, ju = np.triu_indices(n, k=1)
    return n, _pairs(iu, ju)


def star_graph(n):
    """Star S_n: node 0 joined to nodes 1..n-1."""
    return n, _pairs(np.zeros(n - 1, np.int64), np.arange(1, n))


def cycle_graph(n):
    """Cycle C_n (n >= 3)."""
    i = np.arange(n)
    return n, _pairs(i, (i + 1) % n)


def path_graph(n):
    """Path P_n."""
    i = np.arange(n - 1)
    return n, _pairs(i, i + 1)


def grid2d_graph(rows, cols):
    """rows x cols square grid; node id = r * cols + c."""
    r, c = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    node = r * cols + c
    e1 = _pairs(node[:, :-1].ravel(), node[:, 1:].ravel())
    e2 = _pairs(node[:-1, :].ravel(), node[1:, :].ravel())
    return rows * cols, np.concatenate([e1, e2])


def ring_lattice(n, k):
    """Ring lattice: node i joined to i±1, ..., i±k/2 (k even, n > k)."""
    assert k % 2 == 0 and n > k
    i = np.arange(n)
    parts = [_pairs(i, (i + j) % n) for j in range(1, k // 2 + 1)]
    return n, np.concatenate(parts)


def two_components(n1, n2):
    """Disjoint union of a path on n1 nodes and a cycle on n2 nodes, plus one
    isolated node; used to exercise the largest-component extraction."""
    _, e1 = path_graph(n1)
    _, e2 = cycle_graph(n2)
    return n1 + n2 + 1, np.concatenate([e1, e2 + n1])


def erdos_renyi(n, mean_degree, seed):
    """G(n, p) with p = mean_degree / (n - 1).

    The number of edges is drawn from Binomial(n(n-1)/2, p) and that many
    distinct unordered pairs are then drawn uniformly, which has the same law
    as flipping a coin per pair but costs O(E) instead of O(n^2).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    npairs = n * (n - 1) // 2
    p = mean_degree / (n - 1)
    m = int(rng.binomial(npairs, p))
    keys = np.empty(0, np.int64)
    while keys.size < m:
        need = m - keys.size
        u = rng.integers(0, n, size=int(need * 1.1) + 16)
        v = rng.integers(0, n, size=u.size)
        ok = u != v
        lo = np.minimum(u, v)[ok]
        hi = np.maximum(u, v)[ok]
        keys = np.unique(np.concatenate([keys, lo * n + hi]))
        if keys.size > m:
            keys = rng.permutation(keys)[:m]
            keys.sort()
    return n, _pairs(keys // n, keys % n)


def barabasi_albert(n, m_attach, seed):
    """Preferential attachment: start from K_{m+1}; every later node joins m
    distinct existing nodes drawn with probability proportional to degree."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = m_attach
    n0 = m + 1
    _, seed_edges = complete_graph(n0)
    total_endpoints = 2 * (seed_edges.shape[0] + (n - n0) * m)
    ends = np.empty(total_endpoints, np.int64)      # node repeated deg times
    ends[: 2 * seed_edges.shape[0]] = seed_edges.ravel()
    fill = 2 * seed_edges.shape[0]
    new_u = np.empty((n - n0) * m, np.int64)
    new_v = np.empty((n - n0) * m, np.int64)
    w = 0
    # draw uniform positions in bulk; rejection keeps targets distinct
    pool = rng.random(4 * m * (n - n0) + 64)
    pp = 0
    for node in range(n0, n):
        chosen = []
        while len(chosen) < m:
            if pp >= pool.size:
                pool = rng.random(pool.size)
                pp = 0
            t = int(ends[int(pool[pp] * fill)])
            pp += 1
            if t not in chosen:
                chosen.append(t)
        for t in chosen:
            new_u[w] = node
            new_v[w] = t
            w += 1
            ends[fill] = node
            ends[fill + 1] = t
            fill += 2
    return n, np.concatenate([seed_edges, _pairs(new_u, new_v)])


def watts_strogatz(n, k, p, seed):
    """Watts-Strogatz: ring lattice with k/2 neighbours per side; each lattice
    edge (i, i+j) is rewired with probability p to (i, w), w uniform, avoiding
    self loops and existing edges."""
    rng = np.random.Generator(np.random.PCG64(seed))
    _, e = ring_lattice(n, k)
    u = e[:, 0].copy()
    v = e[:, 1].copy()
    rewire = np.flatnonzero(rng.random(u.size) < p)
    keep_mask = np.ones(u.size, bool)
    keep_mask[rewire] = False
    key = lambda a, b: np.minimum(a, b) * n + np.maximum(a, b)
    existing = np.sort(key(u[keep_mask], v[keep_mask]))
    new_v = rng.integers(0, n, size=rewire.size)
    for _ in range(64):
        ku = key(u[rewire], new_v)
        bad = (new_v == u[rewire]) | np.isin(ku, existing)
        # duplicates among the rewired edges themselves
        order = np.argsort(ku, kind="stable")
        dup = np.zeros(rewire.size, bool)
        sk = ku[order]
        dup[order[1:]] = sk[1:] == sk[:-1]
        bad |= dup
        if not bad.any():
            break
        new_v[bad] = rng.integers(0, n, size=int(bad.sum()))
    v[rewire] = new_v
    return n, _pairs(u, v)
