"""Pins of the greedy distance-d colouring (Algorithm 1, eq. (3.3))."""
from collections import deque

import networkx as nx
import numpy as np
import pytest

import oracle
import synth


def _graph(kind, n, seed):
    if kind == "er":
        return oracle.laplacian_from_edges(*synth.erdos_renyi(n, 4.0, seed))
    if kind == "ba":
        return oracle.laplacian_from_edges(*synth.barabasi_albert(n, 2, seed))
    if kind == "ws":
        return oracle.laplacian_from_edges(*synth.watts_strogatz(n, 6, 0.2, seed))
    return oracle.laplacian_from_edges(*synth.grid2d_graph(9, 11))


def _nbrs(g):
    out = []
    for i in range(g.n):
        c = g.col_idx[g.row_ptr[i]:g.row_ptr[i + 1]]
        out.append([int(x) for x in c if x != i])
    return out


def _dist_within(nbr, s, d):
    seen = {s: 0}
    q = deque([s])
    while q:
        x = q.popleft()
        if seen[x] == d:
            continue
        for y in nbr[x]:
            if y not in seen:
                seen[y] = seen[x] + 1
                q.append(y)
    return seen


@pytest.mark.parametrize("kind", ["er", "ba", "ws", "grid"])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_valid_and_bounded(kind, d):
    g = _graph(kind, 150, 7)
    col, s = oracle.greedy_distance_coloring(g.row_ptr, g.col_idx, g.n, d)
    nbr = _nbrs(g)
    for i in range(g.n):
        for j, dist in _dist_within(nbr, i, d).items():
            if j != i:
                assert col[i] != col[j]
    delta = max(len(x) for x in nbr)
    assert s <= delta ** d + 1
    assert set(np.unique(col)) == set(range(s))


@pytest.mark.parametrize("kind", ["er", "ba", "ws"])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_matches_first_fit_on_power_graph(kind, d):
    g = _graph(kind, 200, 8)
    col, _ = oracle.greedy_distance_coloring(g.row_ptr, g.col_idx, g.n, d)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    for i, nb in enumerate(_nbrs(g)):
        G.add_edges_from((i, j) for j in nb)
    deg = dict(G.degree())
    order = sorted(range(g.n), key=lambda i: (-deg[i], i))
    Gd = nx.power(G, d)
    ref = nx.greedy_color(Gd, strategy=lambda _g, _c: iter(order))
    assert all(col[i] == ref[i] for i in range(g.n))


@pytest.mark.parametrize("n,k,d", [(35, 4, 2), (50, 6, 3), (66, 10, 1)])
def test_ring_lattice_gives_banded_colouring(n, k, d):
    # all degrees equal: order is 0..n-1; with n a multiple of d*k/2 + 1 the
    # greedy colouring is the banded colouring (3.3) and uses d*beta + 1 colours
    g = oracle.laplacian_from_edges(*synth.ring_lattice(n, k))
    beta = k // 2
    col, s = oracle.greedy_distance_coloring(g.row_ptr, g.col_idx, g.n, d)
    assert s == d * beta + 1
    assert np.array_equal(col, np.arange(n) % (d * beta + 1))
