"""Pins of the oracle's density-matrix builder (eq. (2.3), Section 6.1)."""
from collections import deque

import numpy as np
import pytest

import oracle
import synth


def _bfs_components(n, edges):
    nbr = [set() for _ in range(n)]
    for u, v in edges:
        if u != v:
            nbr[u].add(v)
            nbr[v].add(u)
    seen = [-1] * n
    comps = []
    for s in range(n):
        if seen[s] >= 0:
            continue
        q = deque([s])
        seen[s] = len(comps)
        comp = [s]
        while q:
            x = q.popleft()
            for y in nbr[x]:
                if seen[y] < 0:
                    seen[y] = len(comps)
                    comp.append(y)
                    q.append(y)
        comps.append(sorted(comp))
    return comps, nbr


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_lcc_matches_breadth_first_search(seed):
    n, e = synth.erdos_renyi(120, 1.3, seed)          # sparse: many components
    g = oracle.laplacian_from_edges(n, e)
    comps, nbr = _bfs_components(n, e.tolist())
    best = max(comps, key=lambda c: (len(c), -c[0]))
    assert g.node_ids.tolist() == best
    # every row: diagonal = degree, off-diagonals -1 on the BFS neighbours
    pos = {v: i for i, v in enumerate(best)}
    for i, v in enumerate(best):
        cols = g.col_idx[g.row_ptr[i]:g.row_ptr[i + 1]]
        vals = g.values[g.row_ptr[i]:g.row_ptr[i + 1]]
        expect = sorted([pos[w] for w in nbr[v]] + [i])
        assert cols.tolist() == expect
        assert vals[cols == i][0] == len(nbr[v])
        assert np.all(vals[cols != i] == -1.0)


def test_component_tie_goes_to_smallest_id():
    # two disjoint triangles: both of size 3, the first holds node 0
    e = np.array([[3, 4], [4, 5], [5, 3], [0, 1], [1, 2], [2, 0]])
    g = oracle.laplacian_from_edges(6, e)
    assert g.node_ids.tolist() == [0, 1, 2]


def test_self_loops_and_duplicates_are_dropped():
    n, e = synth.cycle_graph(9)
    noisy = np.concatenate([e, e[::-1, ::-1], np.array([[2, 2], [5, 5]]), e[:3]])
    a = oracle.laplacian_from_edges(n, e)
    b = oracle.laplacian_from_edges(n, noisy)
    for f in ("row_ptr", "col_idx", "values", "node_ids"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    assert a.scale == b.scale == 1.0 / 18


@pytest.mark.parametrize("maker", [lambda: synth.erdos_renyi(300, 6.0, 11),
                                   lambda: synth.barabasi_albert(300, 3, 12),
                                   lambda: synth.watts_strogatz(300, 6, 0.2, 13),
                                   lambda: synth.grid2d_graph(7, 9)])
def test_density_matrix_properties(maker):
    n, e = maker()
    g = oracle.laplacian_from_edges(n, e)
    rho = oracle.dense_matrix(g)
    assert np.allclose(rho, rho.T, atol=0)
    assert np.abs(rho.sum(axis=1)).max() < 1e-15           # L 1 = 0
    assert abs(np.trace(rho) - 1.0) < 1e-14                  # unit trace
    assert np.linalg.eigvalsh(rho).min() > -1e-15            # PSD
    assert g.scale == 1.0 / g.values[g.col_idx == np.repeat(np.arange(g.n), np.diff(g.row_ptr))].sum()


def test_two_components_keeps_the_larger():
    n, e = synth.two_components(5, 12)
    g = oracle.laplacian_from_edges(n, e)
    assert g.n == 12 and g.node_ids.tolist() == list(range(5, 17))
