"""Greedy distance-d colouring (paper Section 3.1, Algorithm 1).

Nodes are visited in order of descending degree (the ordering the paper
recommends); the paper does not break ties, so equal degrees are visited in
increasing node index.  Degree = number of distinct off-diagonal entries of
the row.  Each node takes the smallest colour not used by an earlier node at
geodesic distance <= d in the graph of the matrix.  Colours are numbered from
0 here (the paper numbers from 1).

The distance-d neighbourhoods come from the sparsity pattern of (|A| + I)^d,
computed with nonnegative pattern arithmetic, which is the route the paper's
own implementation takes ("computing A^d").

Pinned by: validity (same-coloured nodes are more than d apart, checked by
breadth-first search), the Delta^d + 1 bound on the number of colours, the
banded colouring (3.3) on a ring lattice, and an independent first-fit
colouring of the d-th power graph (tests).
"""
import numpy as np
import scipy.sparse as sp


def coloring_order(row_ptr, col_idx, n):
    row_ptr = np.asarray(row_ptr, np.int64)
    col_idx = np.asarray(col_idx, np.int64)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    deg = np.bincount(rows[col_idx != rows], minlength=n)
    return np.lexsort((np.arange(n), -deg)), deg


def greedy_distance_coloring(row_ptr, col_idx, n, d):
    """Returns (colors int64[n], n_colors)."""
    if d < 1:
        raise ValueError("distance must be >= 1")
    row_ptr = np.asarray(row_ptr, np.int64)
    col_idx = np.asarray(col_idx, np.int64)
    P = sp.csr_matrix((np.ones(col_idx.size, np.float64), col_idx, row_ptr), shape=(n, n))
    P = (P + sp.identity(n, format="csr")).tocsr()
    P.data[:] = 1.0
    Pd = P
    for _ in range(d - 1):
        Pd = (Pd @ P).tocsr()
        Pd.data[:] = 1.0
    order, _ = coloring_order(row_ptr, col_idx, n)
    colors = np.full(n, -1, np.int64)
    for i in order:
        nb = Pd.indices[Pd.indptr[i]:Pd.indptr[i + 1]]
        used = colors[nb]
        used = used[(used >= 0) & (used <= nb.size)]
        taken = np.zeros(nb.size + 1, bool)
        taken[used] = True
        colors[i] = int(np.argmin(taken))
    return colors, int(colors.max()) + 1 if n else 0
