"""Graph density matrix rho = L / tr(L) (paper Section 2, eq. (2.3) and the
scaling relation (2.2); preprocessing of Section 6.1: binary edge weights,
largest connected component, unit trace).

Readings where the paper is silent:
* self loops are dropped and repeated edges count once (binary weights);
* the largest connected component is kept; if several have the largest
  size, the one holding the smallest original node id wins;
* kept nodes are renumbered in increasing order of their original id;
* the CSR stores every diagonal entry explicitly and sorted column indices;
  values are the exact integers of L and the scale is 1 / tr(L) in float64,
  so rho = scale * L.

Pinned by: row sums zero, symmetry, tr(rho) = 1, positive semidefiniteness,
and a brute-force breadth-first search for the component (tests).
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


@dataclass
class GraphCSR:
    n: int
    row_ptr: np.ndarray   # int64[n+1]
    col_idx: np.ndarray   # int64[nnz]
    values: np.ndarray    # float64[nnz], exact integers of L
    node_ids: np.ndarray  # int64[n], original id of each kept node
    scale: float          # 1 / tr(L)

    @property
    def nnz(self):
        return int(self.row_ptr[-1])

    def scipy(self):
        """rho = scale * L as a scipy CSR matrix (float64)."""
        return sp.csr_matrix((self.values * self.scale, self.col_idx, self.row_ptr),
                             shape=(self.n, self.n))

    def laplacian(self):
        return sp.csr_matrix((self.values, self.col_idx, self.row_ptr),
                             shape=(self.n, self.n))


def laplacian_from_edges(n_nodes, edges):
    """Build the graph Laplacian L = D - Adj of the largest connected component.

    eq. (2.3): Adj has ones on edges, D = diag(Adj 1).
    """
    edges = np.asarray(edges, np.int64).reshape(-1, 2)
    u, v = edges[:, 0], edges[:, 1]
    if n_nodes < 1:
        raise ValueError("graph has no nodes")
    if edges.size and (u.min() < 0 or v.min() < 0 or max(u.max(), v.max()) >= n_nodes):
        raise ValueError("edge endpoint out of range")
    off = u != v
    u, v = u[off], v[off]
    adj = sp.coo_matrix((np.ones(2 * u.size), (np.concatenate([u, v]), np.concatenate([v, u]))),
                        shape=(n_nodes, n_nodes)).tocsr()
    adj.sum_duplicates()
    adj.data[:] = 1.0                                     # binary weights
    ncomp, labels = connected_components(adj, directed=False)
    sizes = np.bincount(labels, minlength=ncomp)
    best_size = sizes.max()
    # among the largest components, the one that holds the smallest node id
    first_node = np.full(ncomp, n_nodes, np.int64)
    np.minimum.at(first_node, labels, np.arange(n_nodes))
    cands = np.flatnonzero(sizes == best_size)
    best = cands[np.argmin(first_node[cands])]
    keep = np.flatnonzero(labels == best)                 # ascending original ids
    sub = adj[keep][:, keep].tocsr()
    deg = np.asarray(sub.sum(axis=1)).ravel()
    L = (sp.diags(deg) - sub).tocsr()
    # keep every diagonal entry explicitly (a single-node component has L = [0])
    L = (L + sp.diags(np.full(keep.size, 1.0))).tocsr()
    L.sort_indices()
    L.data[L.indices == np.repeat(np.arange(keep.size), np.diff(L.indptr))] -= 1.0
    trace = float(deg.sum())
    scale = 1.0 / trace if trace > 0 else float("nan")
    return GraphCSR(n=int(keep.size), row_ptr=L.indptr.astype(np.int64),
                    col_idx=L.indices.astype(np.int64), values=L.data.astype(np.float64),
                    node_ids=keep.astype(np.int64), scale=scale)


def dense_matrix(g):
    """rho = scale * L as a dense float64 array (small n only)."""
    return g.scipy().toarray()
