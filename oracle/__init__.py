"""Plain CPU FP64 oracle for Lanczos-quadrature estimation of the von Neumann
entropy (Benzi, Rinelli, Simunec, "Computation of the von Neumann entropy of
large matrices via trace estimators and rational Krylov methods").

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
CPU-baseline leg may import this package.  The HIP library never calls it and
shares no code with it: the two meet only through the seeded edge lists of
the ``synth`` package and through the published definition of the SplitMix64
counter hash, which each side implements on its own.

Everything here is written for a reader checking it against the paper by eye:
NumPy/SciPy in float64, no blocking, no fusion, no reordering beyond what the
cited definitions state.  Parity status of every function is listed in the
module that defines it; a function without an independent pin says
"parity unpinned".
"""
from .laplacian import laplacian_from_edges, GraphCSR, dense_matrix
from .entropy import f_entropy, entropy_from_eigenvalues, exact_entropy, exact_quadform
from .probes import splitmix64_mix, rademacher_block, indicator_block, desingularize
from .lanczos import lanczos, lanczos_full_reorth, breakdown_tau
from .quadrature import gauss_quadrature, f_of_T_e1
from .estimators import hutchinson, probing_sum, hutchpp, quadforms
from .coloring import greedy_distance_coloring, coloring_order
from . import bounds, rational, probing

__all__ = [
    "laplacian_from_edges", "GraphCSR", "dense_matrix", "f_entropy",
    "entropy_from_eigenvalues", "exact_entropy", "exact_quadform",
    "splitmix64_mix", "rademacher_block", "indicator_block", "desingularize",
    "lanczos", "lanczos_full_reorth", "breakdown_tau", "gauss_quadrature",
    "f_of_T_e1", "hutchinson", "probing_sum", "hutchpp", "quadforms",
    "greedy_distance_coloring", "coloring_order", "bounds", "rational", "probing",
]
