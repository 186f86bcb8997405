"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package only draws random graphs (edge lists) and fixes the seeds and
sizes of the workloads.  It holds none of the entropy method's arithmetic:
no Laplacian, no probe vectors, no Krylov step.  Both the oracle and the HIP
path consume what it returns and build everything else on their own.
"""
from .graphs import (complete_graph, star_graph, cycle_graph, path_graph,
                     grid2d_graph, ring_lattice, erdos_renyi, barabasi_albert,
                     watts_strogatz, two_components)
from . import workloads

__all__ = ["complete_graph", "star_graph", "cycle_graph", "path_graph",
           "grid2d_graph", "ring_lattice", "erdos_renyi", "barabasi_albert",
           "watts_strogatz", "two_components", "workloads"]
