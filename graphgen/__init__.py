"""Seeded synthetic graph generators shared by the oracle tests, the GPU tests and the benchmark.

This package holds no Louvain arithmetic. It only builds symmetric CSR graphs (arcs in both
directions, integer weights) from counter-based random draws, so that the same seed gives the
same graph bit for bit on the CPU and on the GPU (every step is integer tensor arithmetic).

The workloads stand in for the paper's dataset (its Table 1: web, social, collaboration and
road graphs from SuiteSparse, made undirected by duplicating each edge in the reverse
direction). Those graphs are not used here; R-MAT stands in for the skewed web/social class,
the planted-partition (SBM) model for community-structured graphs, and lattices with random
shortcuts for road networks.
"""

from .rng import splitmix64_mix, draw, stream_key  # noqa: F401
from .csr import Csr, csr_from_arcs, csr_from_edges, csr_sha256, pack_graphs  # noqa: F401
from .generators import (  # noqa: F401
    rmat,
    rmat_edges,
    sbm,
    lattice_shortcuts,
    ring_of_cliques,
    two_triangles,
    single_edge,
    erdos_renyi,
    add_self_loops,
    planted_hubs,
    batch_sizes,
    batch_graph,
    batch_config,
    serving_pool,
    config_graph,
)
