"""Seeded synthetic inputs for the edge-bundling hot path.

This package only draws inputs: node positions, edge lists, edge groups,
interaction matrices and the per-iteration radius lists of each workload.
It holds none of the bundling arithmetic, so both the GPU path and the
CPU oracle can take their inputs from it without sharing method code.
"""

from .graphs import (  # noqa: F401
    Workload,
    uniform_graph,
    clustered_graph,
    zipf_cluster_graph,
    matrix_pattern_graph,
    kmeans_groups,
    interaction_eq4,
    interaction_constant,
    radius_schedule,
    tiny,
    mid,
    stack3d,
    differentiation,
    batched,
    scaled,
    WORKLOADS,
)
