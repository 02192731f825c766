"""Seeded synthetic inputs shaped like the paper's workloads.

This package holds none of the method's arithmetic: it draws points and
queries, builds exact k-nearest-neighbour lists by brute force (the step
before the base graph's RobustPrune), picks the medoid start vertex, and draws
per-node degree targets and node samples.  Both the HIP path and the CPU
oracle consume what it produces; neither is imported here.
"""
from .synth import (  # noqa: F401
    Workload,
    CONFIGS,
    make_points,
    make_queries,
    knn_lists,
    medoid,
    degree_targets,
    node_sample,
    build,
)
