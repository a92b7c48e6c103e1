"""Seeded synthetic graph and request generators.

This package produces inputs only: edge lists, weights and request traces.
It holds none of the embedding arithmetic, so both the FP64 oracle and the
GPU library can be fed from it without sharing any of the method's code.
"""

from .graphs import (  # noqa: F401
    Graph,
    erdos_renyi,
    chung_lu,
    bipartite_zipf,
    random_graph,
    workload,
    WORKLOADS,
)
from .trace import Request, materialize, served_trace  # noqa: F401
