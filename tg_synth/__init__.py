"""Seeded synthetic typed-graph generators.

This package only produces inputs: CSR arrays and node types. It holds none
of the counting arithmetic, so both the CPU oracle and the GPU path can use
it without sharing any of the method's code.
"""

from .graphs import (  # noqa: F401
    Graph,
    GraphBatch,
    csr_from_edges,
    er_graph,
    chung_lu_typed,
    tripartite_graph,
    random_small_graph,
    config_graph,
    batch_graphs,
    serving_requests,
    CONFIG_NAMES,
)
