"""Seeded synthetic hypergraph workloads.

This package produces inputs only.  It holds none of the motif-counting
arithmetic: both the CPU oracle and the HIP library consume what it returns,
and it imports neither of them.

A hypergraph is returned as a CSR incidence ``(edge_ptr, edge_nodes,
num_nodes)``: ``edge_ptr`` is int64[|E|+1], ``edge_nodes`` is int32 with the
node ids of hyperedge ``e`` in ``edge_nodes[edge_ptr[e]:edge_ptr[e+1]]``,
strictly ascending.
"""
from .generators import (  # noqa: F401
    Hypergraph,
    powerlaw_hypergraph,
    stub_matching_copy,
    chung_lu_copy,
    chung_lu_incidences,
    from_edge_lists,
    induced_prefix,
    CONFIGS,
    make_config,
    serving_request,
    serving_copies,
    poisson_arrivals,
)
