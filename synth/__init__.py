"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This package only draws random graphs, seed nodes and update streams.  It
holds none of the random-walk-with-restart arithmetic: no normalisation, no
propagation, no scores.  Both the product path and the oracle consume what it
produces, and neither side's code lives here.
"""

from .rmat import rmat_graph, RmatGraph, pick_max_outdeg_seed, sample_seeds
from .stream import (
    Batch,
    EdgeSetModel,
    single_edge_stream,
    mixed_batch,
    loguniform_batch_stream,
    undirected_churn_batch,
)
from .configs import WORKLOADS, workload

__all__ = [
    "rmat_graph",
    "RmatGraph",
    "pick_max_outdeg_seed",
    "sample_seeds",
    "Batch",
    "EdgeSetModel",
    "single_edge_stream",
    "mixed_batch",
    "loguniform_batch_stream",
    "undirected_churn_batch",
    "WORKLOADS",
    "workload",
]
