"""The five synthetic workloads, named by what they are.

Each entry fixes the graph recipe, the seed nodes, the restart probability,
the tolerances and the update stream.  RNG seeds: graph 1, permutation 2,
seed nodes 3, update stream 4, model init 5, train/eval split 6.

The paper measures on SNAP graphs that are not available here; these R-MAT
graphs stand in for them at matching sizes (scale 20 ~ Berkstan, scale 21-22 ~
LiveJournal, scale 23 ~ WikiLink/Orkut).
"""

from __future__ import annotations

import dataclasses
from typing import Callable

import numpy as np

from .rmat import RmatGraph, pick_max_outdeg_seed, rmat_graph, sample_seeds
from .stream import Batch, EdgeSetModel, loguniform_batch_stream, mixed_batch, single_edge_stream, undirected_churn_batch


@dataclasses.dataclass
class Workload:
    name: str
    scale: int
    m: int
    undirected: bool
    dead_end_self_loops: bool
    c: float
    eps: tuple
    n_seeds: int
    gate: str
    description: str

    def graph(self) -> RmatGraph:
        return rmat_graph(
            self.scale,
            self.m,
            dead_end_self_loops=self.dead_end_self_loops,
            undirected=self.undirected,
        )

    def seeds(self, g: RmatGraph) -> np.ndarray:
        if self.n_seeds == 1:
            return np.array([pick_max_outdeg_seed(g)], dtype=np.int32)
        return sample_seeds(g, self.n_seeds, seed=3)

    def model(self, g: RmatGraph) -> EdgeSetModel:
        if self.undirected:
            return EdgeSetModel(g.n, g.pair_u, g.pair_v, undirected=True)
        return EdgeSetModel(g.n, g.src, g.dst)


WORKLOADS: dict[str, Workload] = {}


def _reg(w: Workload) -> Workload:
    WORKLOADS[w.name] = w
    return w


RMAT13_ONE_BATCH = _reg(
    Workload(
        name="rmat13_one_batch_exact",
        scale=13,
        m=131072,
        undirected=False,
        dead_end_self_loops=True,
        c=0.15,
        eps=(1e-14,),
        n_seeds=1,
        gate="L1 < 1e-12 against the static solve (FP64 propagation)",
        description="directed R-MAT 2^13 nodes, 131072 edges + dead-end self-loops, seed = max out-degree node, "
        "one batch of 64 insertions of absent pairs + 64 deletions of existing edges",
    )
)

RMAT20_SINGLE_EDGE = _reg(
    Workload(
        name="rmat20_single_edge_stream",
        scale=20,
        m=16777216,
        undirected=False,
        dead_end_self_loops=True,
        c=0.15,
        eps=(1e-9, 1e-6),
        n_seeds=1,
        gate="L1 <= 1e-9 (exact mode) / 2*eps/c (OSP-T)",
        description="directed R-MAT 2^20 nodes, 16777216 edges + dead-end self-loops, seed = max out-degree node, "
        "1000 single-edge updates (50% insert of a new uniform pair, 50% delete of a uniform existing edge)",
    )
)

RMAT22_BATCHED = _reg(
    Workload(
        name="rmat22_batched_seeds",
        scale=22,
        m=67108864,
        undirected=False,
        dead_end_self_loops=True,
        c=0.15,
        eps=(1e-6,),
        n_seeds=64,
        gate="L1 <= 2*eps/c",
        description="directed R-MAT 2^22 nodes, 67108864 edges + dead-end self-loops, 64 uniform seeds, "
        "200 batches of log-uniform size in [1, 10000] with 1% new nodes (1-8 out-edges each)",
    )
)

RMAT21_LEARNED = _reg(
    Workload(
        name="rmat21_learned_warm_start",
        scale=21,
        m=33554432,
        undirected=False,
        dead_end_self_loops=True,
        c=0.15,
        eps=(1e-6,),
        n_seeds=16,
        gate="L1 <= 2*eps/c",
        description="directed R-MAT 2^21 nodes, 33554432 edges, 16 uniform seeds, 100-edge random batches "
        "(5000 train / 500 held out)",
    )
)

RMAT23_UNDIRECTED = _reg(
    Workload(
        name="rmat23_undirected_churn",
        scale=23,
        m=134217728,
        undirected=True,
        dead_end_self_loops=False,
        c=0.05,
        eps=(1e-9,),
        n_seeds=16,
        gate="L1 <= 2*eps/c",
        description="symmetrised R-MAT 2^23 nodes, 134217728 pairs (268435456 stored directed edges), c = 0.05, "
        "16 seeds, 100 batches each deleting 1% of pairs and inserting as many plus 1000 new nodes",
    )
)


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def one_batch_rmat13(model: EdgeSetModel, seed: int = 4) -> Batch:
    rng = np.random.Generator(np.random.PCG64(seed))
    return mixed_batch(rng, model, 64, 64)


def stream_for(w: Workload, model: EdgeSetModel, count: int) -> list[Batch]:
    if w.name == RMAT13_ONE_BATCH.name:
        return [one_batch_rmat13(model)]
    if w.name == RMAT20_SINGLE_EDGE.name:
        return single_edge_stream(model, count, seed=4)
    if w.name == RMAT22_BATCHED.name:
        return loguniform_batch_stream(model, count, seed=4)
    if w.name == RMAT21_LEARNED.name:
        rng = np.random.Generator(np.random.PCG64(4))
        return [mixed_batch(rng, model, 50, 50) for _ in range(count)]
    if w.name == RMAT23_UNDIRECTED.name:
        rng = np.random.Generator(np.random.PCG64(4))
        return [undirected_churn_batch(rng, model, 0.01, 1000) for _ in range(count)]
    raise KeyError(w.name)


StreamFn = Callable[[EdgeSetModel, int], list]
