"""The vectorised churn generator names present pairs for deletion and absent
pairs for insertion, and its pool tracks the graph (checked by applying its
batches with the oracle's validating batch apply)."""

import numpy as np

import oracle
from synth import rmat_graph
from synth.churn import PairPool, churn_stream


def test_churn_batches_are_valid_and_tracked():
    g = rmat_graph(10, 4000, undirected=True)
    pool = PairPool(g.n, g.pair_u, g.pair_v)
    n, s, d = g.n, g.src, g.dst
    for b in churn_stream(pool, 4, frac=0.05, n_new_nodes=7, seed=11):
        assert b.n_ins == b.n_del + int(np.sum(b.ins_dst >= n))  # pairs are (min, max)
        n, s, d = oracle.apply_batch(n, s, d, b, undirected=True)  # raises on an invalid batch
        lo, hi = np.minimum(s, d).astype(np.int64), np.maximum(s, d).astype(np.int64)
        assert n == pool.n
        assert np.array_equal(np.unique(lo * (1 << 32) + hi), pool.keys)
