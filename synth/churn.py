"""Vectorised churn batches over a large undirected pair set.

:class:`PairPool` keeps the current unordered pairs as one sorted int64 key
array (key = min * 2^32 + max).  A churn batch deletes a uniform sample of
existing pairs and inserts as many uniform absent pairs (no self-loops),
plus new nodes each joined to 1..8 uniform existing nodes; every step is an
array operation (sorted merges, searchsorted), so batches of millions of
pairs on graphs of hundreds of millions of pairs take seconds.  Same
semantics as ``stream.mixed_batch`` on an undirected model: deletions name
present pairs, insertions absent ones, no pair appears twice in a batch.
"""

from __future__ import annotations

import numpy as np

from .stream import Batch

KEY = np.int64(1) << np.int64(32)


def _keys(u: np.ndarray, v: np.ndarray) -> np.ndarray:
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    return np.minimum(u, v) * KEY + np.maximum(u, v)


class PairPool:
    def __init__(self, n: int, pair_u: np.ndarray, pair_v: np.ndarray):
        self.n = int(n)
        self.keys = np.unique(_keys(pair_u, pair_v))

    @property
    def count(self) -> int:
        return int(self.keys.shape[0])

    def has(self, u: int, v: int) -> bool:
        k = int(_keys(np.array([u]), np.array([v]))[0])
        i = int(np.searchsorted(self.keys, k))
        return i < self.count and int(self.keys[i]) == k

    def _absent(self, cand: np.ndarray) -> np.ndarray:
        i = np.searchsorted(self.keys, cand)
        i = np.minimum(i, self.count - 1)
        return self.keys[i] != cand

    def churn_batch(self, rng: np.random.Generator, k: int, n_new_nodes: int = 0,
                    new_node_edges: tuple[int, int] = (1, 8)) -> Batch:
        # deletions: k distinct positions of the sorted pool
        k = min(int(k), self.count)
        pos = np.unique(rng.integers(0, self.count, size=k + k // 8 + 16))
        while pos.shape[0] < k:
            pos = np.unique(np.concatenate([pos, rng.integers(0, self.count, size=k)]))
        pos = rng.permutation(pos)[:k]
        dkeys = self.keys[np.sort(pos)]
        # insertions: uniform pairs u != v, absent before the batch, distinct
        # among themselves (the deleted pairs are present, so never drawn)
        got = np.zeros(0, np.int64)
        while got.shape[0] < k:
            need = k - got.shape[0]
            u = rng.integers(0, self.n, size=need + need // 8 + 16)
            v = rng.integers(0, self.n, size=u.shape[0])
            ok = u != v
            cand = _keys(u[ok], v[ok])
            cand = cand[self._absent(cand)]
            _, first = np.unique(np.concatenate([got, cand]), return_index=True)
            merged = np.concatenate([got, cand])[np.sort(first)]
            got = merged[:k]
        ikeys = got
        # new nodes n .. n+n_new-1, each joined to 1..8 distinct old nodes
        n_old = self.n
        nu, nv = [], []
        for w in range(n_old, n_old + int(n_new_nodes)):
            d = int(rng.integers(new_node_edges[0], new_node_edges[1] + 1))
            nb = np.unique(rng.integers(0, n_old, size=d * 2 + 4))[:d]
            nu.append(np.full(nb.shape[0], w, np.int64))
            nv.append(nb.astype(np.int64))
        self.n += int(n_new_nodes)
        nkeys = _keys(np.concatenate(nu), np.concatenate(nv)) if nu else np.zeros(0, np.int64)
        # advance the pool: drop deleted, merge inserted (sorted runs)
        keep = np.ones(self.count, bool)
        keep[np.searchsorted(self.keys, dkeys)] = False
        add = np.sort(np.concatenate([ikeys, nkeys]))
        self.keys = np.sort(np.concatenate([self.keys[keep], add]), kind="stable")
        ins = np.concatenate([ikeys, nkeys])
        return Batch(
            ins_src=(ins // KEY).astype(np.int32), ins_dst=(ins % KEY).astype(np.int32),
            del_src=(dkeys // KEY).astype(np.int32), del_dst=(dkeys % KEY).astype(np.int32),
            n_new_nodes=int(n_new_nodes),
        )


def churn_stream(pool: PairPool, count: int, frac: float = 0.01, n_new_nodes: int = 1000, seed: int = 4):
    """``count`` batches, each deleting ``frac`` of the current pairs and
    inserting as many, plus ``n_new_nodes`` new nodes; generated lazily."""
    rng = np.random.Generator(np.random.PCG64(seed))
    for _ in range(count):
        yield pool.churn_batch(rng, int(round(frac * pool.count)), n_new_nodes)
