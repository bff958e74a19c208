"""Seeded update streams over a directed (or undirected) edge set.

A :class:`Batch` is a *set* of edge insertions and deletions plus a number of
new nodes (ids ``n .. n+k-1``, usable by the batch's edges).  Every stream is
drawn against an :class:`EdgeSetModel`, a plain membership model of the
current edge set, so that each insertion names an absent edge and each
deletion an existing one at the time its batch is applied.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Batch:
    ins_src: np.ndarray
    ins_dst: np.ndarray
    del_src: np.ndarray
    del_dst: np.ndarray
    n_new_nodes: int = 0
    # nodes whose incident edges are all removed (ids of existing nodes)
    del_nodes: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.int32))

    @property
    def n_ins(self) -> int:
        return int(self.ins_src.shape[0])

    @property
    def n_del(self) -> int:
        return int(self.del_src.shape[0])

    @property
    def size(self) -> int:
        """Edge modifications plus node insertions and deletions in the batch."""
        return self.n_ins + self.n_del + int(self.n_new_nodes) + int(self.del_nodes.shape[0])


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


class EdgeSetModel:
    """Current edge set with O(1) uniform sampling of an existing edge.

    Keys are ``u * KEY + v``.  For undirected models a pair is keyed by
    ``(min, max)`` and stands for both stored directions.
    """

    KEY = np.int64(1) << np.int64(32)

    def __init__(self, n: int, src: np.ndarray, dst: np.ndarray, undirected: bool = False):
        self.n = int(n)
        self.undirected = undirected
        s = np.asarray(src, dtype=np.int64)
        d = np.asarray(dst, dtype=np.int64)
        if undirected:
            lo, hi = np.minimum(s, d), np.maximum(s, d)
            keys = np.unique(lo * self.KEY + hi)
        else:
            keys = s * self.KEY + d
        self.keys = np.array(keys, dtype=np.int64)  # sampling pool (unordered)
        self.count = int(self.keys.shape[0])
        self._sorted0 = np.sort(self.keys)  # membership of the initial set
        self._delta: dict[int, bool] = {}  # key -> present, for touched keys
        self._pos: dict[int, int] = {}  # key -> index in self.keys (touched only)

    def _key(self, u: int, v: int) -> int:
        if self.undirected and u > v:
            u, v = v, u
        return int(u) * int(self.KEY) + int(v)

    def has(self, u: int, v: int) -> bool:
        k = self._key(u, v)
        if k in self._delta:
            return self._delta[k]
        i = int(np.searchsorted(self._sorted0, k))
        return i < self._sorted0.shape[0] and int(self._sorted0[i]) == k

    def _index_of(self, k: int) -> int:
        if k in self._pos:
            return self._pos[k]
        # untouched initial key: locate it in the pool once
        idx = int(np.nonzero(self.keys[: self.count] == k)[0][0])
        self._pos[k] = idx
        return idx

    def insert(self, u: int, v: int) -> None:
        k = self._key(u, v)
        if self.count == self.keys.shape[0]:
            self.keys = np.concatenate([self.keys, np.zeros(max(1024, self.count // 8), np.int64)])
        self.keys[self.count] = k
        self._pos[k] = self.count
        self.count += 1
        self._delta[k] = True

    def delete_at(self, idx: int) -> tuple[int, int]:
        k = int(self.keys[idx])
        last = int(self.keys[self.count - 1])
        self.keys[idx] = last
        self._pos[last] = idx
        self.count -= 1
        self._pos.pop(k, None)
        self._delta[k] = False
        return k // int(self.KEY), k % int(self.KEY)

    def delete(self, u: int, v: int) -> None:
        k = self._key(u, v)
        self.delete_at(self._index_of(k))

    def add_nodes(self, k: int) -> None:
        self.n += int(k)


def _draw_absent(rng, model: EdgeSetModel, taken: set, lo_src: int = 0, src_fixed: int | None = None):
    while True:
        u = int(src_fixed) if src_fixed is not None else int(rng.integers(lo_src, model.n))
        v = int(rng.integers(0, model.n))
        if u == v:
            continue
        key = model._key(u, v)
        if key in taken or model.has(u, v):
            continue
        return u, v, key


def mixed_batch(
    rng: np.random.Generator,
    model: EdgeSetModel,
    n_ins: int,
    n_del: int,
    *,
    n_new_nodes: int = 0,
    new_node_edges: tuple[int, int] = (1, 8),
) -> Batch:
    """One batch: ``n_del`` deletions of uniform existing edges, ``n_ins``
    insertions of uniform absent pairs (no self-loops), and ``n_new_nodes`` new
    nodes each with a uniform 1..8 edges to existing nodes (out-edges when
    directed, undirected edges otherwise).  The model is advanced."""
    taken: set = set()
    dels = []
    for _ in range(n_del):
        if model.count == 0:
            break
        idx = int(rng.integers(0, model.count))
        u, v = model.delete_at(idx)
        dels.append((u, v))
        taken.add(model._key(u, v))
    ins = []
    for _ in range(n_ins):
        u, v, key = _draw_absent(rng, model, taken)
        taken.add(key)
        ins.append((u, v))
    n_before = model.n
    model.add_nodes(n_new_nodes)
    for w in range(n_before, n_before + n_new_nodes):
        k = int(rng.integers(new_node_edges[0], new_node_edges[1] + 1))
        chosen: set = set()
        while len(chosen) < k:
            v = int(rng.integers(0, n_before))
            if v not in chosen:
                chosen.add(v)
        for v in sorted(chosen):
            ins.append((w, v))
            taken.add(model._key(w, v))
    for u, v in ins:
        model.insert(u, v)
    ins_a = np.array(ins, dtype=np.int64).reshape(-1, 2)
    del_a = np.array(dels, dtype=np.int64).reshape(-1, 2)
    return Batch(
        ins_src=_i32(ins_a[:, 0]),
        ins_dst=_i32(ins_a[:, 1]),
        del_src=_i32(del_a[:, 0]),
        del_dst=_i32(del_a[:, 1]),
        n_new_nodes=int(n_new_nodes),
    )


def single_edge_stream(model: EdgeSetModel, count: int, *, seed: int = 4, p_insert: float = 0.5) -> list[Batch]:
    """``count`` one-edge batches: each inserts a new uniform pair with
    probability ``p_insert``, otherwise deletes a uniform existing edge."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        if rng.random() < p_insert:
            out.append(mixed_batch(rng, model, 1, 0))
        else:
            out.append(mixed_batch(rng, model, 0, 1))
    return out


def loguniform_batch_stream(
    model: EdgeSetModel,
    count: int,
    *,
    max_size: int = 10000,
    new_node_frac: float = 0.01,
    seed: int = 4,
) -> list[Batch]:
    """``count`` batches whose sizes are ``floor(exp(U(0, ln max_size)))``
    edge modifications, half insertions and half deletions; a fraction
    ``new_node_frac`` of each batch's size (binomially drawn) is new nodes,
    each with 1..8 random out-edges."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        size = int(math.floor(math.exp(rng.uniform(0.0, math.log(max_size)))))
        size = max(1, size)
        k_new = int(rng.binomial(size, new_node_frac))
        n_del = size // 2
        n_ins = size - n_del
        out.append(mixed_batch(rng, model, n_ins, n_del, n_new_nodes=k_new))
    return out


def undirected_churn_batch(rng: np.random.Generator, model: EdgeSetModel, frac: float, n_new_nodes: int) -> Batch:
    """Delete ``frac`` of the current undirected pairs uniformly, insert as many
    new uniform pairs, and add ``n_new_nodes`` nodes with 1..8 random
    undirected edges each.  Pairs are reported once, as (u, v) with u < v for
    the churn and (new node, old node) for new nodes."""
    if not model.undirected:
        raise ValueError("undirected model required")
    k = int(round(frac * model.count))
    return mixed_batch(rng, model, k, k, n_new_nodes=n_new_nodes)
