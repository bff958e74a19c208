"""Recursive-matrix (R-MAT) graph generator, seeded and vectorised.

R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004) places every edge by descending
``scale`` levels of a 2x2 quadrant split with probabilities (a, b, c, d) for
(top-left, top-right, bottom-left, bottom-right); the row bit of a level is the
source bit, the column bit the destination bit.  No noise is added.

Conventions used for every workload:
  * self-loops and repeated pairs are dropped, more pairs are drawn until at
    least ``m`` distinct ones exist, and a uniformly random subset of exactly
    ``m`` of them is kept;
  * vertex ids are then relabelled by a seeded random permutation, so that id
    order carries no locality (the usual Graph500 practice);
  * optionally every node left without out-edges gets one self-loop;
  * optionally the graph is symmetrised: each unordered pair {u, v} is kept
    once and both directions are stored.
"""

from __future__ import annotations

import dataclasses

import numpy as np

RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)


@dataclasses.dataclass
class RmatGraph:
    n: int
    src: np.ndarray  # int32, stored directed edges
    dst: np.ndarray  # int32
    undirected: bool = False
    # for undirected graphs: the distinct unordered pairs (u <= v) the stored
    # directed edges came from
    pair_u: np.ndarray | None = None
    pair_v: np.ndarray | None = None

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    def out_degree(self) -> np.ndarray:
        return np.bincount(self.src, minlength=self.n).astype(np.int64)


def _draw_pairs(rng: np.random.Generator, scale: int, k: int, abcd) -> tuple[np.ndarray, np.ndarray]:
    """``k`` R-MAT pairs; one uniform float32 per level picks the quadrant."""
    a, b, c, _ = abcd
    src = np.zeros(k, dtype=np.uint32)
    dst = np.zeros(k, dtype=np.uint32)
    t_a, t_ab, t_abc = np.float32(a), np.float32(a + b), np.float32(a + b + c)
    r = np.empty(k, dtype=np.float32)
    sbit = np.empty(k, dtype=bool)
    dbit = np.empty(k, dtype=bool)
    tmp = np.empty(k, dtype=bool)
    for _ in range(scale):
        rng.random(out=r, dtype=np.float32)
        np.left_shift(src, 1, out=src)
        np.left_shift(dst, 1, out=dst)
        np.greater_equal(r, t_ab, out=sbit)  # quadrants c, d: row bit set
        np.greater_equal(r, t_abc, out=dbit)  # quadrant d
        np.greater_equal(r, t_a, out=tmp)
        np.greater(tmp, sbit, out=tmp)  # quadrant b: a <= r < a+b
        np.logical_or(dbit, tmp, out=dbit)
        np.bitwise_or(src, sbit, out=src, casting="unsafe")
        np.bitwise_or(dst, dbit, out=dst, casting="unsafe")
    return src.astype(np.int64), dst.astype(np.int64)


def rmat_graph(
    scale: int,
    m: int,
    *,
    seed_graph: int = 1,
    seed_perm: int = 2,
    abcd=RMAT_ABCD,
    dead_end_self_loops: bool = False,
    undirected: bool = False,
) -> RmatGraph:
    """Draw an R-MAT graph with 2**scale nodes and ``m`` distinct edges.

    For ``undirected=True``, ``m`` counts distinct unordered pairs; the stored
    directed edge list holds both directions of every pair.
    """
    n = 1 << scale
    if m > n * (n - 1) // (2 if undirected else 1):
        raise ValueError("too many edges for the node count")
    rng = np.random.Generator(np.random.PCG64(seed_graph))
    kept = np.empty(0, dtype=np.int64)
    while kept.shape[0] < m:
        need = m - kept.shape[0]
        k = int(need * 1.15) + 4096
        s, d = _draw_pairs(rng, scale, k, abcd)
        ok = s != d
        s, d = s[ok], d[ok]
        if undirected:
            keys = np.minimum(s, d) * n + np.maximum(s, d)
        else:
            keys = s * n + d
        kept = np.unique(np.concatenate([kept, keys]))
    # keep a uniformly random subset of exactly m distinct pairs
    pick = np.sort(rng.permutation(kept.shape[0])[:m])
    kept = kept[pick]
    s = (kept // n).astype(np.int64)
    d = (kept % n).astype(np.int64)
    prng = np.random.Generator(np.random.PCG64(seed_perm))
    perm = prng.permutation(n).astype(np.int64)
    s = perm[s]
    d = perm[d]
    if undirected:
        pu = np.minimum(s, d).astype(np.int32)
        pv = np.maximum(s, d).astype(np.int32)
        src = np.concatenate([pu, pv])
        dst = np.concatenate([pv, pu])
        g = RmatGraph(n=n, src=src, dst=dst, undirected=True, pair_u=pu, pair_v=pv)
    else:
        g = RmatGraph(n=n, src=s.astype(np.int32), dst=d.astype(np.int32))
    if dead_end_self_loops:
        if undirected:
            raise ValueError("self-loops on dead ends apply to directed graphs only")
        deg = g.out_degree()
        dead = np.nonzero(deg == 0)[0].astype(np.int32)
        g.src = np.concatenate([g.src, dead])
        g.dst = np.concatenate([g.dst, dead])
    return g


def pick_max_outdeg_seed(g: RmatGraph) -> int:
    """Node with the largest out-degree; ties go to the lowest id."""
    deg = g.out_degree()
    return int(np.argmax(deg))  # argmax returns the first maximum


def sample_seeds(g: RmatGraph, k: int, *, seed: int = 3) -> np.ndarray:
    """``k`` distinct seed nodes, uniform among nodes with at least one
    out-edge to another node (dead-end self-loops do not make a node
    eligible)."""
    keep = g.src != g.dst
    deg = np.bincount(g.src[keep], minlength=g.n)
    elig = np.nonzero(deg >= 1)[0]
    if k > elig.shape[0]:
        raise ValueError("not enough eligible seed nodes")
    rng = np.random.Generator(np.random.PCG64(seed))
    pick = rng.choice(elig.shape[0], size=k, replace=False)
    return np.sort(elig[pick]).astype(np.int32)
