"""Oracle for general restart vectors (global PageRank when q = 1/n), pinned
by the seed-node special case (a different C routine), a closed form (a
directed cycle), a dense LU solve, superposition without dead ends, and
Theorem 4's normalisation when the support of q reaches a dead end."""

import numpy as np
import pytest

import oracle
from synth import rmat_graph

C = 0.15


def test_unit_vector_is_the_seed_node_solve():
    g = rmat_graph(9, 3000, dead_end_self_loops=False)
    s = int(np.argmax(np.bincount(g.src, minlength=g.n)))
    q = np.zeros(g.n)
    q[s] = 1.0
    assert np.abs(oracle.rwr_static_vector(g.n, g.src, g.dst, q, C) - oracle.rwr_static(g.n, g.src, g.dst, s, C)
                  ).sum() < 1e-12


def test_cycle_with_uniform_restart_is_uniform():
    n = 17
    src = np.arange(n, dtype=np.int32)
    dst = ((np.arange(n) + 1) % n).astype(np.int32)
    r = oracle.rwr_static_vector(n, src, dst, np.full(n, 1.0 / n), C)
    assert np.allclose(r, 1.0 / n, atol=1e-14)


@pytest.mark.parametrize("kind", ["uniform", "random"])
def test_dense_lu_agrees(kind):
    g = rmat_graph(7, 500, dead_end_self_loops=False)  # with dead ends
    rng = np.random.default_rng(4)
    q = np.full(g.n, 1.0 / g.n) if kind == "uniform" else rng.random(g.n) * (rng.random(g.n) < 0.2)
    q = q / q.sum()
    A = oracle.row_normalised_dense(g.n, g.src, g.dst)
    r = np.linalg.solve(np.eye(g.n) - (1 - C) * A.T, C * q)
    deg = np.bincount(g.src, minlength=g.n)
    if np.any(oracle.reachable_from(g.n, g.src, g.dst, np.flatnonzero(q)) & (deg == 0)):
        r = r / r.sum()
    got = oracle.rwr_static_vector(g.n, g.src, g.dst, q, C)
    assert np.abs(got - r).sum() < 1e-12
    # dead ends are reachable here, so the mass was renormalised
    assert abs(got.sum() - 1.0) < 1e-12


def test_superposition_without_dead_ends():
    g = rmat_graph(8, 2000, dead_end_self_loops=True)
    a, b = 3, 40
    qa = np.zeros(g.n)
    qa[a] = 1.0
    qb = np.zeros(g.n)
    qb[b] = 1.0
    r = oracle.rwr_static_vector(g.n, g.src, g.dst, 0.25 * qa + 0.75 * qb, C)
    ra = oracle.rwr_static(g.n, g.src, g.dst, a, C)
    rb = oracle.rwr_static(g.n, g.src, g.dst, b, C)
    assert np.abs(r - (0.25 * ra + 0.75 * rb)).sum() < 1e-12


def test_reachability():
    src = np.array([0, 1, 3], np.int32)
    dst = np.array([1, 2, 4], np.int32)
    assert oracle.reachable_from(5, src, dst, [0]).tolist() == [True, True, True, False, False]
    assert oracle.reachable_from(5, src, dst, [3, 2]).tolist() == [False, False, True, True, True]
