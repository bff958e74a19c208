"""General restart vectors on the GPU (global PageRank for q = 1/n): the
static scores and every update of a stream against the oracle, for uniform
and random restart vectors, FP64 (exact) and FP32 (OSP-T gate), directed and
undirected, with new nodes (q = 0) and a node deletion; argument checks."""

import numpy as np
import pytest

import oracle
from synth import EdgeSetModel, rmat_graph
from synth.stream import Batch, mixed_batch

pytestmark = pytest.mark.gpu

rwr = pytest.importorskip("paper_1712_00595_amd.rwr")

C = 0.15


def _q(n, kind, S, rng):
    if kind == "uniform":
        return np.full((n, S), 1.0 / n)
    q = rng.random((n, S)) * (rng.random((n, S)) < 0.1)
    return q / q.sum(axis=0, keepdims=True)


@pytest.mark.parametrize("kind,S,precision,undirected", [
    ("uniform", 1, "fp64", False), ("random", 3, "fp64", False), ("uniform", 1, "fp32", False),
    ("random", 2, "fp32", True)])
def test_stream_matches_oracle(kind, S, precision, undirected):
    print(f"[vectors] {kind} S={S} {precision} undirected={undirected}", flush=True)
    g = rmat_graph(11, 20000, dead_end_self_loops=not undirected, undirected=undirected)
    rng = np.random.default_rng(11)
    q = _q(g.n, kind, S, rng)
    eps = 1e-14 if precision == "fp64" else 1e-9
    kw = dict(c=C, eps=eps, precision=precision, undirected=undirected)
    if precision == "fp64":
        kw.update(build_tol=1e-13, err_budget=1e-12)
    gate = 1e-11 if precision == "fp64" else 2 * eps / C
    es, ed = (g.pair_u, g.pair_v) if undirected else (g.src, g.dst)
    model = EdgeSetModel(g.n, es, ed, undirected=undirected)
    with rwr.Context(g.n, es, ed, q=q, **kw) as ctx:
        n, s, d = g.n, g.src, g.dst
        for j in range(S):
            assert np.abs(ctx.scores(j) - oracle.rwr_static_vector(n, s, d, q[:, j], C)).sum() < gate
        batches = [mixed_batch(rng, model, 30, 30, n_new_nodes=2), mixed_batch(rng, model, 1, 0),
                   mixed_batch(rng, model, 200, 200, n_new_nodes=5)]
        for b in batches:
            ctx.update_batch(b)
            n, s, d = oracle.apply_batch(n, s, d, b, undirected=undirected)
            qp = np.zeros((n, S))
            qp[: q.shape[0]] = q  # new nodes restart with probability 0
            for j in range(S):
                err = np.abs(ctx.scores(j) - oracle.rwr_static_vector(n, s, d, qp[:, j], C)).sum()
                assert err < gate, (j, err)


def test_node_deletion_keeps_the_restart_entry():
    print("[vectors] node deletion", flush=True)
    g = rmat_graph(10, 8000, dead_end_self_loops=True)
    q = np.full(g.n, 1.0 / g.n)
    dn = np.array([int(np.argsort(-g.out_degree())[3])], np.int32)
    E = np.zeros(0, np.int32)
    b = Batch(E, E, E, E, 0, dn)
    with rwr.Context(g.n, g.src, g.dst, q=q, eps=1e-14, precision="fp64", build_tol=1e-13,
                     err_budget=1e-12) as ctx:
        ctx.update_batch(b)
        n, s, d = oracle.apply_batch(g.n, g.src, g.dst, b)
        err = np.abs(ctx.scores(0) - oracle.rwr_static_vector(n, s, d, q, C)).sum()
        assert err < 1e-11, err


def test_arguments_are_checked():
    g = rmat_graph(8, 1000, dead_end_self_loops=True)
    bad = np.full(g.n, 1.0 / g.n)
    bad[0] = -bad[0]
    with pytest.raises(rwr.RwrError):
        rwr.Context(g.n, g.src, g.dst, q=bad)
    with pytest.raises(rwr.RwrError):
        rwr.Context(g.n, g.src, g.dst, q=np.full(g.n, 2.0 / g.n))
    with rwr.Context(g.n, g.src, g.dst, q=np.full(g.n, 1.0 / g.n)) as ctx:
        with pytest.raises(rwr.RwrError) as e:
            ctx.warm_start("predict")
        assert e.value.code == -8
