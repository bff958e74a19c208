"""GPU parity of the warm start's training step inside rwr_update: the region,
the network output, dL/do of the residual loss (through the mass
correction) and every parameter-gradient block, read back through
rwr_warm_inspect, against the CPU oracle (oracle/gnn.py) computed from the
graph, the batch and the oracle's own static scores.  The oracle's exact
gradient is pinned by central differences in
tests/test_oracle_residual_loss.py."""

import numpy as np
import pytest

import oracle
from oracle import gnn
from synth import EdgeSetModel, rmat_graph
from synth.rmat import sample_seeds
from synth.stream import mixed_batch

pytestmark = pytest.mark.gpu

rwr = pytest.importorskip("paper_1712_00595_amd.rwr")

C = 0.15


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _params(seed):
    """The propagation prior plus seeded noise on every weight, so that every
    parameter block carries gradient."""
    from paper_1712_00595_amd.warm import init_params

    th = init_params(seed, prior="propagation", c=C).astype(np.float64)
    th += 0.01 * np.random.default_rng(seed).normal(size=th.shape)
    return th.astype(np.float32)


@pytest.mark.parametrize("undirected,n_seeds,hops,push", [(False, 3, 2, None), (True, 2, 2, None),
                                                          (False, 5, 3, None), (False, 3, 2, "1"),
                                                          (True, 2, 2, "1")])
def test_in_update_training_step_matches_oracle(undirected, n_seeds, hops, push, monkeypatch):
    """push "1": the residual formed from the region alone (RWR_WS_PUSH=1)."""
    print(f"[warm grad] undirected={undirected} seeds={n_seeds} hops={hops} push={push}", flush=True)
    if push is not None:
        monkeypatch.setenv("RWR_WS_PUSH", push)
    g = rmat_graph(10, 6000, dead_end_self_loops=not undirected, undirected=undirected)
    seeds = sample_seeds(g, n_seeds, seed=3)
    es, ed = (g.pair_u, g.pair_v) if undirected else (g.src, g.dst)
    model = EdgeSetModel(g.n, es, ed, undirected=undirected)
    b = mixed_batch(np.random.default_rng(6), model, 12, 12)
    theta = _params(11)
    kw = dict(c=C, eps=1e-14, precision="fp64", build_tol=1e-13, err_budget=1e-12, undirected=undirected)
    with rwr.Context(g.n, es, ed, seeds, **kw) as ctx:
        ctx.model_set(theta)
        ctx.warm_start("train", hops=hops, lr=0.0, weight_decay=0.0)
        st = ctx.update_batch(b)
        got = ctx.warm_inspect()
    S = got["o"].shape[1]
    assert S >= n_seeds and got["nodes"].shape[0] == st["ws_region"] > 0

    # the oracle from its own static scores of the graph before the batch
    n0, s0, d0 = g.n, g.src, g.dst
    n1, s1, d1 = oracle.apply_batch(n0, s0, d0, b, undirected=undirected)
    r_old = np.zeros((n1, S))
    for j, sd in enumerate(seeds):
        r_old[:n0, j] = oracle.rwr_static(n0, s0, d0, int(sd), C)
    P_old = gnn.propagation_operator(n1, s0, d0, C)
    P = gnn.propagation_operator(n1, s1, d1, C)
    q = P @ r_old - P_old @ r_old  # (1-c)(B~^T - A~^T) r_old, Section 3.1
    level0 = gnn.offset_support((n0, s0, d0), (n1, s1, d1), r_old[:n0])
    nodes_ref, hops_ref = gnn.region(n1, s1, d1, level0, hops, cap=10 ** 9)
    # the same region, level by level
    assert sorted(zip(got["nodes"].tolist(), got["hops"].tolist())) == sorted(
        zip(nodes_ref.tolist(), hops_ref.tolist()))

    # rows in the device's order (the network is equivariant to it)
    nodes = got["nodes"].astype(np.int64)
    hop = got["hops"].astype(np.int64)
    sig = r_old.sum(axis=0)
    seeds_p = list(seeds) + [-1] * (S - n_seeds)
    F = gnn.features(n1, s1, d1, nodes, hop, q, r_old, sig, seeds_p)
    ls, ld = gnn.local_edges(s1, d1, nodes)
    deg = np.bincount(s1, minlength=n1)
    dinv = np.where(deg > 0, 1.0 / np.maximum(deg, 1), 0.0)[nodes].astype(np.float32).astype(np.float64)
    ref = gnn.residual_loss(theta.astype(np.float64), F, ls, ld, dinv, nodes, q, P, deg[nodes] > 0, C, rnd=True)
    act = ref["active"]
    assert act[:n_seeds].all() and not act[n_seeds:].any()

    # network output on the active columns, loss, dL/do, gradient by block
    assert _rel(got["o"][:, act], ref["o"][:, act]) < 2e-3, _rel(got["o"][:, act], ref["o"][:, act])
    assert abs(st["ws_loss"] - ref["loss"]) <= 1e-3 * ref["loss"], (st["ws_loss"], ref["loss"])
    assert _rel(got["dout"], ref["do"]) < 1e-2, _rel(got["dout"], ref["do"])
    gd = got["grad"].astype(np.float64)
    gr = ref["grad"]
    off = 0
    for k in gnn.ORDER:
        nb = int(np.prod(gnn.SHAPES[k]))
        a, bb = gd[off:off + nb], gr[off:off + nb]
        assert _rel(a, bb) < 1e-2 or np.linalg.norm(a - bb) < 1e-4 * np.linalg.norm(gr), (k, _rel(a, bb))
        off += nb
    assert _rel(gd, gr) < 5e-3, _rel(gd, gr)
    # the device follows the correction: the fixed-correction gradient is
    # farther from what it computed than the exact one
    fixed = gnn.residual_loss(theta.astype(np.float64), F, ls, ld, dinv, nodes, q, P, deg[nodes] > 0, C, rnd=True,
                              follow=False)
    if np.any(np.abs(ref["beta"][act]) > 1e-3):
        assert _rel(gd, fixed["grad"]) > 2 * _rel(gd, gr)
