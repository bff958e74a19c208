"""Cost model of an update (effects of Delta G, Section 3.3; Theorem 2):
the oracle's ||D r_old||_1 against closed forms for single-edge edits, the
inequality ||q_offset||_1 <= (1-c) ||D r_old||_1 (an equality when one row
changes) with q_offset from the oracle's Algorithm 1, and the iteration
bound against the oracle's iteration counts."""

import numpy as np
import pytest

import oracle
from paper_1712_00595_amd import costmodel
from synth import EdgeSetModel, rmat_graph
from synth.stream import Batch, mixed_batch

C = 0.15


def _graph():
    g = rmat_graph(9, 4000, dead_end_self_loops=True)
    r = oracle.rwr_static(g.n, g.src, g.dst, 0, C)
    return g, r


def _single(g, ins=None, dele=None):
    e = np.zeros(0, np.int32)
    b = Batch(ins_src=np.array([ins[0]] if ins else e, np.int32), ins_dst=np.array([ins[1]] if ins else e, np.int32),
              del_src=np.array([dele[0]] if dele else e, np.int32), del_dst=np.array([dele[1]] if dele else e, np.int32),
              n_new_nodes=0)
    return b, oracle.apply_batch(g.n, g.src, g.dst, b)


def test_closed_forms_for_single_edges():
    g, r = _graph()
    deg = np.bincount(g.src, minlength=g.n)
    # delete one of u's d >= 2 out-edges: D_uu = (d-1)|1/(d-1) - 1/d| + 1/d = 2/d
    u = int(np.flatnonzero(deg >= 3)[0])
    v = int(g.dst[np.flatnonzero(g.src == u)[0]])
    _, new = _single(g, dele=(u, v))
    assert oracle.delta_weight((g.n, g.src, g.dst), new, r) == pytest.approx(2 * r[u] / deg[u], rel=1e-13)
    # insert an absent edge: D_uu = d|1/(d+1) - 1/d| + 1/(d+1) = 2/(d+1)
    have = set(g.dst[g.src == u].tolist())
    w = next(x for x in range(g.n) if x not in have)
    _, new = _single(g, ins=(u, w))
    assert oracle.delta_weight((g.n, g.src, g.dst), new, r) == pytest.approx(2 * r[u] / (deg[u] + 1), rel=1e-13)
    # delete a single out-edge: the row becomes empty, D_uu = 1
    u1 = int(np.flatnonzero(deg == 1)[0])
    v1 = int(g.dst[np.flatnonzero(g.src == u1)[0]])
    _, new = _single(g, dele=(u1, v1))
    assert oracle.delta_weight((g.n, g.src, g.dst), new, r) == pytest.approx(r[u1], rel=1e-13)
    # an unchanged graph
    assert oracle.delta_weight((g.n, g.src, g.dst), (g.n, g.src, g.dst), r) == 0.0


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_seed_norm_inequality_and_iteration_bound(seed):
    g, r = _graph()
    model = EdgeSetModel(g.n, g.src, g.dst)
    b = mixed_batch(np.random.default_rng(seed), model, 30, 30, n_new_nodes=2)
    old = (g.n, g.src, g.dst)
    new = oracle.apply_batch(g.n, g.src, g.dst, b)
    eps = 1e-9
    res = oracle.osp(old, new, r, C, eps)
    q = np.abs(res["q_off"]).sum()
    dw = oracle.delta_weight(old, new, r)
    assert q <= (1 - C) * dw * (1 + 1e-12)
    assert q > 0.2 * (1 - C) * dw  # not vacuous: cancellation between rows is partial
    assert res["iters"] <= costmodel.iterations_bound(q, eps, C)
    assert res["iters"] <= costmodel.iterations_bound_before(dw, eps, C)


def test_single_row_change_is_an_equality():
    g, r = _graph()
    deg = np.bincount(g.src, minlength=g.n)
    u = int(np.argmax(deg))
    nb = g.dst[g.src == u][:3]
    e = np.zeros(0, np.int32)
    b = Batch(ins_src=e, ins_dst=e, del_src=np.full(3, u, np.int32), del_dst=nb.astype(np.int32), n_new_nodes=0)
    old = (g.n, g.src, g.dst)
    new = oracle.apply_batch(g.n, g.src, g.dst, b)
    q = np.abs(oracle.osp(old, new, r, C, 1e-9)["q_off"]).sum()
    assert q == pytest.approx((1 - C) * oracle.delta_weight(old, new, r), rel=1e-12)


def test_iteration_bound_formula():
    # (1-c)^i q <= eps at the bound and not one step before
    for q in (1e-3, 3e-7, 2e-9):
        k = costmodel.iterations_bound(q, 1e-9, C)
        assert (1 - C) ** k * q <= 1e-9 * (1 + 1e-12)
        if k > 1:
            assert (1 - C) ** (k - 1) * q > 1e-9
    assert costmodel.iterations_bound(5e-10, 1e-9, C) == 1
