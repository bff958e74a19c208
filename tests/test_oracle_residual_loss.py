"""Pins of the warm start's in-update training loss in the oracle
(oracle/gnn.py: offset_support, features, mass_correction, residual_loss):
central differences of the exact gradient through the mass correction, the
measured gap of the gradient that holds the correction fixed, the zero-sum
residual, the reductions for a silent network and for the propagation
prior, and closed forms for the region's level 0 and the features."""

import numpy as np
import pytest

import oracle
from oracle import gnn

C = 0.15


def _graph(seed, n=70, m=260, dead=2):
    rng = np.random.default_rng(seed)
    keys = set()
    while len(keys) < m:
        u, v = (int(x) for x in rng.integers(0, n, 2))
        if u != v and u >= dead:  # nodes 0 .. dead-1 stay dead ends
            keys.add((u, v))
    src = np.array([k[0] for k in keys], np.int64)
    dst = np.array([k[1] for k in keys], np.int64)
    return n, src, dst


def _case(seed, S=2, nR=45):
    """A region of nR nodes in a small graph with two dead ends, a zero-sum
    offset seed on a few region nodes, features as the update computes them,
    and parameters: the propagation prior (so that the prediction follows
    the signs of q) plus seeded noise on every weight and bias (so that
    every block carries gradient)."""
    from paper_1712_00595_amd.warm import init_params

    rng = np.random.default_rng(seed)
    n, src, dst = _graph(seed)
    nodes = np.sort(rng.choice(n, nR, replace=False))
    q = np.zeros((n, S))
    for j in range(S):
        sup = rng.choice(nodes, 6, replace=False)
        vals = rng.normal(size=6)
        q[sup, j] = vals - vals.mean()
    ls, ld = gnn.local_edges(src, dst, nodes)
    deg = np.bincount(src, minlength=n)
    dinv = np.where(deg > 0, 1.0 / np.maximum(deg, 1), 0.0)[nodes]
    live = deg[nodes] > 0
    hop = rng.integers(0, 4, nR)
    r_old = np.abs(rng.normal(size=(n, S))) / n
    F = gnn.features(n, src, dst, nodes, hop, q, r_old, r_old.sum(axis=0), [-1] * S)
    theta = init_params(seed + 1, prior="propagation", c=C).astype(np.float64)
    theta = theta + 0.01 * rng.normal(size=theta.shape)
    P = gnn.propagation_operator(n, src, dst, C)
    return dict(theta=theta, F=F, lsrc=ls, ldst=ld, dinv=dinv, nodes=nodes, q=q, P=P, live=live, c=C)


def _L(case, theta):
    a = dict(case)
    a["theta"] = theta
    return gnn.residual_loss(**a)["loss"]


def _pattern(case, theta):
    """Signs of the residual and of the prediction, and the ReLU masks: a
    central difference is only meaningful when the two points share them
    (no kink in between)."""
    a = dict(case)
    a["theta"] = theta
    res = gnn.residual_loss(**a)
    _, cache = gnn.forward(theta, case["F"], case["lsrc"], case["ldst"], case["dinv"])
    return [np.sign(res["rho"]), np.sign(res["xhat"])] + [h > 0 for h in cache["h"]]


def _same(p1, p2):
    return all(np.array_equal(a, b) for a, b in zip(p1, p2))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_exact_gradient_matches_central_differences(seed):
    case = _case(seed)
    res = gnn.residual_loss(**case)
    g = res["grad"]
    assert np.linalg.norm(g) > 0
    theta = case["theta"]
    rng = np.random.default_rng(50 + seed)
    h = 1e-7
    off = 0
    checked = skipped = 0
    for k in gnn.ORDER:
        n = int(np.prod(gnn.SHAPES[k]))
        for i in rng.choice(n, size=min(n, 3), replace=False):
            e = np.zeros_like(theta)
            e[off + i] = h
            if not _same(_pattern(case, theta + e), _pattern(case, theta - e)):
                skipped += 1
                continue
            fd = (_L(case, theta + e) - _L(case, theta - e)) / (2 * h)
            assert abs(fd - g[off + i]) <= 1e-5 * abs(fd) + 1e-7, (k, i, fd, g[off + i])
            checked += 1
        off += n
    assert checked >= 40 and skipped <= 5, (checked, skipped)
    for _ in range(3):
        d = rng.normal(size=theta.shape)
        d /= np.linalg.norm(d)
        if not _same(_pattern(case, theta + h * d), _pattern(case, theta - h * d)):
            continue
        fd = (_L(case, theta + h * d) - _L(case, theta - h * d)) / (2 * h)
        assert abs(fd - g @ d) <= 1e-5 * abs(fd) + 1e-7


def test_holding_the_correction_fixed_is_a_measured_approximation():
    # the gradient that ignores the correction's derivative (the correction
    # taken as a constant) has the same loss but differs from the exact
    # gradient by 30 % or more of its norm in every case here; without the
    # first layer's homogeneity (weights on the degree inputs) it is not
    # even a descent direction in some of them
    gaps, cosines = [], []
    for seed in range(6):
        case = _case(seed)
        exact = gnn.residual_loss(**case)
        fixed = gnn.residual_loss(**case, follow=False)
        assert exact["loss"] == fixed["loss"]
        ge, gf = exact["grad"], fixed["grad"]
        gaps.append(np.linalg.norm(ge - gf) / np.linalg.norm(ge))
        cosines.append(ge @ gf / (np.linalg.norm(ge) * np.linalg.norm(gf)))
    assert min(gaps) > 0.3, gaps
    neg = []
    for seed in range(6):
        case = _case(seed)
        p = gnn.unpack(case["theta"])
        p["W0"] = p["W0"] + 0.3 * np.random.default_rng(seed).uniform(-1, 1, p["W0"].shape)
        case["theta"] = gnn.pack(p)
        ge = gnn.residual_loss(**case)["grad"]
        gf = gnn.residual_loss(**case, follow=False)["grad"]
        neg.append(ge @ gf / (np.linalg.norm(ge) * np.linalg.norm(gf)))
    assert min(neg) < 0.0, neg


def test_corrected_residual_sums_to_zero_with_dead_ends():
    case = _case(3)
    res = gnn.residual_loss(**case)
    assert not np.all(case["live"])  # the region holds a dead end
    rho = res["rho"]
    scale = np.abs(rho).sum(axis=0)
    assert np.all(np.abs(rho.sum(axis=0)) <= 1e-12 * scale)
    # without the correction the sum is generally not zero
    xh = np.zeros_like(case["q"])
    o, _ = gnn.forward(case["theta"], case["F"], case["lsrc"], case["ldst"], case["dinv"])
    xh[case["nodes"]] = np.abs(case["q"]).sum(axis=0) * o
    raw = case["q"] - xh + case["P"] @ xh
    assert np.any(np.abs(raw.sum(axis=0)) > 1e-6 * np.abs(raw).sum(axis=0))


def test_silent_network_leaves_the_seed():
    case = _case(4)
    p = gnn.unpack(case["theta"])
    p["wo"][:] = 0.0
    p["bo"][:] = 0.0
    case["theta"] = gnn.pack(p)
    res = gnn.residual_loss(**case)
    assert np.array_equal(res["rho"], case["q"])
    assert res["loss"] == pytest.approx(1.0, abs=1e-15)
    assert np.all(res["beta"] == 0.0)


def test_propagation_prior_predicts_the_partial_sum():
    # the product package's prior makes the network compute the first four
    # terms of the offset series; its residual is then the fifth term
    # ((1-c) B~^T)^4 q (no bfloat16 rounding here), and the mass correction
    # leaves it alone because that term already sums to zero in a graph
    # without dead ends
    from paper_1712_00595_amd.warm import init_params

    rng = np.random.default_rng(9)
    n, src, dst = _graph(9, n=60, m=300, dead=0)
    nodes = np.arange(n)
    q = np.zeros((n, 2))
    for j in range(2):
        sup = rng.choice(n, 5, replace=False)
        vals = rng.normal(size=5)
        q[sup, j] = vals - vals.mean()
    deg = np.bincount(src, minlength=n)
    P = gnn.propagation_operator(n, src, dst, C)
    hop = np.zeros(n, np.int64)
    F = gnn.features(n, src, dst, nodes, hop, q, np.zeros((n, 2)), np.ones(2), [-1, -1])
    ls, ld = gnn.local_edges(src, dst, nodes)
    theta = init_params(5, prior="propagation", c=C).astype(np.float64)
    res = gnn.residual_loss(theta, F, ls, ld, np.where(deg > 0, 1.0 / deg, 0.0), nodes, q, P, deg > 0, C)
    want = q.copy()
    for _ in range(4):
        want = P @ want
    # (the parameters are float32: (1-c) carries a relative error of 3e-8)
    assert np.abs(res["rho"] - want).max() <= 1e-5 * np.abs(want).max()
    assert np.all(np.abs(res["beta"]) < 1e-6)
    assert res["loss"] < 0.5


def test_offset_support_closed_forms():
    # u has out-neighbours {1, 2, 3}; r_old(u) != 0
    n = 6
    src = np.array([0, 0, 0, 4], np.int64)
    dst = np.array([1, 2, 3, 5], np.int64)
    r = np.zeros((n, 1))
    r[0] = 0.3
    old = (n, src, dst)
    # insertion of (0, 4): every old neighbour changes weight, and 4 is new
    new = oracle.apply_batch(n, src, dst, _b([0], [4], [], []))
    assert list(gnn.offset_support(old, new, r)) == [1, 2, 3, 4]
    # one insertion and one deletion in the same row: the degree is kept,
    # only the two changed entries move
    new = oracle.apply_batch(n, src, dst, _b([0], [4], [0], [2]))
    assert list(gnn.offset_support(old, new, r)) == [2, 4]
    # a changed row with a zero score moves nothing
    new = oracle.apply_batch(n, src, dst, _b([4], [1], [], []))
    assert list(gnn.offset_support(old, new, r)) == []


def _b(isrc, idst, dsrc, ddst, n_new=0):
    from synth.stream import Batch

    a = lambda x: np.array(x, np.int32)  # noqa: E731
    return Batch(a(isrc), a(idst), a(dsrc), a(ddst), n_new)


def test_features_closed_forms():
    # a path 0 -> 1 -> 2 plus 2 -> 0 and a dead end 3 with an edge 1 -> 3
    n = 4
    src = np.array([0, 1, 2, 1], np.int64)
    dst = np.array([1, 2, 0, 3], np.int64)
    q = np.array([[0.0], [0.5], [-0.25], [-0.25]])
    r = np.array([[0.4], [0.3], [0.2], [0.1]])
    F = gnn.features(n, src, dst, np.array([1, 3]), np.array([0, 2]), q, r, np.array([1.0]), [1])
    f1, f3 = F[0, 0], F[1, 0]
    assert f1[0] == pytest.approx(np.log(2) / 8, rel=1e-6) and f1[1] == pytest.approx(np.log(3) / 8, rel=1e-6)
    assert f1[2] == pytest.approx(0.5) and f1[3] == pytest.approx(0.5)
    assert f3[2] == pytest.approx(-0.25) and f3[3] == pytest.approx(0.25)
    assert f1[4] == pytest.approx(np.log1p(1.2) / 8, rel=1e-6)
    assert list(f1[5:9]) == [1, 0, 0, 0] and list(f3[5:9]) == [0, 0, 1, 0]
    assert f1[9] == 0 and f3[9] == 1
    assert f1[10] == 1 and f3[10] == 0
    assert f1[11] == pytest.approx(0.5) and f3[11] == 0
    assert f1[12] == pytest.approx(1.0) and f3[12] == pytest.approx(1.0)
    assert f1[13] == pytest.approx(0.5 * np.log(2) / 8, rel=1e-6)
    assert f1[14] == pytest.approx(0.5 * np.log(3) / 8, rel=1e-6)
    assert f3[15] == pytest.approx(-0.25 * np.log(2) / 8, rel=1e-6)
