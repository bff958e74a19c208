"""Pins of the learned-warm-start oracle (oracle/gnn.py): finite differences
for every gradient, adjointness of the aggregation, the residual identity
that keeps OSP exact, bfloat16 rounding, the region search and AdamW."""

import numpy as np
import pytest

from oracle import gnn


def _tiny(seed=0, nR=9, S=2, m=20):
    rng = np.random.default_rng(seed)
    F = rng.normal(size=(nR, S, gnn.FEAT))
    src = rng.integers(0, nR, m)
    dst = rng.integers(0, nR, m)
    dinv = 1.0 / rng.integers(1, 6, nR)
    dinv[0] = 0.0  # a dead end
    theta = gnn.init_params(seed + 1)
    # non-zero biases so that every code path carries signal
    p = gnn.unpack(theta)
    for k in gnn.ORDER:
        if k.startswith("b"):
            p[k] = rng.normal(scale=0.1, size=p[k].shape)
    theta = gnn.pack(p)
    t = rng.normal(scale=0.5, size=(nR, S))
    return theta, F, src, dst, dinv, t


def _loss(theta, F, src, dst, dinv, t, active):
    o, _ = gnn.forward(theta, F, src, dst, dinv)
    return gnn.loss(o, t, active)[0]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_backward_matches_central_differences(seed):
    theta, F, src, dst, dinv, t = _tiny(seed)
    active = np.array([True, seed != 1])
    o, cache = gnn.forward(theta, F, src, dst, dinv)
    # Huber in its quadratic zone for part of the entries, linear elsewhere
    L, do = gnn.loss(o, t, active)
    g = gnn.backward(theta, F, src, dst, dinv, cache, do)
    rng = np.random.default_rng(100 + seed)
    h = 1e-6
    # every parameter block, coordinate-wise on a sample, plus random directions
    off = 0
    for k in gnn.ORDER:
        n = int(np.prod(gnn.SHAPES[k]))
        for i in rng.choice(n, size=min(n, 4), replace=False):
            e = np.zeros_like(theta)
            e[off + i] = h
            fd = (_loss(theta + e, F, src, dst, dinv, t, active) - _loss(theta - e, F, src, dst, dinv, t, active)) / (2 * h)
            assert abs(fd - g[off + i]) <= 1e-6 * max(1.0, abs(fd)), (k, i, fd, g[off + i])
        off += n
    for _ in range(3):
        d = rng.normal(size=theta.shape)
        d /= np.linalg.norm(d)
        fd = (_loss(theta + h * d, F, src, dst, dinv, t, active) - _loss(theta - h * d, F, src, dst, dinv, t, active)) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * max(1.0, abs(fd))


def test_aggregation_adjoint():
    rng = np.random.default_rng(4)
    nR, S = 11, 3
    src = rng.integers(0, nR, 40)
    dst = rng.integers(0, nR, 40)
    dinv = rng.uniform(0, 1, nR)
    m = rng.normal(size=(nR, S, gnn.MSG))
    da = rng.normal(size=(nR, S, gnn.MSG))
    lhs = np.sum(gnn.aggregate(m, src, dst, dinv, nR) * da)
    rhs = np.sum(m * gnn.aggregate_t(da, src, dst, dinv, nR))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_residual_keeps_offset_exact():
    # r_offset = xhat + sum_i P^i rho for ANY xhat (Section 3.1's series with
    # the seed replaced by the residual); checked against a dense solve
    rng = np.random.default_rng(7)
    n, c = 30, 0.15
    A = (rng.uniform(size=(n, n)) < 0.15).astype(float)
    deg = A.sum(axis=1)
    At = np.where(deg[:, None] > 0, A / np.maximum(deg, 1)[:, None], 0.0)
    P = (1 - c) * At.T
    q = rng.normal(size=n)
    q -= q.mean()
    xhat = rng.normal(size=n)
    rho = gnn.residual(q, xhat, P)
    series = np.zeros(n)
    x = rho.copy()
    for _ in range(2000):
        series += x
        x = P @ x
    exact = np.linalg.solve(np.eye(n) - P, q)
    assert np.abs(xhat + series - exact).sum() < 1e-10
    # the perfect prediction leaves no residual
    assert np.abs(gnn.residual(q, exact, P)).sum() < 1e-12


def test_bf16_rounding():
    one = 1.0
    ulp = 2.0 ** -7
    vals = np.array([one, one + ulp / 2, one + ulp / 2 + 2 ** -20, one + 1.5 * ulp, -3.0, 0.0, 1e-30])
    r = gnn.bf16(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0  # tie to even
    assert r[2] == one + ulp  # above the tie
    assert r[3] == one + 2 * ulp  # tie to even (odd neighbour below)
    assert r[4] == -3.0 and r[5] == 0.0
    assert abs(r[6] - 1e-30) < 1e-30 * 2 ** -7


def test_region_levels_and_cap():
    # path 0 -> 1 -> 2 -> 3 -> 4 plus 0 -> 5: hop = out-distance from the start
    src = np.array([0, 1, 2, 3, 0])
    dst = np.array([1, 2, 3, 4, 5])
    nodes, hop = gnn.region(6, src, dst, [0], hops=3, cap=100)
    assert dict(zip(nodes.tolist(), hop.tolist())) == {0: 0, 1: 1, 5: 1, 2: 2, 3: 3}
    # a level that does not fit is left out entirely
    nodes, hop = gnn.region(6, src, dst, [0], hops=3, cap=2)
    assert nodes.tolist() == [0]
    nodes, hop = gnn.region(6, src, dst, [0], hops=3, cap=3)
    assert nodes.tolist() == [0, 1, 5]


def test_adamw_first_step():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    th, m, v = gnn.adamw(theta, g, np.zeros(3), np.zeros(3), 1, lr=0.01, wd=0.1)
    # the bias-corrected first step moves each coordinate by lr * sign(g),
    # plus decoupled decay lr * wd * theta
    expect = theta - 0.01 * (np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8) + 0.1 * theta)
    assert np.allclose(th, expect, rtol=0, atol=1e-12)


def test_parameter_count_and_layout():
    assert gnn.N_PARAMS == 16 * 64 + 64 + 3 * (64 * 16 + 64 * 64 + 16 * 64 + 64) + 64 + 1
    theta = gnn.init_params(5)
    assert np.array_equal(gnn.pack(gnn.unpack(theta)), theta)
    # identical inputs in two columns give identical outputs (weights shared
    # across seed columns); permuting region nodes permutes the outputs
    _, F, src, dst, dinv, _ = _tiny(3, S=2)
    F[:, 1] = F[:, 0]
    o, _ = gnn.forward(theta, F, src, dst, dinv)
    assert np.allclose(o[:, 0], o[:, 1])
    perm = np.random.default_rng(0).permutation(F.shape[0])
    inv = np.argsort(perm)
    o2, _ = gnn.forward(theta, F[perm], inv[src], inv[dst], dinv[perm])
    assert np.allclose(o2, o[perm], atol=1e-13)
