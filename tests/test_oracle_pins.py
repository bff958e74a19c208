"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each checks a closed form, a
textbook solve, an invariant or a bound that the paper states, so that a
dropped factor, a transposed operand, a wrong dead-end rule or a wrong loop
start in the oracle fails at least one of them.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle.core import RENORM_ALWAYS, RENORM_NEVER, RENORM_PAPER, OracleError
from synth.stream import Batch

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_graph(rng, n, m, dead_frac=0.0, self_loops=False):
    """Random simple directed graph; a fraction of nodes keep no out-edges."""
    keys = set()
    dead = set(rng.choice(n, size=int(dead_frac * n), replace=False).tolist()) if dead_frac else set()
    while len(keys) < m:
        u, v = int(rng.integers(n)), int(rng.integers(n))
        if u in dead or (u == v and not self_loops):
            continue
        keys.add((u, v))
    e = np.array(sorted(keys), dtype=np.int32)
    rng.shuffle(e)
    return e[:, 0].copy(), e[:, 1].copy()


def _no_dead_ends(n, src, dst, rng):
    """Give every node without out-edges one random out-edge."""
    deg = np.bincount(src, minlength=n)
    add_s, add_d = [], []
    for u in np.nonzero(deg == 0)[0]:
        v = int(rng.integers(n))
        while v == u:
            v = int(rng.integers(n))
        add_s.append(u)
        add_d.append(v)
    return np.concatenate([src, np.array(add_s, np.int32)]), np.concatenate([dst, np.array(add_d, np.int32)])


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n,c", [(7, 0.15), (12, 0.05), (3, 0.5)])
def test_directed_cycle_closed_form(n, c):
    # 0 -> 1 -> ... -> n-1 -> 0, seed 0: the walk reaches node k after exactly
    # k, k+n, k+2n, ... steps, so r(k) = c (1-c)^k / (1 - (1-c)^n).
    src = np.arange(n, dtype=np.int32)
    dst = (src + 1) % n
    expect = np.array([c * (1 - c) ** k / (1 - (1 - c) ** n) for k in range(n)])
    r = oracle.rwr_static(n, src, dst, 0, c)
    # the static solve stops at ||x||_1 <= 1e-14: its tail is <= (1-c)/c * 1e-14
    assert np.abs(r - expect).sum() < (1 - c) / c * 1e-14 + 1e-14
    rd = oracle.rwr_dense(n, src, dst, 0, c)
    assert np.abs(rd - expect).sum() < 1e-13


@pytest.mark.parametrize("leaves,c", [(5, 0.15), (40, 0.05)])
def test_undirected_star_closed_form(leaves, c):
    # centre 0 with `leaves` leaves, each edge stored in both directions;
    # seed = centre: r(centre) = 1/(2-c), r(leaf) = (1-c)/((2-c) * leaves).
    n = leaves + 1
    a = np.zeros(leaves, dtype=np.int32)
    b = np.arange(1, n, dtype=np.int32)
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    tail = (1 - c) / c * 1e-14  # truncation of the static solve at 1e-14
    r = oracle.rwr_static(n, src, dst, 0, c)
    assert abs(r[0] - 1 / (2 - c)) < tail
    assert np.abs(r[1:] - (1 - c) / ((2 - c) * leaves)).sum() < tail
    rd = oracle.rwr_dense(n, src, dst, 0, c)
    assert abs(rd[0] - 1 / (2 - c)) < 1e-15
    assert np.abs(rd[1:] - (1 - c) / ((2 - c) * leaves)).max() < 1e-15


@pytest.mark.parametrize("c", [0.15, 0.3])
def test_two_node_dead_end_closed_form(c):
    # 0 -> 1, node 1 is a dead end, seed 0.  Sub-stochastic scores are
    # [c, c(1-c)]; Theorem 4 divides by their sum: [1/(2-c), (1-c)/(2-c)].
    src = np.array([0], np.int32)
    dst = np.array([1], np.int32)
    r = oracle.rwr_static(2, src, dst, 0, c)
    assert np.allclose(r, [1 / (2 - c), (1 - c) / (2 - c)], rtol=0, atol=1e-15)
    # without the normalisation the series sums to [c, c(1-c)]
    q = np.array([c, 0.0])
    raw, it = oracle.cpi(2, src, dst, q, c, 1e-15)
    assert np.allclose(raw, [c, c * (1 - c)], atol=1e-16)
    assert it == 2  # x^(1) = (0, c(1-c)), x^(2) = 0


def test_table3_cpi_iteration_count():
    g = json.load(open(os.path.join(GOLDEN, "table3_cpi.json")))
    c, eps = g["c"], g["eps"]
    rng = np.random.default_rng(11)
    n = 300
    src, dst = _no_dead_ends(n, *_rand_graph(rng, n, 1500), rng)
    q = np.zeros(n)
    q[5] = c
    r, it, norms = oracle.cpi(n, src, dst, q, c, eps, with_norms=True)
    assert it == g["iterations"]
    # with no dead ends A~^T is column stochastic: ||x^(i)||_1 = c (1-c)^i
    expect = c * (1 - c) ** np.arange(it + 1)
    assert np.abs(norms / expect - 1).max() < 1e-12


# ------------------------------------------------------------- library solves

@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("dead_frac", [0.0, 0.2])
def test_cpi_matches_dense_lu(seed, dead_frac):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(20, 200))
    m = int(rng.integers(n, 6 * n))
    src, dst = _rand_graph(rng, n, m, dead_frac=dead_frac, self_loops=True)
    s = int(src[0])
    for c in (0.15, 0.05):
        r = oracle.rwr_static(n, src, dst, s, c)
        rd = oracle.rwr_dense(n, src, dst, s, c)
        assert np.abs(r - rd).sum() < 1e-12


def test_mass_is_one_without_dead_ends():
    rng = np.random.default_rng(3)
    n = 150
    src, dst = _no_dead_ends(n, *_rand_graph(rng, n, 500), rng)
    q = np.zeros(n)
    q[7] = 0.15
    r, _ = oracle.cpi(n, src, dst, q, 0.15, 1e-14)
    assert abs(r.sum() - 1) < 1e-12
    assert not oracle.dead_end_reachable(n, src, dst, 7)


def test_dead_end_normalisation_equals_explicit_restart_edges():
    # Theorem 4: normalising the sub-stochastic scores gives the scores of the
    # graph in which every dead end has one edge back to the seed.
    rng = np.random.default_rng(5)
    n = 120
    src, dst = _rand_graph(rng, n, 300, dead_frac=0.3)
    s = int(src[0])
    deg = np.bincount(src, minlength=n)
    dead = np.nonzero(deg == 0)[0].astype(np.int32)
    assert dead.size > 0
    src2 = np.concatenate([src, dead])
    dst2 = np.concatenate([dst, np.full(dead.size, s, np.int32)])
    for c in (0.15, 0.05):
        r = oracle.rwr_static(n, src, dst, s, c)
        r2 = oracle.rwr_static(n, src2, dst2, s, c)
        assert np.abs(r - r2).sum() < 1e-12
        assert abs(r.sum() - 1) < 1e-12


def test_undirected_reversibility():
    # undirected graph, no isolated node: d(s) r_s(v) = d(v) r_v(s)
    rng = np.random.default_rng(9)
    n = 60
    pairs = set()
    for u in range(n):  # a ring keeps every node connected
        pairs.add((min(u, (u + 1) % n), max(u, (u + 1) % n)))
    while len(pairs) < 200:
        u, v = int(rng.integers(n)), int(rng.integers(n))
        if u != v:
            pairs.add((min(u, v), max(u, v)))
    p = np.array(sorted(pairs), np.int32)
    src = np.concatenate([p[:, 0], p[:, 1]])
    dst = np.concatenate([p[:, 1], p[:, 0]])
    deg = np.bincount(src, minlength=n)
    c = 0.15
    R = np.stack([oracle.rwr_static(n, src, dst, s, c) for s in range(n)])  # R[s, v] = r_s(v)
    lhs = deg[:, None] * R
    assert np.abs(lhs - lhs.T).max() < 1e-13


# ------------------------------------------------------------------ OSP pins

def _mixed_batch(rng, n, src, dst, n_ins, n_del, n_new=0, out_only_new=True):
    cur = set(zip(src.tolist(), dst.tolist()))
    dels = [tuple(e) for e in np.array(list(cur))[rng.choice(len(cur), size=n_del, replace=False)]]
    ins = set()
    n2 = n + n_new
    while len(ins) < n_ins:
        u, v = int(rng.integers(n)), int(rng.integers(n))
        if (u, v) not in cur and (u, v) not in ins:
            ins.add((u, v))
    for w in range(n, n2):
        for v in rng.choice(n, size=int(rng.integers(1, 4)), replace=False):
            ins.add((w, int(v)))
        if not out_only_new:
            ins.add((int(rng.integers(n)), w))
    ins = sorted(ins)
    return Batch(
        ins_src=np.array([e[0] for e in ins], np.int32), ins_dst=np.array([e[1] for e in ins], np.int32),
        del_src=np.array([e[0] for e in dels], np.int32), del_dst=np.array([e[1] for e in dels], np.int32),
        n_new_nodes=n_new,
    )


@pytest.mark.parametrize("seed", range(8))
def test_theorem1_osp_is_exact(seed):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(30, 150))
    src, dst = _rand_graph(rng, n, 4 * n, dead_frac=0.1 * (seed % 3), self_loops=True)
    s = int(src[0])
    c = 0.15 if seed % 2 else 0.05
    r_old = oracle.rwr_static(n, src, dst, s, c)
    b = _mixed_batch(rng, n, src, dst, n_ins=int(rng.integers(0, 10)), n_del=int(rng.integers(0, 10)),
                     n_new=int(rng.integers(0, 3)), out_only_new=bool(seed % 2))
    n2, s2, d2 = oracle.apply_batch(n, src, dst, b)
    out = oracle.osp((n, src, dst), (n2, s2, d2), r_old, c, 1e-16, renorm=RENORM_ALWAYS)
    r_new = oracle.rwr_static(n2, s2, d2, s, c)
    assert np.abs(out["r_new"] - r_new).sum() < 1e-12
    # q_offset is (1-c)(B~^T - A~^T) r_old: check it against dense matrices
    A = np.zeros((n2, n2))
    A[:n, :n] = oracle.row_normalised_dense(n, src, dst)
    B = oracle.row_normalised_dense(n2, s2, d2)
    r0 = np.concatenate([r_old, np.zeros(n2 - n)])
    assert np.abs(out["q_off"] - (1 - c) * (B.T - A.T) @ r0).max() < 1e-16


def test_theorem4_paper_reading_breaks_when_dead_end_disappears():
    # The stored r_old is already normalised.  If the update removes the only
    # reachable dead end, the new sub-stochastic system has mass 1 and the
    # paper's rule (normalise only when a dead end is reachable) would keep
    # the stale scale; dividing by the sum always is exact.
    src = np.array([0, 1, 2], np.int32)
    dst = np.array([1, 2, 0], np.int32)
    src = np.concatenate([src, [0]]).astype(np.int32)
    dst = np.concatenate([dst, [3]]).astype(np.int32)  # node 3 is a dead end
    n, c = 4, 0.15
    r_old = oracle.rwr_static(n, src, dst, 0, c)
    b = Batch(ins_src=np.array([3], np.int32), ins_dst=np.array([0], np.int32),
              del_src=np.zeros(0, np.int32), del_dst=np.zeros(0, np.int32))
    n2, s2, d2 = oracle.apply_batch(n, src, dst, b)
    exact = oracle.rwr_static(n2, s2, d2, 0, c)
    good = oracle.osp((n, src, dst), (n2, s2, d2), r_old, c, 1e-16, renorm=RENORM_ALWAYS, seed=0)
    paper = oracle.osp((n, src, dst), (n2, s2, d2), r_old, c, 1e-16, renorm=RENORM_PAPER, seed=0)
    assert np.abs(good["r_new"] - exact).sum() < 1e-13
    assert np.abs(paper["r_new"] - exact).sum() > 1e-3


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("eps", [1e-3, 1e-6])
def test_theorem2_3_osp_t_bounds(seed, eps):
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(50, 200))
    src, dst = _rand_graph(rng, n, 5 * n, dead_frac=0.05 * (seed % 2))
    s = int(src[0])
    c = 0.15
    r_old = oracle.rwr_static(n, src, dst, s, c)
    b = _mixed_batch(rng, n, src, dst, n_ins=int(rng.integers(1, 20)), n_del=int(rng.integers(1, 20)))
    n2, s2, d2 = oracle.apply_batch(n, src, dst, b)
    out = oracle.osp((n, src, dst), (n2, s2, d2), r_old, c, eps, renorm=RENORM_ALWAYS)
    qn = out["norms"][0]
    assert qn <= 2 * (1 - c) + 1e-15
    # Theorem 2: ||x^(i)||_1 <= (1-c)^i ||q_offset||_1, hence the count bound
    i = np.arange(out["iters"] + 1)
    assert np.all(out["norms"] <= (1 - c) ** i * qn * (1 + 1e-12))
    bound = max(1, math.ceil(math.log(eps / qn) / math.log(1 - c))) if qn > eps else 1
    assert out["iters"] <= bound
    assert out["iters"] < math.log(eps / 2) / math.log(1 - c)
    # Theorem 3 (error O(eps/c)); with the normalisation the bound is 2eps/c
    exact = oracle.rwr_static(n2, s2, d2, s, c)
    assert np.abs(out["r_new"] - exact).sum() <= 2 * eps / c
    # un-normalised, the truncation tail alone is below (1-c)/c * ||x^(k)||_1
    raw = oracle.osp((n, src, dst), (n2, s2, d2), r_old, c, eps, renorm=RENORM_NEVER)
    full = oracle.osp((n, src, dst), (n2, s2, d2), r_old, c, 1e-17, renorm=RENORM_NEVER)
    tail = np.abs(raw["r_new"] - full["r_new"]).sum()
    assert tail <= (1 - c) / c * raw["norms"][-1] * (1 + 1e-9) + 1e-15


@pytest.mark.parametrize("d", [1, 2, 5, 9])
def test_single_edge_offset_norms(d):
    # node 0 has d out-edges; scores r_old arbitrary positive
    c = 0.15
    n = 12
    src = np.zeros(d, np.int32)
    dst = np.arange(1, d + 1, dtype=np.int32)
    rest_s = np.arange(1, n, dtype=np.int32)
    rest_d = np.zeros(n - 1, np.int32)  # every other node points back to 0
    S = np.concatenate([src, rest_s])
    D = np.concatenate([dst, rest_d])
    r_old = np.linspace(1.0, 2.0, n) / np.linspace(1.0, 2.0, n).sum()
    ins = Batch(ins_src=np.array([0], np.int32), ins_dst=np.array([n - 1], np.int32),
                del_src=np.zeros(0, np.int32), del_dst=np.zeros(0, np.int32))
    n2, s2, d2 = oracle.apply_batch(n, S, D, ins)
    q = oracle.osp((n, S, D), (n2, s2, d2), r_old, c, 1.0, renorm=RENORM_NEVER)["q_off"]
    assert abs(np.abs(q).sum() - 2 * (1 - c) * r_old[0] / (d + 1)) < 1e-16
    assert abs(q.sum()) < 1e-16
    dele = Batch(ins_src=np.zeros(0, np.int32), ins_dst=np.zeros(0, np.int32),
                 del_src=np.array([0], np.int32), del_dst=np.array([1], np.int32))
    n2, s2, d2 = oracle.apply_batch(n, S, D, dele)
    q = oracle.osp((n, S, D), (n2, s2, d2), r_old, c, 1.0, renorm=RENORM_NEVER)["q_off"]
    if d >= 2:
        assert abs(np.abs(q).sum() - 2 * (1 - c) * r_old[0] / d) < 1e-16
        assert abs(q.sum()) < 1e-16
    else:  # the row empties: the node becomes a dead end
        assert abs(np.abs(q).sum() - (1 - c) * r_old[0]) < 1e-16
        assert abs(q.sum() + (1 - c) * r_old[0]) < 1e-16


def test_new_node_with_only_out_edges_changes_nothing():
    rng = np.random.default_rng(17)
    n = 80
    src, dst = _rand_graph(rng, n, 300)
    s = int(src[0])
    c = 0.15
    r_old = oracle.rwr_static(n, src, dst, s, c)
    b = Batch(ins_src=np.array([n, n, n], np.int32), ins_dst=np.array([3, 9, 40], np.int32),
              del_src=np.zeros(0, np.int32), del_dst=np.zeros(0, np.int32), n_new_nodes=1)
    n2, s2, d2 = oracle.apply_batch(n, src, dst, b)
    out = oracle.osp((n, src, dst), (n2, s2, d2), r_old, c, 1e-16, renorm=RENORM_ALWAYS)
    assert np.all(out["q_off"] == 0)
    assert np.abs(out["r_new"][:n] - r_old).max() < 1e-16
    assert out["r_new"][n] == 0


def test_apply_batch_validation():
    src = np.array([0, 1, 2], np.int32)
    dst = np.array([1, 2, 0], np.int32)
    E = np.zeros(0, np.int32)
    with pytest.raises(OracleError, match="EEXIST"):
        oracle.apply_batch(3, src, dst, Batch(np.array([0], np.int32), np.array([1], np.int32), E, E))
    with pytest.raises(OracleError, match="ENOENT"):
        oracle.apply_batch(3, src, dst, Batch(E, E, np.array([1], np.int32), np.array([0], np.int32)))
    with pytest.raises(OracleError, match="EINVAL"):
        oracle.apply_batch(3, src, dst, Batch(np.array([0], np.int32), np.array([7], np.int32), E, E))
    with pytest.raises(OracleError, match="EINVAL"):
        oracle.apply_batch(3, src, dst, Batch(np.array([0], np.int32), np.array([2], np.int32),
                                              np.array([0], np.int32), np.array([2], np.int32)))
    # node deletion removes every incident edge
    n2, s2, d2 = oracle.apply_batch(3, src, dst, Batch(E, E, E, E), del_nodes=[1])
    assert n2 == 3 and set(zip(s2.tolist(), d2.tolist())) == {(2, 0)}
    # ... and takes the list from the batch as well
    n2, s2, d2 = oracle.apply_batch(3, src, dst, Batch(E, E, E, E, del_nodes=np.array([1], np.int32)))
    assert set(zip(s2.tolist(), d2.tolist())) == {(2, 0)}
    # deleted nodes: existing ids, listed once, not named by the batch's edges
    for dn, b in (([3], Batch(E, E, E, E)), ([1, 1], Batch(E, E, E, E)),
                  ([1], Batch(np.array([1], np.int32), np.array([0], np.int32), E, E)),
                  ([2], Batch(E, E, np.array([2], np.int32), np.array([0], np.int32)))):
        with pytest.raises(OracleError, match="EINVAL"):
            oracle.apply_batch(3, src, dst, b, del_nodes=dn)


def test_node_deletion_equals_deleting_its_edges_and_osp_stays_exact():
    # Section 3.4.1: a deleted node's row and column become zero; Theorem 1:
    # OSP from the old scores reaches the static scores of the new graph
    rng = np.random.default_rng(11)
    n = 60
    pairs = {(int(u), int(v)) for u, v in rng.integers(0, n, size=(400, 2))}
    pairs |= {(u, u) for u in range(n) if not any(a == u for a, _ in pairs)}
    src = np.array([p[0] for p in sorted(pairs)], np.int32)
    dst = np.array([p[1] for p in sorted(pairs)], np.int32)
    E = np.zeros(0, np.int32)
    gone = [3, 17, 18]
    n2, s2, d2 = oracle.apply_batch(n, src, dst, Batch(E, E, E, E), del_nodes=gone)
    inc = np.isin(src, gone) | np.isin(dst, gone)
    n3, s3, d3 = oracle.apply_batch(n, src, dst, Batch(E, E, src[inc], dst[inc]))
    assert n2 == n3 == n
    assert set(zip(s2.tolist(), d2.tolist())) == set(zip(s3.tolist(), d3.tolist()))
    assert not (np.isin(s2, gone) | np.isin(d2, gone)).any()
    seed = 0
    r_old = oracle.rwr_static(n, src, dst, seed, 0.15)
    out = oracle.osp((n, src, dst), (n2, s2, d2), r_old, 0.15, 1e-15, renorm=oracle.core.RENORM_ALWAYS)
    ref = oracle.rwr_static(n2, s2, d2, seed, 0.15)
    assert np.abs(out["r_new"] - ref).sum() < 1e-12
    # nothing reaches a deleted node any more
    assert np.abs(ref[gone]).max() < 1e-15


def test_literal_node_deletion_zeroes_the_row_only():
    # Section 3.4.1 read literally: the deleted node's row becomes zero and
    # its in-edges stay, so it turns into a dead end and Theorem 4's
    # rescaling applies; the same as deleting its out-edges, and OSP from
    # the old scores still reaches the static scores (Theorem 1)
    rng = np.random.default_rng(12)
    n = 50
    pairs = {(int(u), int(v)) for u, v in rng.integers(0, n, size=(300, 2))}
    pairs |= {(u, u) for u in range(n) if not any(a == u for a, _ in pairs)}
    src = np.array([p[0] for p in sorted(pairs)], np.int32)
    dst = np.array([p[1] for p in sorted(pairs)], np.int32)
    E = np.zeros(0, np.int32)
    gone = [4, 9]
    n2, s2, d2 = oracle.apply_batch(n, src, dst, Batch(E, E, E, E), del_nodes=gone, rows_only=True)
    out_e = np.isin(src, gone)
    n3, s3, d3 = oracle.apply_batch(n, src, dst, Batch(E, E, src[out_e], dst[out_e]))
    assert set(zip(s2.tolist(), d2.tolist())) == set(zip(s3.tolist(), d3.tolist()))
    assert not np.isin(s2, gone).any() and np.isin(d2, gone).any()  # in-edges stay
    # every node lost its whole row in the default reading instead
    n4, s4, d4 = oracle.apply_batch(n, src, dst, Batch(E, E, E, E), del_nodes=gone)
    assert s4.shape[0] < s2.shape[0]
    seed = 0
    r_old = oracle.rwr_static(n, src, dst, seed, 0.15)
    out = oracle.osp((n, src, dst), (n2, s2, d2), r_old, 0.15, 1e-15, renorm=oracle.core.RENORM_ALWAYS)
    ref = oracle.rwr_static(n2, s2, d2, seed, 0.15)
    assert np.abs(out["r_new"] - ref).sum() < 1e-12
    assert abs(ref.sum() - 1.0) < 1e-12  # Theorem 4: the dead ends rescale to unit mass


def test_apply_stream_equals_batch_by_batch():
    # the one-pass stream apply gives the same edge set as applying each
    # batch in turn, and rejects a batch that is invalid at its position
    from synth import EdgeSetModel, rmat_graph
    from synth.stream import mixed_batch, single_edge_stream

    g = rmat_graph(9, 3000, dead_end_self_loops=True)
    model = EdgeSetModel(g.n, g.src, g.dst)
    stream = single_edge_stream(model, 40)
    rng = np.random.default_rng(3)
    stream += [mixed_batch(rng, model, 15, 15, n_new_nodes=2) for _ in range(3)]
    n, s, d = g.n, g.src, g.dst
    for b in stream:
        n, s, d = oracle.apply_batch(n, s, d, b)
    n2, s2, d2 = oracle.apply_stream(g.n, g.src, g.dst, stream)
    assert n2 == n and s2.shape[0] == s.shape[0]
    assert set(zip(s.tolist(), d.tolist())) == set(zip(s2.tolist(), d2.tolist()))
    E = np.zeros(0, np.int32)
    # re-inserting an edge deleted earlier in the stream is valid; deleting it
    # twice is not
    dels = [b for b in stream if b.n_del == 1]
    u, v = int(dels[0].del_src[0]), int(dels[0].del_dst[0])
    again = Batch(np.array([u], np.int32), np.array([v], np.int32), E, E)
    oracle.apply_stream(g.n, g.src, g.dst, stream + [again])
    with pytest.raises(OracleError, match="ENOENT"):
        oracle.apply_stream(g.n, g.src, g.dst, stream + [Batch(E, E, np.array([u], np.int32),
                                                               np.array([v], np.int32))])
