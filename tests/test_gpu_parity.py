"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs."""

import os

import numpy as np
import pytest

import oracle
from oracle.core import RENORM_ALWAYS
from synth import EdgeSetModel, rmat_graph
from synth.stream import Batch, mixed_batch, single_edge_stream

pytestmark = pytest.mark.gpu

rwr = pytest.importorskip("paper_1712_00595_amd.rwr")


def _ctx(g, seeds, **kw):
    return rwr.Context(g.n, g.src, g.dst, seeds, **kw)


def _l1(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).sum())


def _batch(rng, n, src, dst, n_ins, n_del, n_new=0):
    model = EdgeSetModel(n, src, dst)
    return mixed_batch(rng, model, n_ins, n_del, n_new_nodes=n_new)


# ---------------------------------------------------------------- static build

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n_seeds", [1, 3])
def test_static_build_matches_oracle(prec, n_seeds):
    print(f"[static] prec={prec} seeds={n_seeds}", flush=True)
    g = rmat_graph(10, 6000, dead_end_self_loops=(n_seeds == 1))
    seeds = np.array([int(np.argmax(g.out_degree()))] + [5, 77][: n_seeds - 1], np.int32)
    tol = 1e-12
    with _ctx(g, seeds, c=0.15, eps=1e-10, precision=prec, build_tol=tol) as ctx:
        for j, s in enumerate(seeds):
            r = ctx.scores(j)
            ref = oracle.rwr_static(g.n, g.src, g.dst, int(s), 0.15)
            assert _l1(r, ref) < tol + 1e-13


# ---------------------------------------------------- one exact batch (FP64)

def test_rmat13_one_batch_exact_fp64():
    print("[rmat13 exact]", flush=True)
    from synth.configs import RMAT13_ONE_BATCH, one_batch_rmat13

    w = RMAT13_ONE_BATCH
    g = w.graph()
    seeds = w.seeds(g)
    model = w.model(g)
    b = one_batch_rmat13(model)
    with _ctx(g, seeds, c=w.c, eps=1e-14, precision="fp64", build_tol=1e-13, err_budget=4e-13) as ctx:
        r0 = ctx.scores(0)
        ref0 = oracle.rwr_static(g.n, g.src, g.dst, int(seeds[0]), w.c)
        assert _l1(r0, ref0) < 1e-12
        st = ctx.update_batch(b)
        n2, s2, d2 = oracle.apply_batch(g.n, g.src, g.dst, b)
        ref = oracle.rwr_static(n2, s2, d2, int(seeds[0]), w.c)
        r = ctx.scores(0)
        assert _l1(r, ref) < 1e-12, st
        # structure after the batch equals G + Delta G
        es, ed, deg = ctx.export()
        assert set(zip(es.tolist(), ed.tolist())) == set(zip(s2.tolist(), d2.tolist()))
        assert np.array_equal(deg, np.bincount(s2, minlength=n2))
        # per-iteration norms against the Algorithm 1 twin started from the
        # oracle's exact scores
        twin = oracle.osp((g.n, g.src, g.dst), (n2, s2, d2), ref0, w.c, 1e-14, renorm=RENORM_ALWAYS)
        norms = ctx.last_norms(0)
        assert norms.shape[0] == twin["norms"].shape[0]
        assert np.allclose(norms, twin["norms"], rtol=1e-9, atol=1e-17)


@pytest.mark.parametrize("prec,reorder", [("fp32", True), ("fp64", True), ("fp32", False)])
def test_twin_norms_and_iterations(prec, reorder):
    print(f"[twin] prec={prec} reorder={reorder}", flush=True)
    g = rmat_graph(12, 40000, dead_end_self_loops=True)
    s = int(np.argmax(g.out_degree()))
    rng = np.random.default_rng(7)
    b = _batch(rng, g.n, g.src, g.dst, 20, 20)
    eps = 1e-9
    with _ctx(g, [s], eps=eps, precision=prec, build_tol=1e-13, reorder=reorder) as ctx:
        r_old = oracle.rwr_static(g.n, g.src, g.dst, s, 0.15)
        ctx.update_batch(b)
        n2, s2, d2 = oracle.apply_batch(g.n, g.src, g.dst, b)
        twin = oracle.osp((g.n, g.src, g.dst), (n2, s2, d2), r_old, 0.15, eps, renorm=RENORM_ALWAYS)
        norms = ctx.last_norms(0)
        k = min(norms.shape[0], twin["norms"].shape[0])
        assert abs(norms.shape[0] - twin["norms"].shape[0]) <= (0 if prec == "fp64" else 1)
        rtol = 1e-9 if prec == "fp64" else 2e-5
        assert np.allclose(norms[:k], twin["norms"][:k], rtol=rtol, atol=1e-18)
        ref = oracle.rwr_static(n2, s2, d2, s, 0.15)
        assert _l1(ctx.scores(0), ref) <= 2 * eps / 0.15


# --------------------------------------------------------------- error paths

def test_invalid_batches_leave_state_unchanged():
    print("[errors]", flush=True)
    g = rmat_graph(9, 3000, dead_end_self_loops=True)
    s = int(np.argmax(g.out_degree()))
    with _ctx(g, [s], eps=1e-10, precision="fp64") as ctx:
        before = ctx.scores(0)
        e_src, e_dst = int(g.src[0]), int(g.dst[0])
        cases = [
            ("RWR_EEXIST", dict(ins_src=[e_src], ins_dst=[e_dst])),
            ("RWR_ENOENT", dict(del_src=[e_dst], del_dst=[e_dst]) if e_dst != e_src else None),
            ("RWR_EINVAL", dict(ins_src=[0], ins_dst=[g.n + 5])),
            ("RWR_EINVAL", dict(ins_src=[1, 1], ins_dst=[2, 2])),
            ("RWR_EINVAL", dict(ins_src=[e_src], ins_dst=[e_dst], del_src=[e_src], del_dst=[e_dst])),
        ]
        for name, kw in cases:
            if kw is None:
                continue
            if name == "RWR_ENOENT":
                # pick a pair that is certainly absent
                model = EdgeSetModel(g.n, g.src, g.dst)
                u, v = 0, 1
                while model.has(u, v) or u == v:
                    v += 1
                kw = dict(del_src=[u], del_dst=[v])
            with pytest.raises(rwr.RwrError) as ei:
                ctx.update(**kw)
            assert ei.value.name == name, (name, kw)
        assert np.array_equal(ctx.scores(0), before)
        es, ed, _ = ctx.export()
        assert set(zip(es.tolist(), ed.tolist())) == set(zip(g.src.tolist(), g.dst.tolist()))


def test_new_node_with_only_out_edges():
    print("[new node]", flush=True)
    g = rmat_graph(9, 3000, dead_end_self_loops=True)
    s = int(np.argmax(g.out_degree()))
    with _ctx(g, [s], eps=1e-12, precision="fp64", build_tol=1e-13) as ctx:
        before = ctx.scores(0)
        st = ctx.update(ins_src=[g.n, g.n], ins_dst=[3, 9], n_new_nodes=1)
        after = ctx.scores(0)
        assert after.shape[0] == g.n + 1
        assert after[g.n] == 0.0
        assert np.abs(after[: g.n] - before).max() < 1e-15
        assert st["q_off_l1"] == 0.0


# ------------------------------------------------------------ streams / modes

@pytest.mark.parametrize("prec,n_seeds", [("fp32", 1), ("fp64", 3)])
def test_carried_residual_matches_oracle(monkeypatch, prec, n_seeds):
    # the residual evaluated after one update, or the last iterate an update
    # left unpropagated, joins a later update's first dense sweep; every
    # update stays within the gate against the oracle, the carried updates
    # included, and matches a context that never carries (RWR_CARRY: 2 both,
    # the default, 1 residual only, 0 off)
    print(f"[carry] prec={prec} seeds={n_seeds}", flush=True)
    g = rmat_graph(11, 20000, dead_end_self_loops=True)
    seeds = [int(v) for v in np.argsort(-g.out_degree())[:n_seeds]]
    model = EdgeSetModel(g.n, g.src, g.dst)
    rng = np.random.default_rng(11)
    # FP32: small batches, so that the rounding term leaves room below the
    # gate for the certified error and no refinement is needed
    k = 3 if prec == "fp32" else 30
    batches = [mixed_batch(rng, model, k, k, n_new_nodes=1 if t % 4 == 0 else 0) for t in range(12)]
    eps = 1e-9 if prec == "fp32" else 1e-12
    kw = dict(eps=eps, precision=prec) if prec == "fp32" else dict(eps=eps, precision=prec, build_tol=1e-12)
    gate = 2 * eps / 0.15
    finals = []
    for carry in ("2", "1", "0"):
        monkeypatch.setenv("RWR_CARRY", carry)
        n, src, dst = g.n, g.src, g.dst
        carried = 0
        with _ctx(g, seeds, **kw) as ctx:
            for t, b in enumerate(batches):
                st = ctx.update_batch(b)
                n, src, dst = oracle.apply_batch(n, src, dst, b)
                assert st["err_bound"] <= gate
                if st["carry_l1"] > 0.0:
                    carried += 1
                    assert st["q_off_l1"] <= (1 - 0.15) * st["dr_l1"] * (1 + 1e-9)
                if carry != "0" and (st["carry_l1"] > 0.0 or t == len(batches) - 1):
                    for j, sd in enumerate(seeds):
                        ref = oracle.rwr_static(n, src, dst, sd, 0.15)
                        err = _l1(ctx.scores(j), ref)
                        assert err <= st["err_bound"] + 1e-13, (t, j, err, st)
            finals.append([ctx.scores(j) for j in range(n_seeds)])
        if carry == "2":
            # every update after one that ended dense carries its last iterate
            assert carried >= len(batches) - 3, carried
        elif carry == "1":
            assert carried >= 3, carried
        else:
            assert carried == 0
    for other in finals[1:]:
        for a, b in zip(finals[0], other):
            assert _l1(a, b) <= 2 * gate


def test_carried_vector_through_errors_sparse_runs_and_warm_start():
    # a carried vector left by one update survives rejected batches and an
    # update whose run never reaches the dense phase (it stays pending), joins
    # the next dense run, and keeps joining with the learned warm start on
    # (the prediction's residual has a buffer of its own); the scores stay
    # within the reported bound of the oracle throughout
    print("[carry paths]", flush=True)
    from oracle import gnn

    g = rmat_graph(11, 20000, dead_end_self_loops=True)
    s = int(np.argmax(g.out_degree()))
    model = EdgeSetModel(g.n, g.src, g.dst)
    rng = np.random.default_rng(21)
    n, src, dst = g.n, g.src, g.dst

    def check(ctx, st, what):
        ref = oracle.rwr_static(n, src, dst, s, 0.15)
        err = _l1(ctx.scores(0), ref)
        assert err <= st["err_bound"] + 1e-13, (what, err, st)
        assert st["err_bound"] <= 2 * 1e-9 / 0.15, (what, st)

    with _ctx(g, [s], eps=1e-9, precision="fp32") as ctx:
        for t in range(2):
            b = mixed_batch(rng, model, 20, 20)
            st = ctx.update_batch(b)
            n, src, dst = oracle.apply_batch(n, src, dst, b)
            check(ctx, st, f"warm-up {t}")
        assert st["dense_iters"] > 0  # its last iterate is left for the next update
        before = ctx.scores(0)
        e_src, e_dst = int(src[0]), int(dst[0])
        with pytest.raises(rwr.RwrError):
            ctx.update(ins_src=[e_src], ins_dst=[e_dst])
        with pytest.raises(rwr.RwrError):
            ctx.update(ins_src=[0], ins_dst=[n + 5])
        assert np.array_equal(ctx.scores(0), before)
        # an edge out of a node with score 0: the offset seed is empty, the run
        # stays sparse and the carried vector stays pending
        sc = ctx.scores(0)
        u = int(np.flatnonzero(sc == 0.0)[0])
        w = next(v for v in range(g.n) if v != u and not model.has(u, v))
        b = Batch(np.array([u], np.int32), np.array([w], np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32), 0)
        model.insert(u, w)
        st = ctx.update_batch(b)
        n, src, dst = oracle.apply_batch(n, src, dst, b)
        assert st["dense_iters"] == 0 and st["carry_l1"] == 0.0, st
        check(ctx, st, "sparse run")
        b = mixed_batch(rng, model, 20, 20)
        st = ctx.update_batch(b)
        n, src, dst = oracle.apply_batch(n, src, dst, b)
        assert st["dense_iters"] > 0 and st["carry_l1"] > 0.0, st
        check(ctx, st, "joined")
        # the learned warm start (a network that predicts the offset seed)
        p = {k: np.zeros(gnn.SHAPES[k]) for k in gnn.ORDER}
        p["W0"][2, 0], p["W0"][2, 1] = 1.0, -1.0
        for layer in range(1, gnn.LAYERS + 1):
            p[f"Ws{layer}"][0, 0] = p[f"Ws{layer}"][1, 1] = 1.0
        p["wo"][0], p["wo"][1] = 1.0, -1.0
        ctx.model_set(gnn.pack(p).astype(np.float32))
        ctx.warm_start("predict", hops=2)
        joined = 0.0
        for t in range(3):
            b = mixed_batch(rng, model, 20, 20)
            st = ctx.update_batch(b)
            n, src, dst = oracle.apply_batch(n, src, dst, b)
            assert st["ws_region"] > 0 and st["ws_accepted"] == 1, st
            joined += st["carry_l1"]
            check(ctx, st, f"warm start {t}")
        assert joined > 0.0


@pytest.mark.parametrize("eps", [1e-6, 1e-9])
def test_single_edge_stream_within_gate(eps):
    print(f"[stream] eps={eps}", flush=True)
    g = rmat_graph(12, 40000, dead_end_self_loops=True)
    s = int(np.argmax(g.out_degree()))
    model = EdgeSetModel(g.n, g.src, g.dst)
    stream = single_edge_stream(model, 60, seed=4)
    gate = 2 * eps / 0.15
    n, src, dst = g.n, g.src, g.dst
    with _ctx(g, [s], eps=eps, precision="fp32") as ctx:
        for t, b in enumerate(stream):
            st = ctx.update_batch(b)
            n, src, dst = oracle.apply_batch(n, src, dst, b)
            assert st["err_bound"] <= gate
            if t in (0, 9, 59):
                ref = oracle.rwr_static(n, src, dst, s, 0.15)
                err = _l1(ctx.scores(0), ref)
                assert err <= gate, (t, err, st)
                assert err <= st["err_bound"] + 1e-13


def test_many_seeds_padded_columns():
    print("[seeds40]", flush=True)
    g = rmat_graph(10, 8000, dead_end_self_loops=True)
    from synth.rmat import sample_seeds

    seeds = sample_seeds(g, 40, seed=3)
    rng = np.random.default_rng(3)
    b = _batch(rng, g.n, g.src, g.dst, 30, 30, n_new=2)
    eps = 1e-8
    with _ctx(g, seeds, eps=eps, precision="fp32") as ctx:
        ctx.update_batch(b)
        n2, s2, d2 = oracle.apply_batch(g.n, g.src, g.dst, b)
        for j in (0, 17, 39):
            ref = oracle.rwr_static(n2, s2, d2, int(seeds[j]), 0.15)
            assert _l1(ctx.scores(j), ref) <= 2 * eps / 0.15


def test_undirected_mode():
    print("[undirected]", flush=True)
    g = rmat_graph(10, 5000, undirected=True)
    seeds = np.array([int(np.argmax(g.out_degree())), 11], np.int32)
    c = 0.05
    model = EdgeSetModel(g.n, g.pair_u, g.pair_v, undirected=True)
    rng = np.random.default_rng(5)
    b = mixed_batch(rng, model, 50, 50, n_new_nodes=3)
    with rwr.Context(g.n, g.pair_u, g.pair_v, seeds, c=c, eps=1e-12, precision="fp64", undirected=True,
                     build_tol=1e-12) as ctx:
        ctx.update_batch(b)
        n2, s2, d2 = oracle.apply_batch(g.n, g.src, g.dst, b, undirected=True)
        for j, s in enumerate(seeds):
            ref = oracle.rwr_static(n2, s2, d2, int(s), c)
            assert _l1(ctx.scores(j), ref) < 1e-10


def test_large_batch_device_sort_path():
    print("[large batch]", flush=True)
    g = rmat_graph(14, 200000, dead_end_self_loops=True)
    s = int(np.argmax(g.out_degree()))
    rng = np.random.default_rng(9)
    b = _batch(rng, g.n, g.src, g.dst, 3000, 3000, n_new=20)
    with _ctx(g, [s], eps=1e-13, precision="fp64", build_tol=1e-12, err_budget=1e-11) as ctx:
        ctx.update_batch(b)
        n2, s2, d2 = oracle.apply_batch(g.n, g.src, g.dst, b)
        ref = oracle.rwr_static(n2, s2, d2, s, 0.15)
        assert _l1(ctx.scores(0), ref) < 1e-11
        es, ed, _ = ctx.export()
        assert set(zip(es.tolist(), ed.tolist())) == set(zip(s2.tolist(), d2.tolist()))


def test_heavy_row_chunks(monkeypatch):
    print("[heavy]", flush=True)
    monkeypatch.setenv("RWR_HEAVY_LIMIT", "8")
    monkeypatch.setenv("RWR_HEAVY_CHUNK", "16")
    g = rmat_graph(11, 20000, dead_end_self_loops=True)
    seeds = np.array([int(np.argmax(g.out_degree())), 3], np.int32)
    rng = np.random.default_rng(1)
    b = _batch(rng, g.n, g.src, g.dst, 100, 100)
    for prec in ("fp64", "fp32"):
        with _ctx(g, seeds, eps=1e-12, precision=prec, build_tol=1e-12, err_budget=1e-11) as ctx:
            for j, sd in enumerate(seeds):
                ref = oracle.rwr_static(g.n, g.src, g.dst, int(sd), 0.15)
                assert _l1(ctx.scores(j), ref) < 1e-11
            ctx.update_batch(b)
            n2, s2, d2 = oracle.apply_batch(g.n, g.src, g.dst, b)
            for j, sd in enumerate(seeds):
                ref = oracle.rwr_static(n2, s2, d2, int(sd), 0.15)
                assert _l1(ctx.scores(j), ref) < 1e-11


def test_relayout_when_arena_fills():
    print("[relayout]", flush=True)
    rng = np.random.default_rng(2)
    g = rmat_graph(15, 60000, dead_end_self_loops=True)
    n = g.n
    s = int(np.argmax(g.out_degree()))
    src, dst = g.src, g.dst
    with _ctx(g, [s], eps=1e-12, precision="fp64", build_tol=1e-12, err_budget=1e-10) as ctx:
        hub = 7
        for rnd in range(3):
            model = EdgeSetModel(n, src, dst)
            # 3 x 9000 new out-edges of one row (of 32768 possible targets):
            # the row outgrows its slack, is moved to the arena twice, and the
            # third move exceeds the arena, which forces a relayout
            free = np.array([v for v in range(n) if v != hub and not model.has(hub, v)], np.int64)
            targets = rng.choice(free, size=9000, replace=False).tolist()
            b = Batch(ins_src=np.full(len(targets), hub, np.int32), ins_dst=np.array(targets, np.int32),
                      del_src=np.zeros(0, np.int32), del_dst=np.zeros(0, np.int32))
            ctx.update_batch(b)
            n, src, dst = oracle.apply_batch(n, src, dst, b)
        es, ed, deg = ctx.export()
        assert set(zip(es.tolist(), ed.tolist())) == set(zip(src.tolist(), dst.tolist()))
        ref = oracle.rwr_static(n, src, dst, s, 0.15)
        assert _l1(ctx.scores(0), ref) < 1e-10


@pytest.mark.parametrize("undirected", [False, True])
def test_hub_rows_batch_check_and_apply(undirected):
    """Rows above 4096 entries in batches of 256 keys or more are checked and
    rewritten by a workgroup each: deletions compact the hub's row (in both
    orientations when directed), a large insertion moves it to the arena, and
    a missing or an existing hub edge among many valid keys is rejected with
    the state kept."""
    print(f"[hub rows] undirected={undirected}", flush=True)
    rng = np.random.default_rng(31)
    base = rmat_graph(13, 30000, dead_end_self_loops=not undirected, undirected=undirected)
    n, hub = base.n, 5
    others = np.setdiff1d(np.arange(n), [hub])
    outs = rng.choice(others, 4500, replace=False)
    ins = rng.choice(others, 4500, replace=False)
    if undirected:
        pu = np.concatenate([base.pair_u, np.full(4500, hub)]).astype(np.int64)
        pv = np.concatenate([base.pair_v, outs]).astype(np.int64)
        key = np.unique(np.minimum(pu, pv) * n + np.maximum(pu, pv))
        eu, ev = (key // n).astype(np.int32), (key % n).astype(np.int32)
        loop = eu == ev
        src = np.concatenate([eu, ev[~loop]]).astype(np.int32)
        dst = np.concatenate([ev, eu[~loop]]).astype(np.int32)
    else:
        s0 = np.concatenate([base.src, np.full(4500, hub), ins]).astype(np.int64)
        d0 = np.concatenate([base.dst, outs, np.full(4500, hub)]).astype(np.int64)
        key = np.unique(s0 * n + d0)
        eu, ev = (key // n).astype(np.int32), (key % n).astype(np.int32)
        src, dst = eu, ev
    seeds = [hub, int(outs[0]), int(outs[1])]
    kw = dict(c=0.15, eps=1e-12, precision="fp64", build_tol=1e-12, err_budget=1e-10, undirected=undirected)
    E = np.zeros(0, np.int32)

    def edges():
        return set(zip(src.tolist(), dst.tolist()))

    def absent_from_hub(model, k, skip=()):
        out = []
        for v in rng.permutation(others).tolist():
            if not model.has(hub, v) and v not in skip:
                out.append(v)
                if len(out) == k:
                    break
        return out

    with rwr.Context(n, eu, ev, seeds, **kw) as ctx:
        model = EdgeSetModel(n, eu, ev, undirected=undirected)
        # 1: 500 hub out-edge (and, directed, 300 hub in-edge) deletions, 300
        #    new hub out-edges, 200 new edges away from the hub
        hub_out = [int(v) for v in outs if model.has(hub, int(v))][:500]
        d_s, d_d = [hub] * 500, hub_out
        if not undirected:
            hub_in = [int(u) for u in ins if model.has(int(u), hub) and int(u) not in set(hub_out)][:300]
            d_s, d_d = d_s + hub_in, d_d + [hub] * 300
        new_out = absent_from_hub(model, 300)
        far = set()
        while len(far) < 200:
            u, v = (int(x) for x in rng.integers(0, n, 2))
            if hub in (u, v) or u == v or model.has(u, v) or (v, u) in far or (u, v) in far:
                continue
            far.add((u, v))
        i_s = [hub] * 300 + [u for u, _ in far]
        i_d = new_out + [v for _, v in far]
        b1 = Batch(np.array(i_s, np.int32), np.array(i_d, np.int32), np.array(d_s, np.int32), np.array(d_d, np.int32))
        ctx.update_batch(b1)
        n, src, dst = oracle.apply_batch(n, src, dst, b1, undirected=undirected)
        assert set(zip(*[x.tolist() for x in ctx.export()[:2]])) == edges()
        # 2: 1500 more hub out-edges: the row outgrows its slack and moves
        model = EdgeSetModel(n, src, dst)
        b2 = Batch(np.full(1500, hub, np.int32), np.array(absent_from_hub(model, 1500), np.int32), E, E)
        ctx.update_batch(b2)
        n, src, dst = oracle.apply_batch(n, src, dst, b2, undirected=undirected)
        assert set(zip(*[x.tolist() for x in ctx.export()[:2]])) == edges()
        before = ctx.scores(0)
        model = EdgeSetModel(n, src, dst)
        fresh = absent_from_hub(model, 301)
        assert len(fresh) == 301
        gone, fresh = fresh[0], fresh[1:]
        present = next(v for v in rng.permutation(others).tolist() if model.has(hub, v))
        for name, extra in (("RWR_ENOENT", dict(del_src=[hub], del_dst=[gone])),
                            ("RWR_EEXIST", dict(ins_src=[hub] * 301, ins_dst=fresh + [present]))):
            kwb = dict(ins_src=[hub] * 300, ins_dst=fresh)
            kwb.update(extra)
            with pytest.raises(rwr.RwrError) as ei:
                ctx.update(**kwb)
            assert ei.value.name == name
        assert np.array_equal(ctx.scores(0), before)
        assert set(zip(*[x.tolist() for x in ctx.export()[:2]])) == edges()
        for j, sd in enumerate(seeds):
            assert _l1(ctx.scores(j), oracle.rwr_static(n, src, dst, sd, 0.15)) < 1e-9, j


# ------------------------------------------------------------- node deletion

@pytest.mark.parametrize("undirected", [False, True])
def test_node_deletion_matches_oracle(undirected):
    # Section 3.4.1: a deleted node's row and column become zero; exact
    # (FP64) update against the static scores of G + Delta G
    print(f"[node deletion] undirected={undirected}", flush=True)
    g = rmat_graph(12, 30000, dead_end_self_loops=not undirected, undirected=undirected)
    deg = g.out_degree()
    s = int(np.argmax(deg))
    order = np.argsort(-deg, kind="stable")
    # the second-largest hub, a few ordinary nodes, two adjacent nodes and a
    # node with a self-loop (when one exists)
    cand = [int(order[1]), int(order[50]), int(order[400])]
    u0, v0 = int(g.src[123]), int(g.dst[123])
    cand += [u0, v0]
    loops = g.src[g.src == g.dst]
    if loops.shape[0]:
        cand.append(int(loops[0]))
    dn = np.array(sorted({x for x in cand if x != s}), np.int32)
    rng = np.random.default_rng(5)
    E = np.zeros(0, np.int32)
    # edge entries elsewhere in the same batch (none names a deleted node)
    es, ed = (g.pair_u, g.pair_v) if undirected else (g.src, g.dst)
    model = EdgeSetModel(g.n, es, ed, undirected=undirected)
    ins_s, ins_d = [], []
    while len(ins_s) < 10:
        u, v = (int(x) for x in rng.integers(0, g.n, 2))
        if u == v or u in dn or v in dn or model.has(u, v) or (u, v) in zip(ins_s, ins_d) or \
                (undirected and (v, u) in zip(ins_s, ins_d)):
            continue
        ins_s.append(u)
        ins_d.append(v)
    b = Batch(np.array(ins_s, np.int32), np.array(ins_d, np.int32), E, E, 0, dn)
    with rwr.Context(g.n, es, ed, [s], c=0.15, eps=1e-14, precision="fp64", build_tol=1e-13, err_budget=4e-13,
                     undirected=undirected) as ctx:
        n0, m0 = ctx.n, ctx.m
        st = ctx.update_batch(b)
        n2, s2, d2 = oracle.apply_batch(g.n, g.src, g.dst, b, undirected=undirected)
        # the running edge count (read before an export recounts it)
        assert ctx.n == n0 and ctx.m == s2.shape[0], (m0, ctx.m, s2.shape[0])
        ref = oracle.rwr_static(n2, s2, d2, s, 0.15)
        assert _l1(ctx.scores(0), ref) < 1e-12, st
        es, ed, _ = ctx.export()
        assert set(zip(es.tolist(), ed.tolist())) == set(zip(s2.tolist(), d2.tolist()))
        # deleting a node that has no edges left is allowed and changes nothing
        before = ctx.scores(0)
        ctx.update_batch(Batch(E, E, E, E, 0, dn[:1]))
        assert _l1(ctx.scores(0), before) < 1e-13


def test_node_deletion_rejections_leave_state_unchanged():
    print("[node deletion errors]", flush=True)
    g = rmat_graph(10, 5000, dead_end_self_loops=True)
    s = int(np.argmax(g.out_degree()))
    E = np.zeros(0, np.int32)
    other = int(np.argsort(-g.out_degree())[3])
    u, v = int(g.src[7]), int(g.dst[7])
    bad = [
        Batch(E, E, E, E, 0, np.array([s], np.int32)),                      # a seed
        Batch(E, E, E, E, 0, np.array([other, other], np.int32)),           # listed twice
        Batch(E, E, E, E, 0, np.array([g.n], np.int32)),                    # out of range
        Batch(E, E, np.array([u], np.int32), np.array([v], np.int32), 0,    # edge names it
              np.array([u if u != s else v], np.int32)),
    ]
    with _ctx(g, [s], eps=1e-10, precision="fp64", build_tol=1e-12) as ctx:
        r0 = ctx.scores(0)
        es0, ed0, _ = ctx.export()
        for b in bad:
            with pytest.raises(rwr.RwrError) as ei:
                ctx.update_batch(b)
            assert ei.value.code == -1
        assert np.array_equal(ctx.scores(0), r0)
        es, ed, _ = ctx.export()
        assert np.array_equal(es, es0) and np.array_equal(ed, ed0)


# ------------------------------------------------- vectorised multi-column sweep

@pytest.mark.parametrize("n_seeds,prec,lanes", [
    (5, "fp32", 32), (9, "fp64", 32), (9, "fp32", 16), (20, "fp32", 64), (20, "fp64", 64),
    (64, "fp32", 16), (64, "fp32", 32), (64, "fp64", 64), (33, "fp32", 64),
])
def test_multi_column_sweep(monkeypatch, n_seeds, prec, lanes):
    # S = 8 .. 64 columns (padded), every lane layout of the dense sweep; each
    # column against the oracle's static scores of G + Delta G
    print(f"[multi-column] seeds={n_seeds} prec={prec} lanes={lanes}", flush=True)
    monkeypatch.setenv("RWR_PULL_LANES", str(lanes))
    from synth.rmat import sample_seeds

    g = rmat_graph(12, 40000, dead_end_self_loops=True)
    seeds = sample_seeds(g, n_seeds, seed=3)
    rng = np.random.default_rng(n_seeds)
    b = _batch(rng, g.n, g.src, g.dst, 200, 200, n_new=3)
    if prec == "fp64":
        kw = dict(eps=1e-13, err_budget=1e-11, build_tol=1e-12)
        gate = 1e-11
    else:
        kw = dict(eps=1e-8)
        gate = 2 * 1e-8 / 0.15
    with _ctx(g, seeds, precision=prec, **kw) as ctx:
        b1 = b
        n1, s1, d1 = oracle.apply_batch(g.n, g.src, g.dst, b1)
        b2 = _batch(rng, n1, s1, d1, 50, 50)
        n2, s2, d2 = oracle.apply_batch(n1, s1, d1, b2)
        ctx.update_batch(b1)
        ctx.update_batch(b2)
        for j, s in enumerate(seeds):
            ref = oracle.rwr_static(n2, s2, d2, int(s), 0.15)
            assert _l1(ctx.scores(j), ref) <= gate, (j, _l1(ctx.scores(j), ref))


@pytest.mark.parametrize("n_seeds,prec", [(9, "fp32"), (64, "fp32"), (20, "fp64")])
def test_multi_column_heavy_chunks(monkeypatch, n_seeds, prec):
    # many heavy in-rows cut into many short chunks (limit 16, chunk 32)
    print(f"[multi-column heavy] seeds={n_seeds} prec={prec}", flush=True)
    monkeypatch.setenv("RWR_HEAVY_LIMIT", "16")
    monkeypatch.setenv("RWR_HEAVY_CHUNK", "32")
    from synth.rmat import sample_seeds

    g = rmat_graph(11, 30000, dead_end_self_loops=True)
    seeds = sample_seeds(g, n_seeds, seed=3)
    rng = np.random.default_rng(1)
    b = _batch(rng, g.n, g.src, g.dst, 300, 300, n_new=2)
    kw = dict(eps=1e-13, err_budget=1e-11, build_tol=1e-12) if prec == "fp64" else dict(eps=1e-8)
    gate = 1e-11 if prec == "fp64" else 2 * 1e-8 / 0.15
    with _ctx(g, seeds, precision=prec, **kw) as ctx:
        for j, s in enumerate(seeds):
            ref = oracle.rwr_static(g.n, g.src, g.dst, int(s), 0.15)
            assert _l1(ctx.scores(j), ref) <= gate
        ctx.update_batch(b)
        n2, s2, d2 = oracle.apply_batch(g.n, g.src, g.dst, b)
        for j, s in enumerate(seeds):
            ref = oracle.rwr_static(n2, s2, d2, int(s), 0.15)
            assert _l1(ctx.scores(j), ref) <= gate, j


@pytest.mark.parametrize("n_seeds", [1, 16])
def test_sweep_shape_tuning(monkeypatch, n_seeds):
    # the build's static solve times candidate shapes and keeps one; the
    # scores do not depend on the shape
    print(f"[tuning] seeds={n_seeds}", flush=True)
    monkeypatch.delenv("RWR_PULL_LANES", raising=False)
    monkeypatch.delenv("RWR_GRID_PULL", raising=False)
    from synth.rmat import sample_seeds

    g = rmat_graph(13, 120000, dead_end_self_loops=True)
    seeds = sample_seeds(g, n_seeds, seed=3)
    kw = dict(eps=1e-12, precision="fp64", build_tol=1e-11)
    with _ctx(g, seeds, autotune=True, **kw) as tuned, _ctx(g, seeds, autotune=False, **kw) as fixed:
        sh = tuned.sweep_shape()
        assert sh["tuned_ms"] > 0.0 and sh["workgroups"] > 0
        assert fixed.sweep_shape()["tuned_ms"] == 0.0
        for j in (0, n_seeds - 1):
            ref = oracle.rwr_static(g.n, g.src, g.dst, int(seeds[j]), 0.15)
            assert _l1(tuned.scores(j), ref) < 1e-11
            assert _l1(fixed.scores(j), ref) < 1e-11


def test_tuning_cache(monkeypatch, tmp_path):
    # RWR_TUNE_CACHE: the first build tunes and appends its shape; a build of
    # the same workload takes it from the file without timing; another
    # workload (more columns) gets a line of its own
    print("[tuning cache]", flush=True)
    monkeypatch.delenv("RWR_PULL_LANES", raising=False)
    monkeypatch.delenv("RWR_GRID_PULL", raising=False)
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("RWR_TUNE_CACHE", str(path))
    from synth.rmat import sample_seeds

    g = rmat_graph(13, 120000, dead_end_self_loops=True)
    seeds = sample_seeds(g, 8, seed=3)
    kw = dict(eps=1e-12, precision="fp64", build_tol=1e-11)
    with _ctx(g, seeds, autotune=True, **kw) as a:
        sa = a.sweep_shape()
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].split()[1:3] == [str(sa["lanes_per_row"]), str(sa["workgroups"])]
    assert "/S8/" in lines[0] and f"/n{g.n}/" in lines[0]
    with _ctx(g, seeds, autotune=True, **kw) as b:
        sb = b.sweep_shape()
        assert (sb["lanes_per_row"], sb["workgroups"]) == (sa["lanes_per_row"], sa["workgroups"])
        assert abs(sb["tuned_ms"] - sa["tuned_ms"]) <= 1e-6 * max(1.0, sa["tuned_ms"])
        ref = oracle.rwr_static(g.n, g.src, g.dst, int(seeds[0]), 0.15)
        assert _l1(b.scores(0), ref) < 1e-11
    assert len(path.read_text().splitlines()) == 1
    with _ctx(g, sample_seeds(g, 16, seed=3), autotune=True, **kw):
        pass
    assert len(path.read_text().splitlines()) == 2


def test_graph_replay_matches_eager(monkeypatch):
    # dense iteration pairs replayed from a captured HIP graph give the same
    # propagation as eager launches, update after update (each update replays
    # the graph several times; eager work and synchronisations in between)
    print("[graph replay]", flush=True)
    g = rmat_graph(13, 120000, dead_end_self_loops=True)
    s = int(np.argmax(g.out_degree()))
    model = EdgeSetModel(g.n, g.src, g.dst)
    rng = np.random.default_rng(12)
    batches = [mixed_batch(rng, model, 20, 20) for _ in range(12)] + single_edge_stream(model, 12)
    kw = dict(eps=1e-12, precision="fp64", build_tol=1e-11, err_budget=1e-10)
    monkeypatch.setenv("RWR_GRAPHS", "0")
    eager = _ctx(g, [s], **kw)
    monkeypatch.setenv("RWR_GRAPHS", "1")
    graph = _ctx(g, [s], **kw)
    try:
        n, src, dst = g.n, g.src, g.dst
        dense = 0
        for b in batches:
            se = eager.update_batch(b)
            sg = graph.update_batch(b)
            dense += sg["dense_iters"]
            assert sg["iters"] == se["iters"], (sg["iters"], se["iters"])
            assert _l1(graph.scores(0), eager.scores(0)) < 1e-13
        assert dense >= 4  # dense pairs ran
        n, src, dst = oracle.apply_stream(g.n, g.src, g.dst, batches)
        assert _l1(graph.scores(0), oracle.rwr_static(n, src, dst, s, 0.15)) < 1e-10
    finally:
        eager.close()
        graph.close()


# ------------------------------------------- full-size workloads (sampled)

@pytest.mark.slow
def test_full_size_single_edge_stream():
    # the bench's workload at full size (R-MAT scale 20, one seed, FP32
    # propagation, eps = 1e-9, the launch shape the bench uses), 100 updates
    # of its stream, against the oracle's static solve of the final graph
    print("[full size scale 20]", flush=True)
    from synth.configs import RMAT20_SINGLE_EDGE, stream_for

    w = RMAT20_SINGLE_EDGE
    g = w.graph()
    seeds = w.seeds(g)
    stream = stream_for(w, w.model(g), 100)
    with _ctx(g, seeds, c=w.c, eps=1e-9, precision="fp32") as ctx:
        stats = [ctx.update_batch(b) for b in stream]
        assert max(s["err_bound"] for s in stats) <= 2e-9 / w.c
        n, s, d = oracle.apply_stream(g.n, g.src, g.dst, stream)
        ref = oracle.rwr_static(n, s, d, int(seeds[0]), w.c)
        got = ctx.scores(0)
        assert _l1(got, ref) <= 2e-9 / w.c
        # rank accuracy (the experiments' second metric): Spearman and top-k
        from paper_1712_00595_amd import accuracy

        acc = accuracy.compare(got, ref, ks=(10, 100, 1000))
        print(acc, flush=True)
        assert acc["spearman"] > 0.9999 and acc["top100_overlap"] >= 0.99, acc


@pytest.mark.slow
def test_full_size_64_columns_scale20():
    # 64 uniform seeds on the scale-20 graph with batches of the batched-seed
    # workload's kind; 4 sampled columns against the oracle
    print("[full size 64 columns]", flush=True)
    from synth.configs import RMAT20_SINGLE_EDGE
    from synth.rmat import sample_seeds
    from synth.stream import loguniform_batch_stream

    g = RMAT20_SINGLE_EDGE.graph()
    seeds = sample_seeds(g, 64, seed=3)
    stream = loguniform_batch_stream(EdgeSetModel(g.n, g.src, g.dst), 8, max_size=2000, seed=4)
    eps = 1e-6
    with _ctx(g, seeds, c=0.15, eps=eps, precision="fp32") as ctx:
        for b in stream:
            ctx.update_batch(b)
        n, s, d = oracle.apply_stream(g.n, g.src, g.dst, stream)
        for j in (0, 21, 42, 63):
            ref = oracle.rwr_static(n, s, d, int(seeds[j]), 0.15)
            assert _l1(ctx.scores(j), ref) <= 2 * eps / 0.15, j


def test_last_norms_are_the_update_run_after_a_refinement():
    # the norm history reported for an update is its own propagation's, also
    # when a residual refinement ran after it
    print("[last norms after refinement]", flush=True)
    g = rmat_graph(11, 20000, dead_end_self_loops=True)
    s = int(np.argmax(g.out_degree()))
    model = EdgeSetModel(g.n, g.src, g.dst)
    b = mixed_batch(np.random.default_rng(3), model, 20, 20)
    # a budget below one update's truncation bound: every update refines
    with _ctx(g, [s], eps=1e-9, precision="fp32", err_budget=2e-9) as ctx:
        st = ctx.update_batch(b)
        assert st["refined"] == 1
        norms = ctx.last_norms(0)
        assert norms.shape[0] == st["iters"] + 1
        assert norms[0] == pytest.approx(st["q_off_l1"], rel=1e-12)
        assert norms[-1] == pytest.approx(st["last_x_l1"], rel=1e-12)
        assert norms[-1] <= 1e-9 < norms[-2]
