"""GPU: the failure paths and the extra fields of the C ABI -- an update that
reaches max_iters (RWR_ENOCONV, stale context, rwr_refine recovers it), a
non-finite score written through rwr_scores_set (RWR_ENUMERIC, recovery by
setting valid scores and refining), the literal node-deletion reading
(node_deletion = 1, the row only) against the oracle, and the per-phase
timings and counters of rwr_stats."""

import numpy as np
import pytest

import oracle
from synth import EdgeSetModel, rmat_graph
from synth.rmat import sample_seeds
from synth.stream import Batch, mixed_batch

pytestmark = pytest.mark.gpu

rwr = pytest.importorskip("paper_1712_00595_amd.rwr")

C = 0.15
E = np.zeros(0, np.int32)


def _l1(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).sum())


def test_max_iters_stale_and_refine():
    print("[boundary] ENOCONV", flush=True)
    g = rmat_graph(10, 8000, dead_end_self_loops=True)
    s = int(np.argmax(g.out_degree()))
    model = EdgeSetModel(g.n, g.src, g.dst)
    rng = np.random.default_rng(3)
    b = mixed_batch(rng, model, 20, 20)
    b2 = mixed_batch(rng, model, 5, 5)
    eps = 1e-9
    with rwr.Context(g.n, g.src, g.dst, [s], c=C, eps=eps, precision="fp64", max_iters=1) as ctx:
        with pytest.raises(rwr.RwrError) as e:
            ctx.update_batch(b)
        assert e.value.code == -6  # RWR_ENOCONV: the graph is updated, the scores hold the partial sum
        with pytest.raises(rwr.RwrError) as e:
            ctx.update_batch(b2)
        assert e.value.code == -8  # RWR_ESTATE until refined
        st = ctx.refine()
        assert st["err_bound"] <= 2 * eps / C / 8 * (1 + 1e-9)
        n2, s2, d2 = oracle.apply_batch(g.n, g.src, g.dst, b)
        ref = oracle.rwr_static(n2, s2, d2, s, C)
        assert _l1(ctx.scores(0), ref) <= st["err_bound"] + 1e-13
        assert ctx.n == n2


def test_non_finite_scores_and_recovery():
    print("[boundary] ENUMERIC", flush=True)
    g = rmat_graph(10, 8000, dead_end_self_loops=True)
    s = int(np.argmax(g.out_degree()))
    eps = 1e-10
    with rwr.Context(g.n, g.src, g.dst, [s], c=C, eps=eps, precision="fp64") as ctx:
        sc = ctx.scores(0)
        u = int(np.argmax(sc))  # the seed: a touched row with a non-zero score
        bad = sc.copy()
        bad[u] = np.nan
        ctx.scores_set(0, bad)
        w = next(v for v in range(g.n) if v != u and not EdgeSetModel(g.n, g.src, g.dst).has(u, v))
        b = Batch(np.array([u], np.int32), np.array([w], np.int32), E, E, 0)
        with pytest.raises(rwr.RwrError) as e:
            ctx.update_batch(b)
        assert e.value.code == -7  # RWR_ENUMERIC
        with pytest.raises(rwr.RwrError) as e:
            ctx.update_batch(Batch(E, E, E, E, 0))
        assert e.value.code == -8
        # valid scores for the updated graph, then a refinement
        n2, s2, d2 = oracle.apply_batch(g.n, g.src, g.dst, b)
        ref = oracle.rwr_static(n2, s2, d2, s, C)
        ctx.scores_set(0, ref + 1e-7 / ref.shape[0])
        st = ctx.refine()
        assert np.all(np.isfinite(ctx.scores(0)))
        assert _l1(ctx.scores(0), ref) <= st["err_bound"] + 1e-13
        assert st["err_bound"] <= 2 * eps / C


@pytest.mark.parametrize("mode", ["row", "incident"])
def test_node_deletion_readings(mode):
    print(f"[boundary] node deletion {mode}", flush=True)
    g = rmat_graph(10, 8000, dead_end_self_loops=True)
    seeds = sample_seeds(g, 2, seed=3)
    deg_in = np.bincount(g.dst, minlength=g.n)
    gone = [int(v) for v in np.argsort(-deg_in)[:6] if int(v) not in seeds][:3]
    b = Batch(E, E, E, E, 0, del_nodes=np.array(gone, np.int32))
    with rwr.Context(g.n, g.src, g.dst, seeds, c=C, eps=1e-14, precision="fp64", build_tol=1e-13,
                     err_budget=1e-12, node_deletion=mode) as ctx:
        ctx.update_batch(b)
        n2, s2, d2 = oracle.apply_batch(g.n, g.src, g.dst, b, rows_only=(mode == "row"))
        es, ed, _ = ctx.export()
        assert set(zip(es.tolist(), ed.tolist())) == set(zip(s2.tolist(), d2.tolist()))
        assert (np.isin(ed, gone).any()) == (mode == "row")
        for j, sd in enumerate(seeds):
            ref = oracle.rwr_static(n2, s2, d2, int(sd), C)
            assert _l1(ctx.scores(j), ref) < 1e-12


def test_phase_timings_and_counters():
    print("[boundary] phase timing, flushed, fallback", flush=True)
    from oracle import gnn

    g = rmat_graph(11, 20000, dead_end_self_loops=True)
    seeds = sample_seeds(g, 3, seed=3)
    model = EdgeSetModel(g.n, g.src, g.dst)
    rng = np.random.default_rng(5)
    with rwr.Context(g.n, g.src, g.dst, seeds, c=C, eps=1e-9, precision="fp32", phase_timing=True) as ctx:
        flushed = 0
        for _ in range(6):
            st = ctx.update_batch(mixed_batch(rng, model, 30, 30))
            parts = [st[k] for k in ("ms_delta", "ms_seed", "ms_model", "ms_prop", "ms_merge")]
            assert st["ms_delta"] > 0 and st["ms_seed"] > 0 and st["ms_prop"] > 0, st
            assert min(parts) >= 0 and sum(parts) <= st["ms_total"] * 1.05 + 0.05, st
            assert (st["flushed"] > 0) == bool(st["refined"]) and st["flushed"] <= 3, st
            flushed += st["flushed"]
        assert st["fallback"] == 0
        # a network that predicts minus the seed: every column falls back
        p = {k: np.zeros(gnn.SHAPES[k]) for k in gnn.ORDER}
        p["W0"][2, 0], p["W0"][2, 1] = 1.0, -1.0
        for layer in range(1, gnn.LAYERS + 1):
            p[f"Ws{layer}"][0, 0] = p[f"Ws{layer}"][1, 1] = 1.0
        p["wo"][0], p["wo"][1] = -3.0, 3.0
        ctx.model_set(gnn.pack(p).astype(np.float32))
        ctx.warm_start("predict")
        st = ctx.update_batch(mixed_batch(rng, model, 30, 30))
        assert st["ws_accepted"] == 0 and st["fallback"] == 3, st
        assert st["ms_model"] > 0
    model = EdgeSetModel(g.n, g.src, g.dst)  # each context below starts from the original graph
    with rwr.Context(g.n, g.src, g.dst, seeds, c=C, eps=1e-9, precision="fp32") as ctx:
        st = ctx.update_batch(mixed_batch(rng, model, 30, 30))
        assert st["ms_prop"] == 0.0  # timing off
    # a refinement flushes the columns above the budget
    model = EdgeSetModel(g.n, g.src, g.dst)
    with rwr.Context(g.n, g.src, g.dst, seeds, c=C, eps=1e-6, precision="fp32", err_budget=2e-6) as ctx:
        total = 0
        for _ in range(8):
            st = ctx.update_batch(mixed_batch(rng, model, 30, 30))
            if st["refined"]:
                assert 1 <= st["flushed"] <= 3
            total += st["flushed"]
        assert total > 0
