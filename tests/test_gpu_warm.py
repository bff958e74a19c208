"""Learned warm start inside rwr_update, on the GPU: the scores stay those of
Algorithm 1 whatever the network predicts (exactness through the residual),
the prediction is taken only where it shrinks the seed, and online training
on updates of the stream lowers the propagated seed norm and the iteration
count on held-out updates."""

import numpy as np
import pytest

import oracle
from oracle import gnn
from synth import EdgeSetModel, rmat_graph
from synth.rmat import sample_seeds
from synth.stream import mixed_batch

pytestmark = pytest.mark.gpu

rwr = pytest.importorskip("paper_1712_00595_amd.rwr")


def _copy_params():
    """A network whose output is its third input, q_offset / ||q||: the
    prediction is then the offset seed itself, so the residual is
    (1-c) B~^T q up to bfloat16 rounding and always smaller than q."""
    p = {k: np.zeros(gnn.SHAPES[k]) for k in gnn.ORDER}
    p["W0"][2, 0] = 1.0
    p["W0"][2, 1] = -1.0
    for l in range(1, gnn.LAYERS + 1):
        p[f"Ws{l}"][0, 0] = 1.0
        p[f"Ws{l}"][1, 1] = 1.0
    p["wo"][0] = 1.0
    p["wo"][1] = -1.0
    return gnn.pack(p).astype(np.float32)


def _l1(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).sum())


@pytest.mark.parametrize("n_seeds,undirected,push", [(1, False, None), (3, False, None), (2, True, None),
                                                     (3, False, "1"), (2, True, "1")])
def test_prediction_path_is_exact(n_seeds, undirected, push, monkeypatch):
    """push "1": the residual formed from the region alone (RWR_WS_PUSH=1),
    None: the library's choice (a pull over every in-row at these sizes)."""
    print(f"[warm exact] seeds={n_seeds} undirected={undirected} push={push}", flush=True)
    if push is not None:
        monkeypatch.setenv("RWR_WS_PUSH", push)
    g = rmat_graph(11, 20000, dead_end_self_loops=not undirected, undirected=undirected)
    seeds = sample_seeds(g, n_seeds, seed=3)
    es, ed = (g.pair_u, g.pair_v) if undirected else (g.src, g.dst)
    model = EdgeSetModel(g.n, es, ed, undirected=undirected)
    rng = np.random.default_rng(8)
    batches = [mixed_batch(rng, model, 40, 40, n_new_nodes=1) for _ in range(3)]
    kw = dict(c=0.15, eps=1e-14, precision="fp64", build_tol=1e-13, err_budget=1e-12, undirected=undirected)
    with rwr.Context(g.n, es, ed, seeds, **kw) as plain, rwr.Context(g.n, es, ed, seeds, **kw) as warm:
        warm.model_set(_copy_params())
        warm.warm_start("predict", hops=2)
        n, s, d = g.n, g.src, g.dst
        for b in batches:
            sp = plain.update_batch(b)
            sw = warm.update_batch(b)
            n, s, d = oracle.apply_batch(n, s, d, b, undirected=undirected)
            assert sw["ws_region"] > 0
            assert sw["ws_accepted"] == n_seeds, sw
            assert sw["ws_resid_ratio"] < 0.9, sw
            assert sw["iters"] <= sp["iters"], (sw["iters"], sp["iters"])
            for j, sd in enumerate(seeds):
                ref = oracle.rwr_static(n, s, d, int(sd), 0.15)
                assert _l1(warm.scores(j), ref) < 1e-12, (j, _l1(warm.scores(j), ref))


def test_bad_prediction_falls_back():
    # a network that predicts minus the seed makes the residual larger than
    # the seed: every column keeps the plain seed, scores still exact
    print("[warm fallback]", flush=True)
    g = rmat_graph(10, 8000, dead_end_self_loops=True)
    seeds = sample_seeds(g, 2, seed=3)
    th = _copy_params()
    p = gnn.unpack(th.astype(np.float64))
    p["wo"][0], p["wo"][1] = -3.0, 3.0
    th = gnn.pack(p).astype(np.float32)
    model = EdgeSetModel(g.n, g.src, g.dst)
    b = mixed_batch(np.random.default_rng(2), model, 30, 30)
    with rwr.Context(g.n, g.src, g.dst, seeds, eps=1e-14, precision="fp64", build_tol=1e-13,
                     err_budget=1e-12) as ctx:
        ctx.model_set(th)
        ctx.warm_start("predict")
        st = ctx.update_batch(b)
        assert st["ws_accepted"] == 0 and st["ws_resid_ratio"] > 1.0
        n, s, d = oracle.apply_batch(g.n, g.src, g.dst, b)
        for j, sd in enumerate(seeds):
            assert _l1(ctx.scores(j), oracle.rwr_static(n, s, d, int(sd), 0.15)) < 1e-12


def test_settings_are_checked():
    g = rmat_graph(8, 1000, dead_end_self_loops=True)
    with rwr.Context(g.n, g.src, g.dst, [0]) as ctx:
        with pytest.raises(rwr.RwrError) as e:
            ctx.warm_start("predict")
        assert e.value.code == -8  # no parameters yet
        ctx.model_set(gnn.init_params(5))
        with pytest.raises(rwr.RwrError):
            ctx.warm_start("predict", hops=99)
        ctx.warm_start("train")
        th = ctx.model_get()
        assert np.array_equal(th, gnn.init_params(5).astype(np.float32))


def test_training_keeps_exactness_and_the_trained_network_gains():
    # online training (residual loss, AdamW on the trainable parameters of the
    # homogeneous network, step-size warm-up) on 600 updates of a stream,
    # starting from the copy prior (the network predicts q itself); then 30
    # held-out updates run plainly, with the untrained copy prior and with
    # the trained network: the scores stay within the OSP-T gate, and the
    # trained network leaves a residual less than half the copy prior's and
    # takes fewer iterations than both the copy prior and plain OSP-T.  The
    # analytic propagation prior (four terms of the offset series) is printed
    # beside it: training from the copy prior comes close to it.
    print("[warm train]", flush=True)
    from paper_1712_00595_amd.warm import init_params, trainable_mask

    g = rmat_graph(12, 40000, dead_end_self_loops=True)
    seeds = sample_seeds(g, 4, seed=3)
    model = EdgeSetModel(g.n, g.src, g.dst)
    rng = np.random.default_rng(4)
    train = [mixed_batch(rng, model, 50, 50) for _ in range(600)]
    held = [mixed_batch(rng, model, 50, 50) for _ in range(30)]
    eps = 1e-9
    kw = dict(eps=eps, precision="fp32")
    th0 = init_params(5, prior="copy")
    with rwr.Context(g.n, g.src, g.dst, seeds, **kw) as trainer:
        trainer.model_set(th0)
        trainer.model_trainable(trainable_mask(), warmup=30)
        trainer.warm_start("predict+train", hops=3, lr=3e-4)
        losses = [trainer.update_batch(b)["ws_loss"] for b in train]
        th = trainer.model_get()
    assert np.all(np.isfinite(losses)) and not np.array_equal(th, th0)
    # parameters outside the mask did not move
    assert np.array_equal(th[trainable_mask() == 0], th0[trainable_mask() == 0])
    assert np.mean(losses[-50:]) < 0.5 * np.mean(losses[:20])
    res = {}
    for name, params in (("plain", None), ("copy prior", th0), ("trained", th),
                         ("propagation prior", init_params(5, prior="propagation"))):
        with rwr.Context(g.n, g.src, g.dst, seeds, **kw) as ctx:
            for b in train:
                ctx.update_batch(b)
            if params is not None:
                ctx.model_set(params)
                ctx.warm_start("predict", hops=3)
            it, ratio = [], []
            for b in held:
                st = ctx.update_batch(b)
                it.append(st["iters"])
                ratio.append(st["ws_resid_ratio"])
            res[name] = (float(np.mean(it)), float(np.mean(ratio)))
            if name == "trained":
                n, s, d = g.n, g.src, g.dst
                for b in train + held:
                    n, s, d = oracle.apply_batch(n, s, d, b)
                for j, sd in enumerate(seeds):
                    ref = oracle.rwr_static(n, s, d, int(sd), 0.15)
                    assert _l1(ctx.scores(j), ref) <= 2 * eps / 0.15
    print("held-out (mean iterations, residual ratio): " + str(res), flush=True)
    it_plain, _ = res["plain"]
    it_copy, r_copy = res["copy prior"]
    it_tr, r_tr = res["trained"]
    assert r_tr < 0.5 * r_copy, res
    assert it_tr < it_copy and it_tr < it_plain, res
