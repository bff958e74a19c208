"""GPU parity at the shapes of the larger workloads, against the CPU oracle's
static solve of the final graph:

* the undirected churn workload (symmetrised R-MAT, c = 0.05, FP32
  propagation, eps = 1e-9, 16 seeds; batches deleting 1% of the pairs and
  inserting as many plus new nodes) at scale 15, every seed column within
  the gate 2 eps / c = 4e-8;
* the batched-seed workload at its full size (R-MAT scale 22, 64 seeds,
  eps = 1e-6, batches of log-uniform size up to 10^4 with 1% new nodes), on
  sampled columns;
* the learned warm start at scale 16 (16 seeds, eps = 1e-6, 100-edge
  batches, prediction and training on), every column within the gate."""

import time

import numpy as np
import pytest

import oracle
from synth import EdgeSetModel, rmat_graph
from synth.churn import PairPool
from synth.rmat import sample_seeds
from synth.stream import loguniform_batch_stream, mixed_batch

pytestmark = pytest.mark.gpu

rwr = pytest.importorskip("paper_1712_00595_amd.rwr")


def _l1(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).sum())


def _oracle_columns(n, src, dst, seeds, c, tol=1e-14, threads=8):
    """The oracle's static solve of every seed, in parallel threads (its C
    solver releases the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(lambda sd: oracle.rwr_static(n, src, dst, int(sd), c, tol=tol), seeds))


def _pairs_to_edges(pool):
    lo = np.minimum(pool.keys // (1 << 32), pool.keys % (1 << 32))
    hi = np.maximum(pool.keys // (1 << 32), pool.keys % (1 << 32))
    loop = lo == hi
    s = np.concatenate([lo, hi[~loop]]).astype(np.int32)
    d = np.concatenate([hi, lo[~loop]]).astype(np.int32)
    return s, d


def test_undirected_churn_shape_scale15():
    print("[configs] undirected churn, scale 15, c=0.05, eps=1e-9, 16 seeds", flush=True)
    c, eps = 0.05, 1e-9
    gate = 2 * eps / c
    g = rmat_graph(15, 16 * (1 << 15), undirected=True)
    seeds = sample_seeds(g, 16, seed=3)
    pool = PairPool(g.n, g.pair_u, g.pair_v)
    rng = np.random.Generator(np.random.PCG64(4))
    batches = [pool.churn_batch(rng, int(round(0.01 * pool.count)), 40) for _ in range(3)]
    with rwr.Context(g.n, g.pair_u, g.pair_v, seeds, c=c, eps=eps, precision="fp32", undirected=True) as ctx:
        for b in batches:
            st = ctx.update_batch(b)
            assert st["err_bound"] <= gate, st
        s2, d2 = _pairs_to_edges(pool)
        t = time.time()
        worst = 0.0
        refs = _oracle_columns(pool.n, s2, d2, seeds, c)
        for j, ref in enumerate(refs):
            err = _l1(ctx.scores(j), ref)
            worst = max(worst, err)
            assert err <= gate, (j, err)
        print(f"max L1 {worst:.3e} vs gate {gate:.1e} ({time.time() - t:.1f}s oracle)", flush=True)


def test_batched_seeds_full_size_sampled_columns():
    print("[configs] R-MAT scale 22, 64 seeds, eps=1e-6, 12 log-uniform batches", flush=True)
    from synth.configs import RMAT22_BATCHED as w

    t = time.time()
    g = w.graph()
    seeds = w.seeds(g)
    stream = loguniform_batch_stream(w.model(g), 12, seed=4)
    print(f"graph and stream in {time.time() - t:.1f}s; batch sizes {[b.size for b in stream]}", flush=True)
    eps = w.eps[0]
    gate = 2 * eps / w.c
    cols = [0, 21, 63]
    with rwr.Context(g.n, g.src, g.dst, seeds, c=w.c, eps=eps, precision="fp32") as ctx:
        for b in stream:
            st = ctx.update_batch(b)
            assert st["err_bound"] <= gate, st
        got = {j: ctx.scores(j) for j in cols}
    t = time.time()
    n2, s2, d2 = oracle.apply_stream(g.n, g.src, g.dst, stream)
    # the oracle's columns in parallel threads (its C solver releases the
    # interpreter lock); tolerance 1e-11, a truncation of at most 6e-11 in
    # L1, far below the gate
    refs = _oracle_columns(n2, s2, d2, [seeds[j] for j in cols], w.c, tol=1e-11, threads=len(cols))
    for j, ref in zip(cols, refs):
        err = _l1(got[j], ref)
        print(f"column {j}: L1 {err:.3e} vs gate {gate:.2e}", flush=True)
        assert err <= gate, (j, err)
    print(f"oracle {time.time() - t:.1f}s", flush=True)


def test_learned_warm_start_shape_scale16():
    print("[configs] learned warm start, scale 16, 16 seeds, eps=1e-6", flush=True)
    from paper_1712_00595_amd.warm import init_params, trainable_mask

    c, eps = 0.15, 1e-6
    gate = 2 * eps / c
    g = rmat_graph(16, 16 * (1 << 16), dead_end_self_loops=True)
    seeds = sample_seeds(g, 16, seed=3)
    model = EdgeSetModel(g.n, g.src, g.dst)
    rng = np.random.default_rng(4)
    batches = [mixed_batch(rng, model, 50, 50) for _ in range(40)]
    with rwr.Context(g.n, g.src, g.dst, seeds, c=c, eps=eps, precision="fp32") as ctx:
        ctx.model_set(init_params(5, prior="copy"))
        ctx.model_trainable(trainable_mask(), warmup=10)
        ctx.warm_start("predict+train", hops=3, lr=3e-4)
        acc = 0
        for b in batches:
            st = ctx.update_batch(b)
            acc += st["ws_accepted"]
            assert st["err_bound"] <= gate, st
        assert acc > 0
        n2, s2, d2 = oracle.apply_stream(g.n, g.src, g.dst, batches)
        for j, ref in enumerate(_oracle_columns(n2, s2, d2, seeds, c)):
            err = _l1(ctx.scores(j), ref)
            assert err <= gate, (j, err)
