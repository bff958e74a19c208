"""Deterministic mode and checkpoint/resume, through the C-ABI.

* Two contexts in deterministic mode fed the same stream give bitwise equal
  scores, statistics and (with the learned warm start training) parameters
  after every batch; the scores stay within Theorem 3's gate of the oracle.
* A context saved mid-stream (rwr_save) and loaded (rwr_load) continues the
  stream bitwise equal to the one that was not interrupted.
* Device memory from torch's caching allocator (the dev_alloc / dev_free
  hooks) gives the same bits as hipMalloc, and every block is returned.

The streams mix single edges, small and large batches (the large one takes
the radix-sort path), new nodes and a node deletion."""

import numpy as np
import pytest

import oracle
from synth import Batch, EdgeSetModel, rmat_graph
from synth.rmat import sample_seeds
from synth.stream import mixed_batch

pytestmark = pytest.mark.gpu

rwr = pytest.importorskip("paper_1712_00595_amd.rwr")

C = 0.15
E = np.zeros(0, np.int32)
STAT_KEYS = ("iters", "dense_iters", "refined", "checked", "visited_edges", "touched_rows", "q_off_l1",
             "last_x_l1", "err_bound", "residual_l1", "ws_region", "ws_accepted", "ws_resid_ratio", "ws_loss",
             "dr_l1", "carry_l1", "fallback", "flushed")


def _node_deletion(model, gone):
    """Batch deleting `gone` (every incident edge); the model follows."""
    keys = model.keys[: model.count]
    u, v = keys // int(model.KEY), keys % int(model.KEY)
    hit = np.isin(u, gone) | np.isin(v, gone)
    for a, b in zip(u[hit].tolist(), v[hit].tolist()):
        model.delete(a, b)
    return Batch(E, E, E, E, 0, del_nodes=np.array(gone, np.int32))


def _stream(g, es, ed, seeds, undirected, seed=6):
    model = EdgeSetModel(g.n, es, ed, undirected=undirected)
    rng = np.random.default_rng(seed)
    deg = np.bincount(np.concatenate([es, ed]), minlength=g.n)
    gone = [int(x) for x in np.argsort(-deg)[:8] if int(x) not in set(seeds.tolist())][:3]
    out = [mixed_batch(rng, model, 1, 0), mixed_batch(rng, model, 30, 30, n_new_nodes=5),
           _node_deletion(model, gone), mixed_batch(rng, model, 0, 1),
           mixed_batch(rng, model, 3000, 3000, n_new_nodes=40), mixed_batch(rng, model, 200, 100),
           mixed_batch(rng, model, 10, 10, n_new_nodes=2), mixed_batch(rng, model, 400, 400)]
    return out


def _apply_all(g, stream, undirected):
    n, s, d = g.n, g.src, g.dst
    for b in stream:
        n, s, d = oracle.apply_batch(n, s, d, b, undirected=undirected)
    return n, s, d


def _bits(x):
    return np.ascontiguousarray(np.asarray(x, np.float64)).view(np.uint64)


def _same_stats(a, b):
    for k in STAT_KEYS:
        assert _bits(a[k]) == _bits(b[k]), (k, a[k], b[k])


def _scores(ctx):
    return [ctx.scores(j) for j in range(ctx.n_seeds)]


def _graph(undirected):
    g = rmat_graph(12, 40000, dead_end_self_loops=not undirected, undirected=undirected)
    es, ed = (g.pair_u, g.pair_v) if undirected else (g.src, g.dst)
    return g, es, ed


@pytest.mark.parametrize("undirected,n_seeds,precision", [(False, 8, "fp32"), (True, 3, "fp64"),
                                                          (False, 1, "fp32")])
def test_two_runs_bitwise_equal(undirected, n_seeds, precision):
    print(f"[det] two runs undirected={undirected} seeds={n_seeds} {precision}", flush=True)
    g, es, ed = _graph(undirected)
    seeds = sample_seeds(g, n_seeds, seed=3)
    stream = _stream(g, es, ed, seeds, undirected)
    kw = dict(c=C, eps=1e-9, precision=precision, undirected=undirected, deterministic=True)
    with rwr.Context(g.n, es, ed, seeds, **kw) as a, rwr.Context(g.n, es, ed, seeds, **kw) as b:
        for i, bt in enumerate(stream):
            sa, sb = a.update_batch(bt), b.update_batch(bt)
            _same_stats(sa, sb)
            for j, (x, y) in enumerate(zip(_scores(a), _scores(b))):
                assert np.array_equal(_bits(x), _bits(y)), (i, j)
        gate = 2 * 1e-9 / C
        n2, s2, d2 = _apply_all(g, stream, undirected)
        for j, sd in enumerate(seeds):
            ref = oracle.rwr_static(n2, s2, d2, int(sd), C)
            assert float(np.abs(a.scores(j) - ref).sum()) <= gate, j


def test_deterministic_matches_default_mode_within_gate():
    print("[det] deterministic vs default mode", flush=True)
    g, es, ed = _graph(False)
    seeds = sample_seeds(g, 4, seed=3)
    stream = _stream(g, es, ed, seeds, False, seed=8)
    gate = 2 * 1e-9 / C
    with rwr.Context(g.n, es, ed, seeds, c=C, eps=1e-9, deterministic=True) as a, \
            rwr.Context(g.n, es, ed, seeds, c=C, eps=1e-9) as b:
        for bt in stream:
            sa, sb = a.update_batch(bt), b.update_batch(bt)
            # the offset seed is the same vector, summed in another order
            assert abs(sa["q_off_l1"] - sb["q_off_l1"]) <= 1e-12 * max(1.0, sb["q_off_l1"])
        for j in range(4):
            assert float(np.abs(a.scores(j) - b.scores(j)).sum()) <= 2 * gate


@pytest.mark.parametrize("undirected,n_seeds", [(False, 5), (True, 64), (False, 1)])
def test_sorted_offset_seed_matches_atomic_scatter(monkeypatch, undirected, n_seeds):
    """RWR_SEED_SORT=1 forms every batch's offset seed by sorting its terms
    and summing them per node (the deterministic mode's form, used by
    default for batches with many terms); RWR_SEED_SORT=0 scatters it with
    atomics.  Same seed vector up to rounding order, scores within Theorem
    3's gate of the oracle.  The 3000-edge batch gives hub nodes more terms
    than one reduction chunk holds."""
    print(f"[det] sorted vs scattered offset seed, undirected={undirected} seeds={n_seeds}", flush=True)
    g, es, ed = _graph(undirected)
    seeds = sample_seeds(g, n_seeds, seed=4)
    stream = _stream(g, es, ed, seeds, undirected, seed=14)
    kw = dict(c=C, eps=1e-9, undirected=undirected)
    gate = 2 * 1e-9 / C
    monkeypatch.setenv("RWR_SEED_SORT", "1")
    a = rwr.Context(g.n, es, ed, seeds, **kw)
    monkeypatch.setenv("RWR_SEED_SORT", "0")
    with a, rwr.Context(g.n, es, ed, seeds, **kw) as b:
        for bt in stream:
            sa, sb = a.update_batch(bt), b.update_batch(bt)
            assert abs(sa["q_off_l1"] - sb["q_off_l1"]) <= 1e-12 * max(1.0, sb["q_off_l1"])
            assert abs(sa["dr_l1"] - sb["dr_l1"]) <= 1e-12 * max(1.0, sb["dr_l1"])
            assert sa["touched_rows"] == sb["touched_rows"]
            assert sa["err_bound"] <= gate
        n2, s2, d2 = _apply_all(g, stream, undirected)
        for j, sd in enumerate(seeds[:8]):
            ref = oracle.rwr_static(n2, s2, d2, int(sd), C)
            assert float(np.abs(a.scores(j) - ref).sum()) <= gate, j
            assert float(np.abs(a.scores(j) - b.scores(j)).sum()) <= 2 * gate, j


def _warm_ctx(g, seeds, **kw):
    from paper_1712_00595_amd.warm import init_params, trainable_mask

    ctx = rwr.Context(g.n, g.src, g.dst, seeds, c=C, eps=1e-6, precision="fp32", deterministic=True, **kw)
    ctx.model_set(init_params(5, prior="copy"))
    ctx.model_trainable(trainable_mask(), warmup=3)
    ctx.warm_start("predict+train", hops=2, lr=3e-4)
    return ctx


def test_warm_start_training_bitwise_equal():
    print("[det] learned warm start, two runs", flush=True)
    g = rmat_graph(12, 40000, dead_end_self_loops=True)
    seeds = sample_seeds(g, 4, seed=3)
    model = EdgeSetModel(g.n, g.src, g.dst)
    rng = np.random.default_rng(9)
    stream = [mixed_batch(rng, model, 40, 40) for _ in range(8)]
    with _warm_ctx(g, seeds) as a, _warm_ctx(g, seeds) as b:
        for i, bt in enumerate(stream):
            sa, sb = a.update_batch(bt), b.update_batch(bt)
            assert sa["ws_region"] > 0
            _same_stats(sa, sb)
            for x, y in zip(_scores(a), _scores(b)):
                assert np.array_equal(_bits(x), _bits(y)), i
        assert np.array_equal(a.model_get().view(np.uint32), b.model_get().view(np.uint32))


@pytest.mark.parametrize("warm", [False, True])
def test_checkpoint_resume_bitwise_equal(tmp_path, warm):
    print(f"[det] checkpoint and resume warm={warm}", flush=True)
    g, es, ed = _graph(False)
    seeds = sample_seeds(g, 8, seed=3)
    if warm:
        model = EdgeSetModel(g.n, g.src, g.dst)
        rng = np.random.default_rng(10)
        stream = [mixed_batch(rng, model, 40, 40, n_new_nodes=3) for _ in range(8)]
        a = _warm_ctx(g, seeds)
    else:
        stream = _stream(g, es, ed, seeds, False, seed=11)
        a = rwr.Context(g.n, es, ed, seeds, c=C, eps=1e-9, deterministic=True)
    path = str(tmp_path / "ctx.ckpt")
    with a:
        for bt in stream[:4]:
            a.update_batch(bt)
        a.save(path)
        with rwr.Context.load(path) as b:
            assert b.n_seeds == 8 and np.array_equal(b.seeds, seeds) and b.n == a.n
            for x, y in zip(_scores(a), _scores(b)):
                assert np.array_equal(_bits(x), _bits(y))
            for i, bt in enumerate(stream[4:]):
                sa, sb = a.update_batch(bt), b.update_batch(bt)
                _same_stats(sa, sb)
                for j, (x, y) in enumerate(zip(_scores(a), _scores(b))):
                    assert np.array_equal(_bits(x), _bits(y)), (i, j)
            if warm:
                assert np.array_equal(a.model_get().view(np.uint32), b.model_get().view(np.uint32))
            ea, eb = a.export(), b.export()
            assert set(zip(ea[0].tolist(), ea[1].tolist())) == set(zip(eb[0].tolist(), eb[1].tolist()))


def test_checkpoint_default_mode_resumes_within_gate(tmp_path):
    print("[det] checkpoint, default mode", flush=True)
    g, es, ed = _graph(True)
    seeds = sample_seeds(g, 2, seed=3)
    stream = _stream(g, es, ed, seeds, True, seed=12)
    path = str(tmp_path / "u.ckpt")
    with rwr.Context(g.n, es, ed, seeds, c=C, eps=1e-9, undirected=True) as a:
        for bt in stream[:3]:
            a.update_batch(bt)
        a.save(path)
    with rwr.Context.load(path) as b:
        assert b.config()["undirected"] == 1
        for bt in stream[3:]:
            st = b.update_batch(bt)
            assert st["err_bound"] <= 2 * 1e-9 / C
        n2, s2, d2 = _apply_all(g, stream, True)
        for j, sd in enumerate(seeds):
            ref = oracle.rwr_static(n2, s2, d2, int(sd), C)
            assert float(np.abs(b.scores(j) - ref).sum()) <= 2 * 1e-9 / C


def test_torch_allocator_hooks():
    print("[det] torch caching allocator hooks", flush=True)
    g, es, ed = _graph(False)
    seeds = sample_seeds(g, 4, seed=3)
    stream = _stream(g, es, ed, seeds, False, seed=13)
    kw = dict(c=C, eps=1e-9, deterministic=True)
    a = rwr.Context(g.n, es, ed, seeds, allocator="torch", **kw)
    alloc = a.allocator
    assert alloc.live > 10
    with a, rwr.Context(g.n, es, ed, seeds, **kw) as b:
        for bt in stream:
            a.update_batch(bt)
            b.update_batch(bt)
        for x, y in zip(_scores(a), _scores(b)):
            assert np.array_equal(_bits(x), _bits(y))
        assert alloc.allocs > alloc.live > 10
    assert alloc.live == 0
