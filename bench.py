#!/usr/bin/env python3
"""Dynamic RWR update throughput on one MI355X.

Headline workload (the largest single-GPU configuration by bytes per sweep):
directed R-MAT scale 22 (4,194,304 nodes, 67,108,864 edges + a self-loop on
every dead end), restart c = 0.15, 64 seed nodes sampled uniformly, eps = 1e-6
(error gate 2*eps/c), a stream of batches of log-uniform size in [1, 10^4]
edge modifications with 1% new nodes carrying 1-8 out-edges.  A step is one
batch: delta-apply, offset seed for all 64 columns, propagation of the N x 64
block until every column has ||x||_1 <= eps, merge and the stream error
check -- the whole hot path.  Propagation runs in FP32, scores accumulate in
FP64.  ``value`` counts edge and node modifications per second with every
column kept within the gate; ``--steps`` counts batches.

The single-seed scale-20 stream of single-edge updates (eps = 1e-9) is
reported under ``modes`` (its working set fits the Infinity Cache: a latency
figure, not an HBM one).

Printed: one JSON line on stdout; progress on stderr.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def dense_sweep_bytes(n: int, m: int, S: int = 1) -> int:
    """Algorithmic bytes of one dense sweep: row offsets 4(n+1), column
    indices 4m, out-degrees 4n, read of x 4nS, write of the next x 4nS, FP64
    score read + write 16nS."""
    return 4 * (n + 1) + 4 * m + 4 * n + 4 * n * S + 4 * n * S + 16 * n * S


def rank_accuracy(accuracy, got, ref) -> dict:
    """Spearman's rank correlation and top-k overlaps of the scores against
    the oracle's (the L1 distance is reported beside them)."""
    out = accuracy.compare(got, ref, ks=(10, 100, 1000))
    out.pop("l1")
    return out


def cpu_count_used() -> int:
    return 1


TRAFFIC_C2 = os.path.join(ROOT, "profiles", "k_pull_wv_rmat20_traffic.md")
TRAFFIC_C3 = os.path.join(ROOT, "profiles", "k_pull_v_rmat22_s64_traffic.md")
SWEEP_SOURCE = os.path.join(ROOT, "paper_1712_00595_amd", "csrc", "k_prop.hip")


def host_cpu_model() -> str:
    """The host CPU's model name as lscpu prints it, with its family, model
    and stepping numbers (a virtualised host may report a short name)."""
    fields = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                k, v = line.split(":", 1)
                fields.setdefault(k.strip(), v.strip())
            if not line.strip() and fields:
                break
    except OSError:
        pass
    name = fields.get("model name") or platform.processor() or platform.machine()
    ids = [f"{k} {fields[k]}" for k in ("cpu family", "model", "stepping") if k in fields]
    return f"{name} ({', '.join(ids)})" if ids else name


def measured_traffic(sweep_bytes: int, summary: str = TRAFFIC_C2):
    """HBM bytes of one sweep from the committed counter summary, or None
    when the sweep kernel's source has changed since the counters were taken
    (its sha256 is recorded in the summary) or the workload differs."""
    import hashlib

    try:
        text = open(summary).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            fields[k.strip("` ")] = v.strip("` ")
    try:
        src_hash = hashlib.sha256(open(SWEEP_SOURCE, "rb").read()).hexdigest()
        if fields.get("kernel_source_sha256") != src_hash:
            return None
        rec = int(fields["algorithmic_bytes_per_sweep"])
        # the same workload up to the few edges a different stream length moves
        if abs(rec - sweep_bytes) > 1e-3 * sweep_bytes:
            return None
        return float(fields["hbm_bytes_per_sweep"]) * sweep_bytes / rec
    except (KeyError, ValueError, OSError):
        return None


def stage_batches(batches):
    """The batches' arrays copied to HBM before the clock starts: one device
    array per field, each batch a view into them."""
    import torch

    cat = {}
    for f in ("ins_src", "ins_dst", "del_src", "del_dst"):
        parts = [getattr(b, f) for b in batches]
        cat[f] = torch.as_tensor(np.concatenate(parts).astype(np.int32), device="cuda")
    oi = np.concatenate([[0], np.cumsum([b.n_ins for b in batches])])
    od = np.concatenate([[0], np.cumsum([b.n_del for b in batches])])
    return [(cat["ins_src"][oi[i]:oi[i + 1]], cat["ins_dst"][oi[i]:oi[i + 1]],
             cat["del_src"][od[i]:od[i + 1]], cat["del_dst"][od[i]:od[i + 1]], b.n_new_nodes)
            for i, b in enumerate(batches)]


def run_batched_seeds(K: int, W: int, check: bool = True, cpu_baseline: bool = True) -> dict:
    """The headline: R-MAT scale 22, 64 uniform seeds, batches of log-uniform
    size in [1, 10^4] edge modifications with 1% new nodes, eps = 1e-6; the
    dense sweep here is the vectorised multi-column kernel.  W warm-up
    batches, then K timed batches staged in HBM.  The timed pass runs the
    library's default path (no per-launch events, HIP-graph replay on); a
    second pass over the same batches on a fresh context times every launch
    of the dense sweep with HIP events for the roofline."""
    import torch

    from paper_1712_00595_amd import rwr
    from synth.configs import RMAT22_BATCHED, stream_for

    w = RMAT22_BATCHED
    S = w.n_seeds
    t = time.time()
    g = w.graph()
    seeds = w.seeds(g)
    stream = stream_for(w, w.model(g), W + K)
    log(f"[{w.name}] graph n={g.n} m={g.m}, {W} warm-up + {K} timed batches ({time.time() - t:.1f}s)")
    eps = w.eps[0]
    dev = stage_batches(stream[W:])
    mods = sum(b.size for b in stream[W:])

    def one_pass(profile: bool):
        t = time.time()
        ctx = rwr.Context(g.n, g.src, g.dst, seeds, c=w.c, eps=eps, precision="fp32")
        torch.cuda.synchronize()
        build_s = time.time() - t
        for b in stream[:W]:
            ctx.update_batch(b)
        ctx.profile(profile)
        ctx.profile_read(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = [ctx.update(*u[:4], n_new_nodes=u[4]) for u in dev]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        return ctx, stats, el, ctx.profile_read(reset=True), build_s

    ctx, stats, el, _, build_s = one_pass(False)
    lat = np.array([s["ms_total"] for s in stats])
    res = {
        "batches": K,
        "warmup_batches": W,
        "edge_and_node_modifications": mods,
        "modifications_per_s": mods / el,
        "batches_per_s": K / el,
        "ms_per_batch": 1e3 * el / K,
        "seed_columns_x_batches_per_s": S * K / el,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "build_s": build_s,
        "mean_iters": float(np.mean([s["iters"] for s in stats])),
        "mean_dense_sweeps": float(np.mean([s["dense_iters"] for s in stats])),
        "residual_checks": int(sum(s["checked"] for s in stats)),
        "refinements": int(sum(s["refined"] for s in stats)),
        "max_err_bound": float(max(s["err_bound"] for s in stats)),
        "gate": 2 * eps / w.c,
        "sweep_shape": ctx.sweep_shape(),
    }
    log(f"[{w.name}] {res['batches_per_s']:.2f} batches/s, {res['modifications_per_s']:.0f} modifications/s, "
        f"iters {res['mean_iters']:.2f} (dense {res['mean_dense_sweeps']:.2f}), checks {res['residual_checks']}, "
        f"refinements {res['refinements']}, bound {res['max_err_bound']:.2e}")
    final_scores = {}
    cols = [0, S - 1]
    if check:
        for j in cols:
            final_scores[j] = ctx.scores(j)
    n_f, m_f = ctx.n, ctx.m
    ctx.close()

    # the roofline pass: the same batches, every sweep launch timed with
    # HIP events on the library's stream
    ctx, stats_p, el_p, P, _ = one_pass(True)
    shape = ctx.sweep_shape()
    ctx.close()
    res["profiled_pass_batches_per_s"] = K / el_p
    launches = P["dense_sweeps"] + P["idle_launches"]
    if P["dense_sweeps"]:
        sweep_bytes = dense_sweep_bytes(n_f, m_f, S)
        avg_us = 1e3 * P["dense_ms"] / launches
        bytes_per_launch = sweep_bytes * P["dense_sweeps"] / launches
        achieved = bytes_per_launch / (avg_us * 1e-6) / 1e9
        traffic = measured_traffic(sweep_bytes, TRAFFIC_C3)
        res["roofline"] = {
            "bound": "hbm",
            "kernel": f"k_pull_v<float, {S}, {shape['lanes_per_row']}, KIND_DENSE> (dense sweep, {S} columns)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None if traffic is None else traffic * P["dense_sweeps"] / launches,
            "bytes_per_sweep": sweep_bytes,
            "bytes_per_launch": bytes_per_launch,
            "avg_launch_us": avg_us,
            "avg_sweep_us": 1e3 * P["dense_ms"] / P["dense_sweeps"],
            "launches": launches,
            "idle_launches": P["idle_launches"],
        }
        log(f"[{w.name}] sweep {res['roofline']['avg_sweep_us']:.1f} us, {achieved:.0f} GB/s algorithmic "
            f"= {achieved / HBM_PEAK_GBS:.3f} of peak")

    if check or cpu_baseline:
        import oracle

        from paper_1712_00595_amd import accuracy
    if check:
        # sampled parity: the first and last columns against the oracle's
        # static solve of the final graph
        t = time.time()
        n2, s2, d2 = oracle.apply_stream(g.n, g.src, g.dst, stream)
        errs, ranks = [], []
        for j in cols:
            ref = oracle.rwr_static(n2, s2, d2, int(seeds[j]), w.c)
            got = final_scores[j]
            errs.append(float(np.abs(got - ref).sum()))
            ranks.append(rank_accuracy(accuracy, got, ref))
        res["parity"] = {"columns": cols, "l1_vs_oracle": errs, "gate": res["gate"], "rank_accuracy": ranks,
                         "ok": max(errs) <= res["gate"], "oracle_s": time.time() - t}
        log(f"[{w.name}] parity: max L1 {max(errs):.3e} vs gate {res['gate']:.3e} ({time.time() - t:.1f}s)")
    if cpu_baseline:
        # the oracle's Algorithm 1 (one seed column, single-threaded FP64,
        # full edge sweeps) on the first batch of the stream from the oracle's
        # static scores; scaled to all 64 columns
        t = time.time()
        r_old = oracle.rwr_static(g.n, g.src, g.dst, int(seeds[0]), w.c)
        static_s = time.time() - t
        b0 = stream[0]
        t = time.time()
        n1, s1, d1 = oracle.apply_batch(g.n, g.src, g.dst, b0)
        oracle.osp((g.n, g.src, g.dst), (n1, s1, d1), r_old, w.c, eps, renorm=1)
        col_s = time.time() - t
        res["cpu_baseline"] = {
            "value": b0.size / (S * col_s),
            "unit": "updates/s",
            "cores": cpu_count_used(),
            "kind": "oracle",
            "sample": f"Algorithm 1 (oracle/rwr_oracle.c, single-threaded FP64, full edge sweeps) for seed column 0 "
                      f"on the first batch of the stream ({b0.size} modifications) from the oracle's static scores, "
                      f"{col_s:.1f}s; rate scaled to all {S} columns; static solve of the initial graph took "
                      f"{static_s:.1f}s",
            "static_solve_s": static_s,
            "host_cpu": host_cpu_model(),
            "host_threads": os.cpu_count(),
        }
        log(f"[{w.name}] cpu baseline: {res['cpu_baseline']['value']:.3f} updates/s ({col_s:.1f}s for one column)")
    return res


def run_learned(n_train: int, n_eval: int, check: bool = True, max_rows: int = 0) -> dict:
    """R-MAT scale 21, 16 uniform seeds, 100-edge batches (50/50), eps = 1e-6:
    online training of the warm-start network on n_train updates (from the
    copy prior, the positively homogeneous parameters only, step-size
    warm-up), a checkpoint of the trained context, then the same n_eval
    held-out updates timed from that checkpoint with the plain method, the
    trained network, and the untrained copy and propagation priors."""
    import tempfile

    import torch

    from paper_1712_00595_amd import rwr
    from paper_1712_00595_amd.warm import init_params, trainable_mask
    from synth.configs import RMAT21_LEARNED, stream_for

    w = RMAT21_LEARNED
    t = time.time()
    g = w.graph()
    seeds = w.seeds(g)
    stream = stream_for(w, w.model(g), n_train + n_eval)
    train, held = stream[:n_train], stream[n_train:]
    log(f"[{w.name}] graph n={g.n} m={g.m}, {n_train} train + {n_eval} held-out batches ({time.time() - t:.1f}s)")
    eps = w.eps[0]
    kw = dict(c=w.c, eps=eps, precision="fp32")
    th_copy = init_params(5, prior="copy")
    th_prop = init_params(5, prior="propagation", c=w.c)
    res = {"train_updates": n_train, "eval_updates": n_eval, "gate": 2 * eps / w.c, "max_rows": max_rows,
           "hops": 3, "lr": 3e-4, "init": "copy prior", "warmup_steps": 10}
    fd, ckpt = tempfile.mkstemp(suffix=".ckpt")
    os.close(fd)
    try:
        t = time.time()
        with rwr.Context(g.n, g.src, g.dst, seeds, **kw) as tr:
            tr.model_set(th_copy)
            tr.model_trainable(trainable_mask(), warmup=10)
            tr.warm_start("predict+train", hops=3, lr=3e-4, max_rows=max_rows)
            st = [tr.update_batch(b) for b in train]
            torch.cuda.synchronize()
            res["train_s"] = time.time() - t
            th = tr.model_get()
            tr.save(ckpt)
        k = min(100, max(1, n_train // 10))
        res["train_loss_first_last"] = [float(np.mean([s["ws_loss"] for s in st[:k]])),
                                        float(np.mean([s["ws_loss"] for s in st[-k:]]))]
        res["train_ms_per_update"] = 1e3 * res["train_s"] / max(1, n_train)
        log(f"[{w.name}] trained in {res['train_s']:.1f}s, loss (first/last {k}) {res['train_loss_first_last']}")
        for name, params in (("plain", None), ("trained", th), ("copy_prior", th_copy),
                             ("propagation_prior", th_prop)):
            with rwr.Context.load(ckpt) as ctx:
                if params is None:
                    ctx.warm_start("off")
                else:
                    ctx.model_set(params)
                    ctx.warm_start("predict", hops=3, max_rows=max_rows)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = [ctx.update_batch(b) for b in held]
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                mods = sum(b.size for b in held)
                r = {"updates_per_s": n_eval / el, "modifications_per_s": mods / el, "ms_per_update": 1e3 * el / n_eval,
                     "mean_iters": float(np.mean([s["iters"] for s in st])),
                     "mean_dense_sweeps": float(np.mean([s["dense_iters"] for s in st])),
                     "residual_checks": int(sum(s["checked"] for s in st)),
                     "max_err_bound": float(max(s["err_bound"] for s in st))}
                if params is not None:
                    r["mean_resid_ratio"] = float(np.mean([s["ws_resid_ratio"] for s in st]))
                    r["mean_accepted_columns"] = float(np.mean([s["ws_accepted"] for s in st]))
                    r["mean_region_nodes"] = float(np.mean([s["ws_region"] for s in st]))
                    r["mean_warm_ms"] = float(np.mean([s["ms_warm"] for s in st]))
                if name == "trained" and check:
                    import oracle

                    from paper_1712_00595_amd import accuracy

                    n2, s2, d2 = oracle.apply_stream(g.n, g.src, g.dst, stream)
                    errs, ranks = [], []
                    for j in (0, 15):
                        ref = oracle.rwr_static(n2, s2, d2, int(seeds[j]), w.c)
                        got = ctx.scores(j)
                        errs.append(float(np.abs(got - ref).sum()))
                        ranks.append(rank_accuracy(accuracy, got, ref))
                    r["parity"] = {"columns": [0, 15], "l1_vs_oracle": errs, "rank_accuracy": ranks,
                                   "ok": max(errs) <= res["gate"]}
                res[name] = r
                log(f"[{w.name}] {name}: {r['updates_per_s']:.1f} updates/s, iters {r['mean_iters']:.2f}"
                    + (f", resid ratio {r['mean_resid_ratio']:.3f}" if params is not None else ""))
    finally:
        os.remove(ckpt)
    return res


def run_delta_study(check: bool, per_group: int = 10) -> dict:
    """Effects of Delta G (Section 3.3; the size and location experiments of
    Section 4) on the scale-20 R-MAT graph, one seed, eps = 1e-9, FP32
    propagation and no error-budget refinement (plain OSP-T, as measured in
    the paper).  Location: nodes sorted by their RWR score in 100 equal
    groups, `per_group` sampled nodes per group with at least one out-edge;
    for each, one out-edge (u, v) is deleted (the measured update) and then
    re-inserted.  Size: k uniform existing edges deleted in one batch for
    k = 1 .. 1e5, then re-inserted.  Every update is checked against the
    cost model: Theorem 2's iteration bound from ||q_offset||_1 and, before
    propagation, from ||D r_old||_1."""
    from paper_1712_00595_amd import accuracy, costmodel, rwr
    from synth.configs import RMAT20_SINGLE_EDGE

    w = RMAT20_SINGLE_EDGE
    t0 = time.time()
    g = w.graph()
    seeds = w.seeds(g)
    eps, c = 1e-9, w.c
    log(f"[rmat20_delta_study] graph n={g.n} m={g.m} ({time.time() - t0:.1f}s)")
    order = np.argsort(g.src, kind="stable")
    dst_sorted = g.dst[order]
    start = np.concatenate([[0], np.cumsum(np.bincount(g.src, minlength=g.n))])
    rng = np.random.default_rng(4)
    e32 = np.zeros(0, np.int32)

    def within(st):
        return (st["iters"] <= costmodel.iterations_bound(st["q_off_l1"], eps, c),
                st["iters"] <= costmodel.iterations_bound_before(st["dr_l1"], eps, c))

    res = {"graph": "directed R-MAT scale 20 (as the headline)", "c": c, "eps": eps, "refinement": "off"}
    # location: groups of nodes by descending score
    with rwr.Context(g.n, g.src, g.dst, seeds, c=c, eps=eps, precision="fp32", err_budget=1.0) as ctx:
        score = ctx.scores(0)
        by_score = np.argsort(-score, kind="stable")
        groups = np.array_split(by_score, 100)
        rows = []
        for gi, grp in enumerate(groups):
            cand = grp[start[grp + 1] > start[grp]]
            pick = rng.choice(cand, size=min(per_group, cand.shape[0]), replace=False)
            for u in pick:
                u = int(u)
                v = int(dst_sorted[start[u] + rng.integers(0, start[u + 1] - start[u])])
                st = ctx.update(del_src=np.array([u], np.int32), del_dst=np.array([v], np.int32))
                ctx.update(ins_src=np.array([u], np.int32), ins_dst=np.array([v], np.int32))
                rows.append((gi, st["iters"], st["ms_total"], st["q_off_l1"], st["dr_l1"], st["visited_edges"],
                             *within(st)))
    R = np.array(rows, dtype=np.float64)
    gmean = lambda col: [float(R[R[:, 0] == gi, col].mean()) for gi in range(100)]  # noqa: E731
    mean_iters = gmean(1)
    res["location"] = {
        "groups": 100, "per_group": per_group, "updates": int(R.shape[0]),
        "mean_iters": mean_iters, "mean_ms": gmean(2), "mean_q_off_l1": gmean(3), "mean_dr_l1": gmean(4),
        "mean_visited_edges": gmean(5),
        # rank correlation of the group's score rank with its iterations
        # (negative: higher scores, more iterations)
        "spearman_group_vs_iters": accuracy.spearman(np.arange(100), mean_iters),
        "iters_within_bound_q": float(R[:, 6].mean()), "iters_within_bound_dr": float(R[:, 7].mean()),
    }
    log(f"[rmat20_delta_study] location: iters top group {mean_iters[0]:.1f}, bottom {mean_iters[-1]:.1f}")
    # size: one batch of k deletions, then the same edges re-inserted
    sizes = []
    with rwr.Context(g.n, g.src, g.dst, seeds, c=c, eps=eps, precision="fp32", err_budget=1.0) as ctx:
        for k in (1, 10, 100, 1000, 10000, 100000):
            idx = rng.choice(g.m, size=k, replace=False)
            ds, dd = g.src[idx].astype(np.int32), g.dst[idx].astype(np.int32)
            st = ctx.update(del_src=ds, del_dst=dd)
            row = {"k": k, "iters": st["iters"], "dense_iters": st["dense_iters"], "ms": st["ms_total"],
                   "q_off_l1": st["q_off_l1"], "dr_l1": st["dr_l1"], "visited_edges": st["visited_edges"],
                   "bound_q": costmodel.iterations_bound(st["q_off_l1"], eps, c),
                   "bound_dr": costmodel.iterations_bound_before(st["dr_l1"], eps, c),
                   "err_bound": st["err_bound"]}
            if check:
                import oracle

                from synth.stream import Batch

                b = Batch(ins_src=e32, ins_dst=e32, del_src=ds, del_dst=dd, n_new_nodes=0)
                n2, s2, d2 = oracle.apply_batch(g.n, g.src, g.dst, b)
                ref = oracle.rwr_static(n2, s2, d2, int(seeds[0]), c)
                got = ctx.scores(0)
                row["l1_vs_oracle"] = float(np.abs(got - ref).sum())
                row["spearman"] = accuracy.spearman(got, ref)
            sizes.append(row)
            ctx.update(ins_src=ds, ins_dst=dd)
            log(f"[rmat20_delta_study] size {k}: iters {row['iters']} (bounds {row['bound_q']}, {row['bound_dr']}), "
                f"{row['ms']:.2f} ms")
    res["size"] = sizes
    return res


def run_churn(n_batches: int, check: bool) -> dict:
    """Symmetrised R-MAT scale 23 (134,217,728 pairs stored in both
    directions), c = 0.05, 16 uniform seeds, eps = 1e-9; each batch deletes
    1% of the pairs, inserts as many uniform absent pairs and adds 1000 nodes
    with 1-8 edges.  Batches are generated before the clock starts."""
    import torch

    from paper_1712_00595_amd import rwr
    from synth.churn import PairPool, churn_stream
    from synth.configs import RMAT23_UNDIRECTED

    w = RMAT23_UNDIRECTED
    t = time.time()
    g = w.graph()
    seeds = w.seeds(g)
    pool = PairPool(g.n, g.pair_u, g.pair_v)
    log(f"[{w.name}] graph n={g.n} pairs={g.pair_u.shape[0]} ({time.time() - t:.1f}s)")
    stream = []
    for b in churn_stream(pool, n_batches, 0.01, 1000, seed=4):
        stream.append(b)
        if len(stream) % 10 == 0:
            log(f"[{w.name}] {len(stream)} of {n_batches} batches drawn ({time.time() - t:.1f}s)")
    eps = w.eps[0]
    t = time.time()
    ctx = rwr.Context(g.n, g.pair_u, g.pair_v, seeds, c=w.c, eps=eps, precision="fp32", undirected=True)
    torch.cuda.synchronize()
    build_s = time.time() - t
    log(f"[{w.name}] context built in {build_s:.1f}s")
    ctx.profile(True)
    ctx.profile_read(reset=True)
    mods = sum(b.size for b in stream)
    t0 = time.perf_counter()
    stats = []
    for i, b in enumerate(stream):
        stats.append(ctx.update_batch(b))
        if (i + 1) % 25 == 0:
            log(f"[{w.name}] {i + 1} batches")  # a line per 25 batches (each takes about a second)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    P = ctx.profile_read(reset=True)
    res = {
        "batches": len(stream),
        "batches_configured": 100,
        "edge_and_node_modifications": mods,
        "modifications_per_s": mods / el,
        "batches_per_s": len(stream) / el,
        "build_s": build_s,
        "mean_iters": float(np.mean([s["iters"] for s in stats])),
        "mean_dense_sweeps": float(np.mean([s["dense_iters"] for s in stats])),
        "refinements": int(sum(s["refined"] for s in stats)),
        "max_err_bound": float(max(s["err_bound"] for s in stats)),
        "gate": 2 * eps / w.c,
    }
    launches = P["dense_sweeps"] + P["idle_launches"]
    if P["dense_sweeps"]:
        sweep_bytes = dense_sweep_bytes(ctx.n, ctx.m, 16)
        res["roofline"] = {
            "bound": "hbm",
            "kernel": "k_pull_v<float, 16, *, KIND_DENSE> (dense sweep, 16 columns)",
            "achieved": sweep_bytes * P["dense_sweeps"] / (P["dense_ms"] * 1e-3) / 1e9,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "bytes_per_sweep": sweep_bytes,
            "avg_launch_us": 1e3 * P["dense_ms"] / launches,
            "avg_sweep_us": 1e3 * P["dense_ms"] / P["dense_sweeps"],
            "launches": launches,
            "idle_launches": P["idle_launches"],
        }
        res["roofline"]["frac"] = res["roofline"]["achieved"] / HBM_PEAK_GBS
    res["sweep_shape"] = ctx.sweep_shape()
    if check:
        import oracle

        t = time.time()
        lo = np.minimum(pool.keys // (1 << 32), pool.keys % (1 << 32))
        hi = np.maximum(pool.keys // (1 << 32), pool.keys % (1 << 32))
        loop = lo == hi
        s2 = np.concatenate([lo, hi[~loop]]).astype(np.int32)
        d2 = np.concatenate([hi, lo[~loop]]).astype(np.int32)
        from paper_1712_00595_amd import accuracy

        ref = oracle.rwr_static(pool.n, s2, d2, int(seeds[0]), w.c, tol=1e-12)
        got = ctx.scores(0)
        err = float(np.abs(got - ref).sum())
        res["parity"] = {"columns": [0], "l1_vs_oracle": [err], "rank_accuracy": [rank_accuracy(accuracy, got, ref)],
                         "oracle_tol": 1e-12, "ok": err <= res["gate"], "oracle_s": time.time() - t}
    ctx.close()
    log(f"[{w.name}] {res['batches_per_s']:.3f} batches/s, {res['modifications_per_s']:.0f} modifications/s")
    return res


def run_c2_modes(names, K: int, W: int, check: bool, cpu_baseline: bool, cpu_sample: int,
                 host_batches: bool = False) -> dict:
    """The scale-20 single-seed stream of single-edge updates: the modes in
    ``names`` (eps = 1e-9 first), each a fresh context, W warm-up and K timed
    updates staged in HBM."""
    import torch

    from paper_1712_00595_amd import rwr
    from synth.configs import RMAT20_SINGLE_EDGE, stream_for

    w = RMAT20_SINGLE_EDGE
    t = time.time()
    g = w.graph()
    seeds = w.seeds(g)
    model = w.model(g)
    stream = stream_for(w, model, W + K)
    log(f"graph n={g.n} m={g.m} seed={int(seeds[0])} stream={len(stream)} updates ({time.time() - t:.1f}s)")

    c = w.c
    all_modes = {
        "eps1e-9": dict(eps=1e-9, err_budget=0.0, gate=2 * 1e-9 / c),
        "eps1e-6": dict(eps=1e-6, err_budget=0.0, gate=2 * 1e-6 / c),
        # exact: the certified budget is the 1e-9 gate itself; eps is chosen so
        # one update's truncation bound is a tenth of it
        "exact": dict(eps=1e-9 * c / (20 * (1 - c)), err_budget=1e-9, gate=1e-9),
        # global PageRank: the uniform restart vector instead of the seed node
        "pagerank": dict(eps=1e-9, err_budget=0.0, gate=2 * 1e-9 / c, q="uniform"),
    }
    headline = names[0]

    # the timed updates' batches, staged in HBM before the clock starts: one
    # device array per field, each update passes views into them
    dev_stream = stage_batches(stream[W:W + K])

    def run(name, host_batches=False, profile=False):
        mcfg = all_modes[name]
        t = time.time()
        if mcfg.get("q") == "uniform":
            ctx = rwr.Context(g.n, g.src, g.dst, q=np.full(g.n, 1.0 / g.n), c=c, eps=mcfg["eps"],
                              err_budget=mcfg["err_budget"], precision="fp32")
        else:
            ctx = rwr.Context(g.n, g.src, g.dst, seeds, c=c, eps=mcfg["eps"], err_budget=mcfg["err_budget"],
                              precision="fp32")
        log(f"[{name}{' host batches' if host_batches else ''}] context built in {time.time() - t:.2f}s")
        for b in stream[:W]:
            ctx.update_batch(b)
        ctx.profile(profile)
        ctx.profile_read(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if host_batches:
            stats = [ctx.update_batch(b) for b in stream[W:W + K]]
        else:
            stats = [ctx.update(*u[:4], n_new_nodes=u[4]) for u in dev_stream]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = ctx.profile_read(reset=True)
        return ctx, stats, t1 - t0, prof

    results = {}
    final_ctx_scores = None
    for name in names:
        mcfg = all_modes[name]
        ctx, stats, el, _ = run(name)
        lat = np.array([s["ms_total"] for s in stats])
        iters = np.array([s["iters"] for s in stats])
        dense = np.array([s["dense_iters"] for s in stats])
        res = {
            "updates_per_s": K / el,
            "ms_per_update": 1e3 * el / K,
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "mean_iters": float(iters.mean()),
            "mean_dense_sweeps": float(dense.mean()),
            "residual_checks": int(sum(s["checked"] for s in stats)),
            "refinements": int(sum(s["refined"] for s in stats)),
            "max_err_bound": float(max(s["err_bound"] for s in stats)),
            "eps": mcfg["eps"],
            "gate": mcfg["gate"],
            "visited_edges_per_update": float(np.mean([s["visited_edges"] for s in stats])),
        }
        if mcfg.get("q") == "uniform" and check:
            import oracle
            from paper_1712_00595_amd import accuracy

            n2, s2, d2 = oracle.apply_stream(g.n, g.src, g.dst, stream[:W + K])
            qp = np.zeros(n2)
            qp[: g.n] = 1.0 / g.n  # nodes added by the stream restart with probability 0
            ref = oracle.rwr_static_vector(n2, s2, d2, qp, c)
            got = ctx.scores(0)
            err = float(np.abs(got - ref).sum())
            res["parity"] = {"l1_vs_oracle": err, "ok": err <= mcfg["gate"],
                             "rank_accuracy": rank_accuracy(accuracy, got, ref)}
        if name == headline:
            src_e, dst_e, _ = ctx.export()
            res["n_final"], res["m_final"] = ctx.n, int(src_e.shape[0])
            if check:
                final_ctx_scores = ctx.scores(0)
        log(f"[{name}] {res['updates_per_s']:.1f} updates/s, {res['ms_per_update']:.3f} ms/update, "
            f"iters {res['mean_iters']:.1f} (dense {res['mean_dense_sweeps']:.1f}), "
            f"checks {res['residual_checks']} refinements {res['refinements']}, bound {res['max_err_bound']:.2e}")
        ctx.close()
        if name == headline:
            # the same updates again with every sweep launch timed by HIP
            # events (the roofline of the single-column sweep)
            ctx, _, el_p, prof = run(name, profile=True)
            res["prof"] = prof
            res["profiled_pass_updates_per_s"] = K / el_p
            ctx.close()
        if name == headline and host_batches:
            # the same updates with each batch handed over in host memory (one
            # small host-to-device copy per update inside the call)
            ctx, _, el_h, _ = run(name, host_batches=True)
            res["host_batches_updates_per_s"] = K / el_h
            log(f"[{name} host batches] {K / el_h:.1f} updates/s")
            ctx.close()
        results[name] = res

    H = results[headline]
    # roofline of the dominant kernel: the dense sweep (k_pull_wv, one pull
    # over every in-row).  Every launch in the timed region is timed; the
    # algorithmic bytes per launch average the launches that swept (launches
    # that found the run converged move no data but count in the time).
    roof = None
    P = H["prof"]
    launches = P["dense_sweeps"] + P["idle_launches"]
    if P["dense_sweeps"] > 0:
        sweep_bytes = dense_sweep_bytes(H["n_final"], H["m_final"])
        avg_us = 1e3 * P["dense_ms"] / launches
        bytes_per_launch = sweep_bytes * P["dense_sweeps"] / launches
        achieved = bytes_per_launch / (avg_us * 1e-6) / 1e9
        traffic = measured_traffic(sweep_bytes, TRAFFIC_C2)
        roof = {
            "bound": "hbm",
            "kernel": "k_pull_wv<float, KIND_DENSE, 4, 6144> (dense sweep, one seed, FP32 gather)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None if traffic is None else traffic * P["dense_sweeps"] / launches,
            "bytes_per_sweep": sweep_bytes,
            "bytes_per_launch": bytes_per_launch,
            "avg_launch_us": avg_us,
            "avg_sweep_us": 1e3 * P["dense_ms"] / P["dense_sweeps"],
            "launches": launches,
            "idle_launches": P["idle_launches"],
        }

    parity = None
    cpu = None
    if check or cpu_baseline:
        import oracle

        if check and final_ctx_scores is not None:
            t = time.time()
            # the final graph: the whole stream applied to the edge list
            n2, s2, d2 = oracle.apply_stream(g.n, g.src, g.dst, stream)
            from paper_1712_00595_amd import accuracy

            ref = oracle.rwr_static(n2, s2, d2, int(seeds[0]), c)
            err = float(np.abs(final_ctx_scores - ref).sum())
            parity = {"l1_vs_oracle": err, "gate": H["gate"], "ok": err <= H["gate"],
                      "rank_accuracy": rank_accuracy(accuracy, final_ctx_scores, ref),
                      "oracle_static_s": time.time() - t}
            log(f"parity: L1 {err:.3e} vs gate {H['gate']:.3e} ({time.time() - t:.1f}s)")
        if cpu_baseline:
            t = time.time()
            r_old = oracle.rwr_static(g.n, g.src, g.dst, int(seeds[0]), c)
            static_s = time.time() - t
            n0, s0, d0 = g.n, g.src, g.dst
            sample = stream[:cpu_sample]
            t = time.time()
            for b in sample:
                n1, s1, d1 = oracle.apply_batch(n0, s0, d0, b)
                out = oracle.osp((n0, s0, d0), (n1, s1, d1), r_old, c, all_modes[headline]["eps"], renorm=1)
                r_old, n0, s0, d0 = out["r_new"], n1, s1, d1
            el = time.time() - t
            cpu = {
                "value": len(sample) / el,
                "unit": "updates/s",
                "cores": cpu_count_used(),
                "kind": "oracle",
                "sample": f"Algorithm 1 (oracle/rwr_oracle.c, single-threaded FP64, full edge sweeps) on the first "
                          f"{len(sample)} updates of the same stream at eps={all_modes[headline]['eps']:g}, from the "
                          f"oracle's static scores; static solve of the initial graph took {static_s:.1f}s",
                "static_solve_s": static_s,
                "host_cpu": host_cpu_model(),
                "host_threads": os.cpu_count(),
            }
            log(f"cpu baseline: {cpu['value']:.3f} updates/s (static solve {static_s:.1f}s)")

    H["roofline"] = roof
    H["cpu_baseline"] = cpu
    H["parity"] = parity
    H["workload"] = w.name
    H["cache_resident"] = "the working set (about 0.1 GB) fits the 256 MB Infinity Cache: a latency figure"
    return results


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed batches of the headline workload")
    ap.add_argument("--warmup", type=int, default=5, help="warm-up batches of the headline workload")
    ap.add_argument("--modes", default="eps1e-9",
                    help="modes of the scale-20 single-edge stream reported under 'modes': comma list of "
                         "eps1e-9, eps1e-6, exact, pagerank; all; or none")
    ap.add_argument("--c2-steps", type=int, default=1000, help="timed updates of the single-edge stream")
    ap.add_argument("--c2-warmup", type=int, default=20, help="warm-up updates of the single-edge stream")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle comparisons")
    ap.add_argument("--no-host-batches", action="store_true",
                    help="skip the single-edge stream's run that hands batches over in host memory")
    ap.add_argument("--cpu-sample", type=int, default=3, help="single-edge updates timed on the CPU oracle")
    ap.add_argument("--workloads", default="",
                    help="extra workloads run after the headline, comma list of: "
                         "rmat21_learned_warm_start, rmat23_undirected_churn, rmat20_delta_study")
    ap.add_argument("--churn-batches", type=int, default=100, help="batches of the undirected churn workload")
    ap.add_argument("--churn-check", action="store_true", help="check one column of the churn workload (slow)")
    ap.add_argument("--learned-train", type=int, default=5000, help="training updates of the learned workload")
    ap.add_argument("--learned-eval", type=int, default=500, help="held-out updates of the learned workload")
    ap.add_argument("--learned-max-rows", type=int, default=0,
                    help="region capacity of the learned warm start in (node, column) rows (0: the default)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run one elementwise copy of MIB MiB (calibrates the traffic counters) and exit")
    args = ap.parse_args()

    if args.copy_calibration:
        # one elementwise kernel that reads and writes MIB MiB each: the
        # traffic counters' reading for it, divided by the bytes, is the
        # factor that turns the sweep's counter readings into bytes
        import torch

        nbytes = args.copy_calibration << 20
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.add(a, 1.0, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"copy_read_bytes": nbytes, "copy_write_bytes": nbytes}))
        return 0

    if args.gpus != 1:
        print(
            "bench.py measures one GPU (--gpus 1): the update path runs on a single MI355X; "
            "sharding it across GPUs is not implemented.",
            file=sys.stderr,
        )
        return 2

    import torch

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 3
    torch.cuda.set_device(0)

    check, cpu = not args.no_check, not args.no_cpu_baseline
    H = run_batched_seeds(args.steps, args.warmup, check, cpu)
    modes = {}
    if args.modes != "none":
        names = ["eps1e-9", "eps1e-6", "exact", "pagerank"] if args.modes == "all" else args.modes.split(",")
        modes = run_c2_modes(names, args.c2_steps, args.c2_warmup, check, False, args.cpu_sample,
                             not args.no_host_batches)

    extra = {}
    for wname in [x for x in args.workloads.split(",") if x]:
        if wname == "rmat21_learned_warm_start":
            extra[wname] = run_learned(args.learned_train, args.learned_eval, check, args.learned_max_rows)
        elif wname == "rmat23_undirected_churn":
            extra[wname] = run_churn(args.churn_batches, args.churn_check)
        elif wname == "rmat20_delta_study":
            extra[wname] = run_delta_study(check)
        else:
            raise SystemExit(f"unknown workload {wname}")

    from synth.configs import RMAT22_BATCHED as w

    out = {
        "metric": "RWR updates/sec at L1 err<=2eps/c",
        "value": H["modifications_per_s"],
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": H["ms_per_batch"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "graph": f"directed R-MAT scale {w.scale} (a,b,c,d)=(.57,.19,.19,.05), {w.m} edges + dead-end "
                     f"self-loops, seeded vertex permutation",
            "c": w.c,
            "eps": w.eps[0],
            "gate_l1": H["gate"],
            "seeds": w.n_seeds,
            "step": "one batch of log-uniform size in [1, 10^4] edge modifications (50% insertions of absent "
                    "pairs / 50% deletions of existing edges) with 1% new nodes carrying 1-8 out-edges; an update "
                    "is one edge or node modification, every seed column within the gate after every batch",
            "propagation": "f32 vectors, f64 score accumulation",
        },
        "roofline": H.get("roofline"),
        "cpu_baseline": H.get("cpu_baseline"),
        "parity": H.get("parity"),
        "headline": {k: v for k, v in H.items() if k not in ("roofline", "cpu_baseline", "parity")},
        "modes": modes,
    }
    if extra:
        out["workloads"] = extra
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
