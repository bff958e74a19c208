/*
 * rwr.h -- C ABI of the MI355X dynamic random-walk-with-restart library.
 *
 * The library keeps, on one GPU, a directed (or undirected) graph and the
 * random-walk-with-restart (RWR) score vectors of S seed nodes, and keeps the
 * scores current while batches of edge and node insertions and deletions
 * arrive, by offset score propagation (OSP, Section 3.1 and Algorithm 1 of
 * Yoon, Jin and Kang, "Fast and Accurate Random Walk with Restart on Dynamic
 * Graphs with Guarantees", WWW 2018), or its tolerance-driven variant OSP-T
 * (Section 3.2).
 *
 * Scores (Eq. 1, Section 2.1): r = (1-c) A~^T r + c q with q = e_s, where A~
 * is the row-normalised adjacency matrix (rows of dead ends are zero; dead
 * ends are handled by Theorem 4's rescaling, Section 3.4.2).
 *
 * Conventions for every entry point
 *   - Every call returns rwr_status (0 = RWR_OK, negative = error); no C++
 *     exception crosses this boundary.  A text for the last error of a
 *     context is returned by rwr_last_error().
 *   - Calls are synchronous with respect to the host on return: every output
 *     (scores, statistics, exported arrays) is final and no array the caller
 *     passed is read any more.  rwr_update may leave work queued on the
 *     context's stream that only prepares the next update from the context's
 *     own buffers; every later call on the context, rwr_destroy included, is
 *     ordered after it.  One context uses one HIP stream; a context is not
 *     thread-safe.
 *   - The caller owns every array it passes; the library copies what it
 *     keeps.  A pointer flagged "on device" must be device memory of the
 *     context's GPU, readable for the duration of the call.
 *   - Node ids are int32 in [0, n); edge counts are int64.
 */
#ifndef RWR_H_
#define RWR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rwr_ctx rwr_ctx;

typedef enum rwr_status {
  RWR_OK = 0,
  RWR_EINVAL = -1,   /* bad argument, id out of range, duplicate entry in a batch */
  RWR_ENOMEM = -2,   /* device or host allocation failed                        */
  RWR_EHIP = -3,     /* a HIP runtime call failed                               */
  RWR_EEXIST = -4,   /* batch inserts an edge that is already present           */
  RWR_ENOENT = -5,   /* batch deletes an edge that is not present               */
  RWR_ENOCONV = -6,  /* max_iters reached before ||x^(i)||_1 <= eps             */
  RWR_ENUMERIC = -7, /* non-finite norm met during propagation                  */
  RWR_ESTATE = -8,   /* context unusable (an earlier call left it stale)        */
  RWR_EIO = -9       /* checkpoint file cannot be written, read or recognised   */
} rwr_status;

/* Precision of the propagated vectors x^(i).  Scores r and their sums are
 * always accumulated in FP64. */
typedef enum rwr_precision { RWR_PROP_FP32 = 0, RWR_PROP_FP64 = 1 } rwr_precision;

typedef struct rwr_config {
  double c;          /* restart probability, 0 < c < 1 (Section 2.1)                    */
  double eps;        /* stop when ||x^(i)||_1 <= eps in every seed column (Alg. 1)      */
  double err_budget; /* L1 error budget per seed column of the scores kept between
                        updates; <= 0 selects 2*eps/c (Theorem 3 with rescaling)        */
  double build_tol;  /* certified L1 error of the initial static solve; <= 0 selects
                        err_budget/4                                                    */
  int32_t precision; /* rwr_precision                                                   */
  int32_t undirected;/* 1: each batch pair (u,v) stands for both directions             */
  int32_t max_iters; /* per-update iteration guard; <= 0 selects 10000                  */
  int32_t pull_ratio;/* switch from sparse push to dense pull once the frontier's
                        out-edges exceed m/pull_ratio; <= 0 selects the tuned default   */
  int32_t reorder;   /* 1: number nodes internally by descending out-degree (ids at
                        this interface are unchanged); 0: keep the caller's order      */
  int32_t autotune;  /* 1: the build's static solve times candidate shapes of the dense
                        sweep (lanes per row, workgroups) on its first sweeps and keeps
                        the fastest; 0: the fixed defaults.  Environment RWR_TUNE_CACHE
                        = a text file: a build whose workload (device, n, m, S,
                        precision, in-degree histogram) is listed there takes the
                        listed shape without timing; a tuned build appends its line   */
  void *stream;      /* hipStream_t to run on; NULL: the library creates its own        */
  int32_t deterministic; /* 1: results do not depend on timing -- no floating-point atomics
                            on the score path: the offset seed's terms are written as
                            keyed records, radix-sorted and summed per node in sorted
                            order (the default mode does this too for large batches at
                            32 or more columns, and scatters with atomics otherwise),
                            propagation runs dense
                            pull sweeps only (no sparse push phase), the sweep shape is not
                            tuned by timing (autotune ignored), and the warm-start
                            network's aggregations sum each row in edge order; two runs of
                            the same stream on the same device give bitwise equal scores,
                            statistics and trained parameters                          */
  int32_t node_deletion; /* 0: a deleted node loses every incident edge (row and column);
                            1: only its row, as Section 3.4.1 states it (its in-edges stay
                            and it becomes a dead end, Theorem 4); undirected graphs store
                            one structure, so there both readings remove every pair     */
  int32_t phase_timing;  /* 1: rwr_stats.ms_delta .. ms_merge from HIP events (a few
                            event records per update); 0: those fields are 0           */
  /* device memory of the context: when dev_alloc is set, every device buffer the
     context keeps or stages comes from dev_alloc(bytes, stream, alloc_user) and goes
     back through dev_free(p, stream, alloc_user) (e.g. a framework's caching
     allocator); `stream` is the context's stream, on which all its device work runs,
     so a freed block may be reused by work queued after the free on that stream.
     Both NULL: hipMalloc / hipFree; one without the other is RWR_EINVAL.  dev_alloc
     returns NULL on failure (RWR_ENOMEM) and 256-byte aligned memory otherwise.
     (Pinned host memory of the control block still comes from hipHostMalloc.)     */
  void *(*dev_alloc)(size_t bytes, void *stream, void *user);
  void (*dev_free)(void *p, void *stream, void *user);
  void *alloc_user;
} rwr_config;

/* A batch is a set (Theorem 1: only the graphs before and after matter).
 * New nodes get ids n .. n+n_new_nodes-1 and may be named by this batch's
 * insertions (Section 3.4.1).  A deleted node loses every incident edge and
 * keeps its id with a zero row and column (Section 3.4.1).  del_nodes lists
 * distinct ids of existing nodes (< n before the batch), none of them a seed
 * (the walk restarts there), none named by this batch's edge entries; the
 * removed edges then count as deletions of the batch.  The same edge may not
 * appear twice, nor be both inserted and deleted.  In undirected mode a pair
 * is given once, in either orientation.  Any violation is RWR_EINVAL. */
typedef struct rwr_batch {
  int64_t n_ins;
  const int32_t *ins_src;
  const int32_t *ins_dst;
  int64_t n_del;
  const int32_t *del_src;
  const int32_t *del_dst;
  int32_t n_new_nodes;
  int32_t n_del_nodes;
  const int32_t *del_nodes;
  int32_t on_device; /* 1: the five arrays above are device pointers */
} rwr_batch;

/* Per-update statistics; norms are maxima over seed columns. */
typedef struct rwr_stats {
  int32_t iters;          /* propagation iterations of this update (Alg. 1 loop)           */
  int32_t dense_iters;    /* of which dense pull sweeps                                    */
  int32_t refined;        /* 1 if a residual refinement ran after this update              */
  int32_t checked;        /* 1 if the FP64 residual was evaluated after this update        */
  int64_t visited_edges;  /* edges read by propagation (Table 3's "visited edges")         */
  int64_t touched_rows;   /* rows of A~ changed by the batch                               */
  double q_off_l1;        /* ||q_offset||_1 (Section 3.1)                                  */
  double last_x_l1;       /* ||x^(k)||_1 of the last iteration                             */
  double err_bound;       /* L1 error bound of the scores after this update                */
  double residual_l1;     /* ||residual||_1 when checked, else 0                           */
  double ms_total;        /* wall time of the call (host clock)                            */
  /* learned warm start (zero when it is off) */
  int32_t ws_region;      /* region nodes the network ran on                               */
  int32_t ws_accepted;    /* seed columns whose seed was replaced by the residual          */
  double ws_resid_ratio;  /* sum_j ||rho_j||_1 / sum_j ||q_j||_1 of the prediction          */
  double ws_loss;         /* training loss of this update, sum_j ||rho_j|| / sum_j ||q_j|| */
  double ms_warm;         /* host wall time of the warm-start steps                        */
  /* cost model of the batch (Section 3.3, effects of Delta G): ||D r_old||_1 with
     D_uu = sum_v |B~[u,v] - A~[u,v]| (row L1 norm of the change of u's row), an
     upper bound of ||q_offset||_1 / (1-c) known before propagation          */
  double dr_l1;
  /* ||p||_1 of a vector carried from an earlier update into this one's first
     dense sweep (the FP64 residual of a check that needed no refinement, or
     the last iterate a run left unpropagated), 0 when none joined          */
  double carry_l1;
  int32_t fallback;       /* warm start: columns with an offset seed that kept it (the
                             prediction's residual was not smaller)                        */
  int32_t flushed;        /* columns whose error bound passed the budget and were refined  */
  /* GPU time per phase (config phase_timing = 1, else 0): batch upload, check and
     structural apply; offset seed (Section 3.1); learned warm start; propagation
     (Algorithm 1's loop); stream error check, refinement and clean-up           */
  double ms_delta, ms_seed, ms_model, ms_prop, ms_merge;
} rwr_stats;

/* Fill *cfg with defaults: c = 0.15, eps = 1e-9, FP32 propagation, directed,
 * internal degree ordering on, sweep-shape tuning on. */
rwr_status rwr_config_default(rwr_config *cfg);

/* Build a context: copy the graph (n nodes, m edges (src[e], dst[e]); in
 * undirected mode m pairs, each stored in both directions) to the GPU, and
 * compute the static scores of each seed column by cumulative power iteration
 * from c*e_s (Section 2.2) followed by FP64 residual refinement until the
 * certified error is below cfg->build_tol.  Multi-edges are rejected
 * (RWR_EINVAL); self-loops are allowed and count in the out-degree.
 * n_seeds in [1, 64]; seeds distinct ids in [0, n).  edges_on_device: src/dst
 * are device pointers.  On success *out owns all device memory of the
 * context. */
rwr_status rwr_build(const rwr_config *cfg, int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                     int32_t n_seeds, const int32_t *seeds, int32_t edges_on_device, rwr_ctx **out);

/* Build a context whose columns restart to general seed vectors instead of
 * seed nodes: column j solves r_j = (1-c) A~^T r_j + c q_j (Eq. (1) with the
 * restart vector q_j in place of e_s; q_j = 1/n everywhere is global
 * PageRank), by cumulative power iteration from c*q_j (Section 2.2).  q is a
 * HOST array of n * n_cols doubles, node-major (q[v * n_cols + j]), copied;
 * every column must be nonnegative, finite and sum to 1 within 1e-9
 * (RWR_EINVAL otherwise).  Updates (rwr_update) propagate offsets exactly as
 * for seed nodes (the offset seed does not depend on q); the residual checks
 * use the full restart term c q.  q stays fixed: nodes added later have
 * q = 0, a deleted node keeps its entry.  The learned warm start is not
 * available on such a context (RWR_ESTATE).  Other arguments and ownership
 * as rwr_build. */
rwr_status rwr_build_vectors(const rwr_config *cfg, int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                             int32_t n_cols, const double *q, int32_t edges_on_device, rwr_ctx **out);

/* Apply one batch and update the scores (Algorithm 1): delta-apply on the
 * device graph, offset seed q_offset = (1-c)(B~^T - A~^T) r_old, cumulative
 * propagation on the new graph until ||x^(i)||_1 <= eps, merge into r, and
 * Theorem 4's rescaling.  If the accumulated error bound exceeds the budget,
 * the FP64 residual is evaluated and, if needed, propagated (refinement).
 * Between updates the library may carry a vector p that r already contains
 * and that r - p has as its residual (the last iterate of a run that ended in
 * the dense phase, or a residual that needed no refinement): the next update
 * then takes the offset seed of r - p and adds p to its first dense sweep
 * (stats->carry_l1); the scores read between updates are r, within
 * stats->err_bound.  Environment RWR_CARRY = 0 / 1 / 2: no carrying / the
 * residual only / both (default).
 * The batch is validated on the device before anything changes: on
 * RWR_EINVAL / RWR_EEXIST / RWR_ENOENT the graph and the scores are
 * unchanged.  On RWR_ENOCONV the graph is updated, the scores hold the
 * partial sum, stats->err_bound says how far off they may be and the context
 * is marked stale (rwr_refine() clears it).  stats may be NULL. */
rwr_status rwr_update(rwr_ctx *ctx, const rwr_batch *batch, rwr_stats *stats);

/* Evaluate the FP64 residual of the current scores and, in the columns whose
 * certified error exceeds an eighth of the budget, propagate it until the
 * certified error is below an eighth of the budget (clears a stale
 * context).  Its iteration guard is the larger of max_iters and Theorem 2's
 * bound for the residual's norm, so a context left stale by RWR_ENOCONV can
 * recover. */
rwr_status rwr_refine(rwr_ctx *ctx, rwr_stats *stats);

/* Replace the scores of seed column j by in[0..n) (normalised scores in
 * caller ids, n = the node count; host memory, or device memory when
 * in_on_device = 1), e.g. scores computed elsewhere.  Their error is unknown:
 * the column's error bound becomes infinite, so the next rwr_update, or
 * rwr_refine, evaluates the FP64 residual and refines.  Carried vectors are
 * dropped. */
rwr_status rwr_scores_set(rwr_ctx *ctx, int32_t j, const double *in, int64_t n, int32_t in_on_device);

/* Copy the normalised scores of seed column j (n doubles) to out (capacity
 * cap elements; host memory, or device memory when out_on_device = 1). */
rwr_status rwr_scores(rwr_ctx *ctx, int32_t j, double *out, int64_t cap, int32_t out_on_device);

/* Current node count and stored directed edge count. */
rwr_status rwr_graph_size(const rwr_ctx *ctx, int32_t *n, int64_t *m);

/* Copy the graph back to the host as a directed edge list in row order
 * (out-neighbours of node 0, then of node 1, ...).  src/dst have capacity
 * cap; *m_out receives the edge count.  Also copies out-degrees (n ints) to
 * deg_out when not NULL.  For checking and checkpointing; not a hot path. */
rwr_status rwr_graph_export(rwr_ctx *ctx, int32_t *src, int32_t *dst, int64_t cap, int64_t *m_out,
                            int32_t *deg_out);

/* Shape of the dense sweep in use: lanes per in-row (multi-column sweep)
 * and workgroups, and the median time of one sweep at that shape measured
 * while tuning, or read from the tuning cache (0 when the shape was not
 * tuned).  Any pointer may be NULL. */
rwr_status rwr_sweep_shape(const rwr_ctx *ctx, int32_t *lanes_per_row, int32_t *workgroups, double *tuned_ms);

/* Per-iteration ||x^(i)||_1 of seed column j during the last update (i = 0 is
 * ||q_offset||_1): copies min(cap, iters+1) values to out, count to *len. */
rwr_status rwr_last_norms(rwr_ctx *ctx, int32_t j, double *out, int32_t cap, int32_t *len);

/* Measurement of the dense sweep kernel (one pull over every in-row of the
 * graph, the bandwidth-bound step of the propagation, Section 2.2).  When
 * enabled, each launch of the sweep kernel in a propagation run is bracketed
 * by two HIP events on the context's stream (the epilogue and decision
 * kernels of the slot are outside the pair); after each run the elapsed
 * times of all these launches are summed.  Launches that swept the graph are
 * counted as sweeps; launches enqueued ahead that found the run already
 * converged return at once and are counted as idle (their time is in the
 * sum).  Residual checks are not included.  Adds two event records per dense
 * launch; off by default. */
rwr_status rwr_profile(rwr_ctx *ctx, int32_t enable);

/* Read (and with reset = 1 clear) the accumulated sweep-kernel time in ms
 * (all launches), the number of launches that swept and the number of idle
 * launches.  Any pointer may be
 * NULL. */
rwr_status rwr_profile_read(rwr_ctx *ctx, double *dense_ms, int64_t *dense_sweeps, int64_t *idle_launches,
                            int32_t reset);

/* Free every resource of the context; NULL is allowed. */
void rwr_destroy(rwr_ctx *ctx);

/* Checkpoint of a context (not part of the paper's method; for restarts of a
 * long update stream).  rwr_save writes everything the next update reads --
 * graph in its internal layout (node numbering, each row's entries in
 * storage order), scores, carried vectors and their bounds, the control block
 * (sigma per column, Theorem 4), run statistics, the sweep shape and the
 * heavy-row / row-order plans, and the warm-start network with its optimiser
 * state -- to `path` (written to path + ".part", then renamed).  rwr_load makes
 * a new context from such a file; `runtime` supplies only the fields that
 * cannot be saved (stream, dev_alloc, dev_free, alloc_user, phase_timing;
 * NULL: defaults), the rest of the configuration comes from the file.  A loaded
 * context continues the stream as the saved one would: with
 * deterministic = 1 on the same device, bitwise.  The format is the library's
 * own (native byte order, tied to this version: RWR_EIO otherwise).  Call
 * rwr_save between updates; the context is unchanged by it. */
rwr_status rwr_save(rwr_ctx *ctx, const char *path);
rwr_status rwr_load(const char *path, const rwr_config *runtime, rwr_ctx **out);

/* The configuration a context runs with (cfg, may be NULL), its column count
 * (n_seeds) and seed ids (seeds: room for RWR_MAX_COLS, -1 for columns built
 * from vectors; may be NULL). */
rwr_status rwr_context_info(const rwr_ctx *ctx, rwr_config *cfg, int32_t *n_seeds, int32_t *seeds);

/* Text of the last error recorded on ctx (or of the last failed rwr_build when
 * ctx is NULL).  The string lives until the next call on the same context. */
const char *rwr_last_error(const rwr_ctx *ctx);

/* ---------------------------------------------------------------------
 * Learned warm start (an addition to the paper's method).
 *
 * A small message-passing network predicts the offset result
 * r_offset = sum_i x^(i) of Section 3.1 on a region around the offset seed;
 * the update then propagates the exact residual
 *   rho = q_offset - (I - (1-c) B~^T) xhat,
 * so that r_offset = xhat + sum_i ((1-c) B~^T)^i rho holds identically and
 * the scores and bounds are those of Algorithm 1 (Theorems 1 and 3).
 *
 * Network: per (node, seed column) row, 16 input features -> ReLU(F W0 + b0)
 * (64 wide) -> three layers h' = ReLU(h Ws + a Wm + b) with
 * a(v) = sum over in-edges u -> v inside the region of (h(u) Wp) / d_out(u)
 * (16 wide) -> o = h wo + bo; xhat(v, j) = ||q_offset(:, j)||_1 o(v, j).
 * Parameters are one float32 vector in the order
 *   W0[16x64] b0[64] {Wp[64x16] Ws[64x64] Wm[16x64] b[64]} x 3 wo[64] bo[1]
 * (row-major).  Products run on the matrix cores with bfloat16 operands and
 * float32 accumulation; everything else in float32.
 * ------------------------------------------------------------------- */

/* Number of float32 parameters of the network (19777). */
int64_t rwr_gnn_num_params(void);

/* Set (copy from host) or read the context's network parameters.  Setting
 * resets the optimiser state.  The first call allocates the warm-start
 * buffers (capacity 2^21 rows unless rwr_warm_start chose another). */
rwr_status rwr_model_set(rwr_ctx *ctx, const float *params, int64_t n);
rwr_status rwr_model_get(rwr_ctx *ctx, float *params, int64_t cap);

/* Training options of the network: mask (rwr_gnn_num_params() floats, or
 * NULL for every parameter) marks the parameters the optimiser steps (1) and
 * those it holds at their value (0); the first warmup_steps steps of AdamW
 * scale the step size linearly from lr / warmup_steps up to lr.  Copied; kept
 * across rwr_model_set.  RWR_EINVAL on a wrong count or a negative
 * warm-up. */
rwr_status rwr_model_trainable(rwr_ctx *ctx, const float *mask, int64_t n, int32_t warmup_steps);

/* Switch the warm start of rwr_update:
 *   mode 0: off;  1: predict (the update propagates the residual of the
 *   prediction in every seed column where ||rho||_1 < ||q_offset||_1, else
 *   the plain offset seed);  2: train (the update runs plainly; one AdamW
 *   step on this update's loss sum_j ||rho_j||_1 / sum_j ||q_j||_1, the L1
 *   distance of the prediction from the exact offset result measured
 *   through I - (1-c) B~^T, relative to the seed; its gradient follows the
 *   correction below);  3: predict and train (the step follows the
 *   prediction of this update).
 * Before the residual is formed, the prediction is corrected so that the
 * residual sums to zero (a residual with a non-zero sum decays only by
 * (1-c) per iteration).
 * hops (0..8): region = offset support plus the nodes within `hops`
 * out-hops; a level that would take the region past max_rows / S nodes is
 * left out (max_rows <= 0 selects 2^21 rows).  lr and weight_decay set
 * AdamW's step size and decoupled decay.  Needs parameters (rwr_model_set);
 * else RWR_ESTATE.  Scores stay those of Algorithm 1 in every mode. */
rwr_status rwr_warm_start(rwr_ctx *ctx, int32_t mode, int32_t hops, int64_t max_rows, float lr,
                          float weight_decay);

/* Read back what the warm start of the last rwr_update computed (for checking
 * it against a reference): the region's nodes in the network's row order
 * (caller ids; nodes[cap]), the hop of each from the offset support
 * (hops[cap]), the network output o and dL/do of the training loss (row =
 * region node * row_cols + seed column; cap * row_cols floats each, row_cols
 * = the seed count rounded up to a power of two, padding columns zero), and
 * the parameter gradient of that training step (rwr_gnn_num_params()
 * floats; the parameters have since taken the AdamW step).  *n_region = 0
 * when the last update ran no warm start.  Any output array may be NULL;
 * dout and grad need a training step in the last update (RWR_ESTATE), cap
 * must be at least *n_region (RWR_EINVAL). */
rwr_status rwr_warm_inspect(rwr_ctx *ctx, int32_t *nodes, int32_t *hops, float *o, float *dout, float *grad,
                            int64_t cap, int32_t *n_region, int32_t *row_cols);

/* Evaluate the network once on an explicit region of nR nodes and S columns
 * (host arrays): in-rows (in_off/in_len/in_adj, local ids, n_in entries) and
 * out-rows (out_off/out_len/out_adj, n_out entries) of the region graph,
 * dinv[nR] = 1/d_out of each node in the whole graph (0 for dead ends),
 * feats[nR*S*16] (row = node*S + column).  Writes out[nR*S] = o when out is
 * not NULL.  With target[nR*S] and active[S] (1: the column counts) it also
 * computes the Huber loss (delta 1e-3, mean over active columns of the sum
 * over rows) into *loss and its gradient into grad[rwr_gnn_num_params()],
 * and with params_after not NULL one AdamW step from zero moments
 * (lr 1e-3, betas 0.9/0.999, eps 1e-8, weight decay 1e-4).  For testing the
 * network against a reference; runs on the current device, allocates and
 * frees its own buffers.  RWR_EINVAL on malformed input (ids out of range,
 * rows past n_in/n_out); the message is rwr_last_error(NULL). */
rwr_status rwr_gnn_eval(const float *params, int32_t nR, int32_t S, const int32_t *in_off, const int32_t *in_len,
                        const int32_t *in_adj, int64_t n_in, const int32_t *out_off, const int32_t *out_len,
                        const int32_t *out_adj, int64_t n_out, const float *dinv, const float *feats,
                        const float *target, const int32_t *active, float *out, float *grad, double *loss,
                        float *params_after);

/* The same evaluation as rwr_gnn_eval, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops): it
 * allocates nothing, running in one fixed array of 24 MiB that each device
 * the library runs on holds from this function's first call on it until the
 * process ends.  Limits: nR * S <= 8192 rows and n_in, n_out <= 131072 edges
 * (RWR_EINVAL beyond them, message in rwr_last_error(NULL)).  stream: the
 * hipStream_t to run on (NULL: the default stream); the call is synchronous
 * on return.  Arguments, outputs and results as rwr_gnn_eval.  Every call on
 * a device shares that device's array: calls that overlap on one device race
 * and must be serialised by the caller. */
rwr_status rwr_gnn_eval_noalloc(const float *params, int32_t nR, int32_t S, const int32_t *in_off,
                                const int32_t *in_len, const int32_t *in_adj, int64_t n_in, const int32_t *out_off,
                                const int32_t *out_len, const int32_t *out_adj, int64_t n_out, const float *dinv,
                                const float *feats, const float *target, const int32_t *active, float *out,
                                float *grad, double *loss, float *params_after, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RWR_H_ */
