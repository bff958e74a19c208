// C ABI of the dynamic-RWR library: context management, the update pipeline
// (batch upload -> keys -> sort/segment -> validate -> offset seed -> apply ->
// propagation slots -> finish) and the error-budget bookkeeping with FP64
// residual refinement.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gnn.h"
#include "rwr.h"
#include "rwr_common.h"
#include "rwr_kernels.h"
#include "warm.h"

namespace {

std::string g_build_error;

struct Orientation {
  DevGraphView v{};
  int64_t e_cap = 0;
};

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

int next_pow2_cols(int n) {
  int s = 1;
  while (s < n) s <<= 1;
  return s;
}

// terms of the offset seed (old degrees of the touched rows plus the batch's
// keys) from which it is sorted and reduced instead of scattered atomically
constexpr int64_t SEED_SORT_MIN = 1 << 16;
constexpr int SEED_SORT_MIN_S = 32;
// batch keys from which rows above BIG_ROW entries get a workgroup each in
// the batch check and apply (smaller batches keep one launch per step)
constexpr int64_t BIG_BATCH = 256;

int bits_for(int64_t v) {
  int b = 1;
  while ((1ll << b) <= v) ++b;
  return b;
}

}  // namespace

struct rwr_ctx {
  rwr_config cfg{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  int32_t n = 0, n_cap = 0;
  int64_t m = 0;  // stored directed edges
  int32_t n_seeds = 0, S = 1;
  std::vector<int32_t> seeds_h;
  int32_t *seeds_d = nullptr;      // internal ids
  int32_t *perm = nullptr;         // external id -> internal id
  int32_t *inv = nullptr;          // internal id -> external id
  bool undirected = false, fp64 = false;
  Orientation g[2];
  double *r = nullptr, *ybuf = nullptr, *gbuf = nullptr;
  double *xres = nullptr;  // r / d_out, gathered by the residual sweep
  double *qvec = nullptr;  // seed vectors in internal ids (node-major), when built from vectors
  bool qmode = false;
  void *x[2] = {nullptr, nullptr};
  int32_t *stamp = nullptr;
  int32_t *fstamp = nullptr;
  int32_t *nmark = nullptr;        // 1 on nodes that the current batch deletes (per node)
  int32_t *row_order = nullptr;    // light in-rows by descending in-degree (S >= 4)
  int64_t *ndel = nullptr;         // node deletions: entry counts, then key offsets
  int64_t ndel_cap = 0;
  int32_t *hfront = nullptr;
  int32_t *hbase = nullptr;
  Ctl *ctl = nullptr;
  Ctl *ctl_h = nullptr;  // pinned mirror
  double *hist = nullptr;
  int32_t max_iters = 10000;   // iteration guard of an update run
  int32_t solve_iters = 10000; // of a build or refinement run (at least Theorem 2's bound)
  bool rows_only = false;      // node deletion removes the row only
  bool det = false;            // no floating-point atomics on the score path
  // the offset seed's records (sort-and-reduce form): two key buffers of
  // srec_cap, the chunk partials, per-row old degrees and their prefix sum
  uint64_t *srec[2] = {nullptr, nullptr};
  double *spart = nullptr;
  int32_t *sdcnt = nullptr, *sroff = nullptr;
  int64_t srec_cap = 0;
  // rows above BIG_ROW entries handled by a workgroup each (batches of
  // BIG_BATCH keys or more): their lists
  int32_t *bigv = nullptr, *biga = nullptr;
  bool big_batch = false;
  int seed_sort_mode = -1;   // RWR_SEED_SORT: 1 always sort and reduce, 0 atomics (outside deterministic mode)
  bool seed_sorted = false;  // the last update's offset seed was sorted and reduced
  hipEvent_t ph_ev[7] = {};    // phase-timing events (created on first use)
  double *part = nullptr;
  int64_t *part_i = nullptr;
  int64_t part_blocks = 0;
  // heavy schedule of the pull orientation
  int32_t *h_item_row = nullptr, *h_item_chunk = nullptr, *h_rows = nullptr, *h_nchunks = nullptr, *h_first = nullptr;
  double *h_part = nullptr;
  int32_t h_items = 0, h_nrows = 0;
  int32_t heavy_limit = 512, heavy_chunk = 4096;
  int32_t fold_max = 2048;  // heavy row-columns finished inside the decision kernel
  int32_t *sel = nullptr, *sel_count = nullptr;
  // row partition of the single-column dense sweep
  int32_t *mp_rows = nullptr;
  int32_t n_mp = 0;
  // batch scratch
  int64_t bcap = 0;  // key capacity per orientation
  int32_t *b_dev = nullptr;
  int32_t *b_host = nullptr;
  int64_t b_host_cap = 0;
  uint64_t *keys[2] = {nullptr, nullptr};
  uint64_t *keys_alt = nullptr;
  int32_t *flags = nullptr, *pos = nullptr;
  int32_t *seg[2] = {nullptr, nullptr}, *row[2] = {nullptr, nullptr};
  int32_t *t_dold[2] = {nullptr, nullptr}, *t_dnew[2] = {nullptr, nullptr};
  void *temp = nullptr;
  size_t temp_bytes = 0;
  // tuning
  int32_t grid_sparse = 512, grid_light = 2048, grid_pull = 2048, light_lanes = 16, pull_lanes = 64;
  int32_t n_cu = 256;
  int32_t pull_ratio = 16;
  // error budget per seed column (normalised L1)
  double err_bound[RWR_MAX_COLS] = {};
  double budget = 0.0;
  double refine_target = 0.9;  // refinements aim at this fraction of the budget
  bool stale = false;
  std::string err;
  std::vector<double> last_hist;  // host copy of the last run's norms (made on request)
  bool hist_host_valid = false;
  int32_t last_iters = 0;
  double decay_ema = 0.8;  // observed per-iteration decay of ||x^(i)||_1
  // sparse and dense iterations of the recent update runs
  double sparse_ema = 1.0, dense_ema = 0.0;
  int32_t update_runs = 0;
  // Carried vectors.  A pending vector p (gbuf, per column) is part of r, and
  // r - p has residual p: the next update takes the offset seed of r - p and
  // adds p to its first dense sweep's input, so the run converges from an
  // exact residual and p's bound leaves the error bound.  Sources: the FP64
  // residual of a check that needed no refinement (checked early when the
  // next update would likely pass the budget), and the last iterate of an
  // update run that ended dense (left in x[tail_slot] instead of being
  // cleared; its truncation bound is then not spent).
  // carry_level: 0 off, 1 residual only, 2 residual and last iterate.
  int carry_level = 2;
  // columns of a run that may leave its last iterate retire together
  // (RWR_LOCKSTEP = 0: each at its own stop test)
  bool lockstep = true;
  // columns with a pending vector in gbuf; gbuf's other columns hold stale
  // values, and every reader takes gbuf only in the columns of pend
  uint64_t pend = 0;
  int tail_slot = -1;        // x buffer holding deferred last iterates (-1: none)
  uint64_t tail_cols = 0;    // their columns
  double pend_b[RWR_MAX_COLS] = {};   // error bound each pending (or deferred) vector carries
  double pend_l1[RWR_MAX_COLS] = {};  // its L1 norm
  double last_carry_l1 = 0.0;         // statistic of the last update
  double tail_ema = -1.0;    // recent per-update bound increments (max over columns)
  bool built = false;  // the static solve is done (update runs follow)
  // measurement: events around dense sweep launches
  bool prof_on = false;
  std::vector<hipEvent_t> prof_ev;
  int prof_used = 0;
  double prof_dense_ms = 0.0;
  int64_t prof_dense_sweeps = 0, prof_idle = 0;
  // sweep-shape tuning: the first dense sweeps of the build's static solve
  // rotate through candidate (lanes per row, workgroups) pairs, each timed
  // with events; the fastest by median is kept
  struct Tune {
    bool on = false;
    std::vector<std::pair<int32_t, int32_t>> cand;
    std::vector<std::vector<float>> ms;
    int reps = 3, launched = 0, limit = 0;
    std::vector<hipEvent_t> ev;
    std::vector<int> pending;  // candidate of each launch of the current chunk
    double best_ms = 0.0;
    bool cached = false;     // the shape came from the tuning cache
    std::string cache_path;  // where a finished tuning appends its line (empty: nowhere)
    std::string cache_key;
  } tune;
  // HIP graph of two consecutive dense iteration slots (an even and an odd
  // one: the kernels depend on the slot index only through its parity),
  // replayed for pairs of dense slots; captured again whenever the kernel
  // arguments change
  bool graphs = true;
  hipGraphExec_t pair_exec = nullptr;
  SlotArgs pair_args{};
  int64_t graph_replays = 0;
  // learned warm start (rwr_warm_start)
  struct Warm {
    int32_t mode = 0, hops = 3;
    int64_t max_rows = 0, max_nodes = 0;
    gnn::Net net;          // laid over net_mem (gnn::net_view)
    void *net_mem = nullptr;
    float *mask_d = nullptr;  // trainable-parameter mask on the device (null: all train)
    bool alloc = false, params = false;
    int32_t *hop1 = nullptr, *loc1 = nullptr, *wlist = nullptr, *flags = nullptr;
    int32_t *R = nullptr, *cnt = nullptr;  // cnt[0]: selected nodes, cnt[1]: touched nodes
    // the region's own edges in local ids (in-rows and out-rows)
    int32_t *lin_cnt = nullptr, *lin_off = nullptr, *lout_cnt = nullptr, *lout_off = nullptr;
    int32_t *lin_adj = nullptr, *lout_adj = nullptr;
    int32_t *items = nullptr, *item_off = nullptr;  // gradient work items over the region's out-rows
    int32_t *lin_items = nullptr, *lout_items = nullptr;  // aggregation work items
    int32_t n_in_items = 0, n_out_items = 0;
    double *gpart = nullptr;  // gradient item partials (one per item and column)
    int64_t gpart_cap = 0;
    int32_t *grow = nullptr;  // row of each gradient item (gpart_cap / S entries)
    int32_t *lin_item_row = nullptr, *lout_item_row = nullptr;  // row of each aggregation item
    int64_t item_row_cap = 0;
    // row items of the region search and of the local rows (two sets: in- and
    // out-rows); lv: the region's level table (see ws_region)
    int32_t *it_tmp[2] = {}, *it_rit[2] = {}, *it_irow[2] = {}, *it_icnt[2] = {}, *it_ioff[2] = {};
    int64_t items_cap = 0;
    int32_t *lv = nullptr;
    double *kpart = nullptr;  // per-workgroup partials of the correction's K
    double *fa = nullptr;     // f(|xhat|) per column
    int64_t ladj_cap = 0;
    void *scan_temp = nullptr;
    size_t scan_bytes = 0;
    float *dinv = nullptr;
    double *xhat = nullptr, *wbuf = nullptr, *qn = nullptr, *part = nullptr, *sums = nullptr;
    int8_t *sg = nullptr;     // signs of the residual (n_cap * S)
    double *pbuf = nullptr;   // the residual rho while it is formed (n_cap * S, zero at rest)
    int32_t out_items = 0;    // 1024-edge items of the region's out-rows (last update)
    bool pushed = false;      // the last update formed rho from the region alone
    void *temp = nullptr;
    size_t temp_bytes = 0;
    // this update
    int32_t nR = 0;
    std::vector<int32_t> level_end;  // end row of each hop level of the last region
    bool trained = false;            // the last update took a training step
    std::vector<float> mask_h;       // trainable-parameter mask (empty: all train)
    int32_t warmup = 0;              // step-size warm-up of the optimiser
    std::vector<double> qn_h;
    int32_t accepted = 0, fallback = 0;
    double ratio = 0.0, loss = 0.0, ms = 0.0;
    int push_mode = -1;  // RWR_WS_PUSH: 0 pull, 1 push, unset: by the region's out-edges
  } ws;
};

// ------------------------------------------------------------------ helpers
#define HIP_TRY(ctx, expr)                                                   \
  do {                                                                       \
    hipError_t _e = (expr);                                                  \
    if (_e != hipSuccess) {                                                  \
      (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(_e);        \
      return RWR_EHIP;                                                       \
    }                                                                        \
  } while (0)

#define RWR_TRY(expr)                  \
  do {                                 \
    rwr_status _s = (expr);            \
    if (_s != RWR_OK) return _s;       \
  } while (0)

// Device memory of a context: the caller's allocator when the configuration
// names one (frees are ordered on the context's stream, which every kernel of
// the context runs on), else hipMalloc / hipFree.
static rwr_status dev_alloc(rwr_ctx *c, void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  if (c->cfg.dev_alloc) {
    *p = c->cfg.dev_alloc(bytes, (void *)c->stream, c->cfg.alloc_user);
    if (!*p) {
      c->err = "dev_alloc(" + std::to_string(bytes) + " bytes) returned NULL";
      return RWR_ENOMEM;
    }
    return RWR_OK;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    c->err = "hipMalloc(" + std::to_string(bytes) + " bytes) failed: " + hipGetErrorString(e);
    *p = nullptr;
    return RWR_ENOMEM;
  }
  return RWR_OK;
}

static rwr_status copy_sync(rwr_ctx *c, void *dst, const void *src, size_t bytes, hipMemcpyKind kind) {
  if (bytes == 0) return RWR_OK;
  HIP_TRY(c, hipMemcpyAsync(dst, src, bytes, kind, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return RWR_OK;
}
#define H2D(c, dst, src, bytes) RWR_TRY(copy_sync((c), (dst), (src), (bytes), hipMemcpyHostToDevice))
#define D2H(c, dst, src, bytes) RWR_TRY(copy_sync((c), (dst), (src), (bytes), hipMemcpyDeviceToHost))

template <typename T>
static rwr_status alloc_zero(rwr_ctx *c, T **p, size_t count) {
  RWR_TRY(dev_alloc(c, (void **)p, sizeof(T) * count));
  launch_zero_bytes(*p, (sizeof(T) * count + 3) / 4 * 4, c->stream);
  return RWR_OK;
}

template <typename T>
static void dev_free(rwr_ctx *c, T *&p) {
  if (p) {
    if (c->cfg.dev_free)
      c->cfg.dev_free((void *)p, (void *)c->stream, c->cfg.alloc_user);
    else
      (void)hipFree((void *)p);
  }
  p = nullptr;
}

static rwr_status ensure_temp(rwr_ctx *c, size_t bytes) {
  if (bytes <= c->temp_bytes) return RWR_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  dev_free(c, c->temp);
  c->temp_bytes = 0;
  RWR_TRY(dev_alloc(c, &c->temp, bytes));
  c->temp_bytes = bytes;
  return RWR_OK;
}

// Timing events: without the system-scope fence an event's recording would
// otherwise add (a write-back and invalidation of the caches, which also slows
// the kernel after it); they are only read after a stream synchronisation.
static hipError_t timing_event(hipEvent_t *e) { return hipEventCreateWithFlags(e, hipEventDisableSystemFence); }

// the next pair of events (created on first use) that brackets one launch
// of the sweep kernel
static rwr_status prof_pair(rwr_ctx *c, hipEvent_t *e0, hipEvent_t *e1) {
  while (c->prof_used + 2 > (int)c->prof_ev.size()) {
    hipEvent_t e;
    HIP_TRY(c, timing_event(&e));
    c->prof_ev.push_back(e);
  }
  *e0 = c->prof_ev[c->prof_used++];
  *e1 = c->prof_ev[c->prof_used++];
  return RWR_OK;
}

// After a run: the first `real` of the `launched` sweep launches swept the
// graph (dense sweeps are contiguous); the rest found the run converged and
// returned at once.  All launches count towards the time.
static rwr_status prof_collect(rwr_ctx *c, int base, int launched, int real) {
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < launched; ++i) {
    float ms = 0.0f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->prof_ev[base + 2 * i], c->prof_ev[base + 2 * i + 1]));
    c->prof_dense_ms += ms;
    if (i < real)
      ++c->prof_dense_sweeps;
    else
      ++c->prof_idle;
  }
  c->prof_used = base;
  return RWR_OK;
}

static int pull_orient(const rwr_ctx *c) { return c->undirected ? 0 : 1; }

static SlotArgs slot_args(const rwr_ctx *c) {
  SlotArgs a{};
  a.out = c->g[0].v;
  a.in = c->g[pull_orient(c)].v;
  a.heavy.item_row = c->h_item_row;
  a.heavy.item_chunk = c->h_item_chunk;
  a.heavy.rows = c->h_rows;
  a.heavy.nchunks = c->h_nchunks;
  a.heavy.first = c->h_first;
  a.heavy.part = c->h_part;
  a.heavy.n_items = c->h_items;
  a.heavy.n_rows = c->h_nrows;
  a.heavy.chunk = c->heavy_chunk;
  a.r = c->r;
  a.ybuf = c->ybuf;
  a.gbuf = c->gbuf;
  a.xres = c->xres;
  a.x[0] = c->x[0];
  a.x[1] = c->x[1];
  a.stamp = c->stamp;
  a.fstamp = c->fstamp;
  a.hfront = c->hfront;
  a.hbase = c->hbase;
  a.seeds = c->seeds_d;
  a.ctl = c->ctl;
  a.hist = c->hist;
  a.part = c->part;
  a.part_i = c->part_i;
  a.n = c->n;
  a.n_seeds = c->n_seeds;
  a.c = c->cfg.c;
  a.grid_sparse = c->grid_sparse;
  a.grid_light = c->grid_light;
  a.grid_pull = c->grid_pull;
  a.light_lanes = c->light_lanes;
  a.pull_lanes = c->pull_lanes;
  a.fold_max = c->fold_max;
  a.zero_seed_rows = c->qmode ? 0 : 1;
  a.qvec = c->qvec;
  a.row_order = c->row_order;
  a.n_order = c->n_cap;
  a.mp_rows = c->mp_rows;
  a.n_mp = c->n_mp;
  return a;
}

static rwr_status read_ctl(rwr_ctx *c) {
  HIP_TRY(c, hipMemcpyAsync(c->ctl_h, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return RWR_OK;
}

// partial-sum buffers sized for the largest grid in use
static rwr_status ensure_partials(rwr_ctx *c) {
  // entries: the largest grid plus the heavy-row kernel's workgroups
  const int64_t blocks = std::max<int64_t>({c->grid_light, c->grid_sparse, c->grid_pull}) + HEAVY_EPI_MAX_GRID + 64;
  if (blocks <= c->part_blocks) return RWR_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  dev_free(c, c->part);
  dev_free(c, c->part_i);
  const int64_t stride = std::max(16, 2 * c->S);  // padded partial-sum entries
  RWR_TRY(alloc_zero(c, &c->part, (size_t)blocks * stride));
  RWR_TRY(alloc_zero(c, &c->part_i, (size_t)blocks * 16));
  c->part_blocks = blocks;
  return RWR_OK;
}

static void tune_defaults(rwr_ctx *c) {
  const int S = c->S;
  if (S == 1) {
    // wave items take rows of up to 1024 in-edges (two rounds); longer rows
    // are cut into 2048-edge chunks (fewer heavy rows to finish per sweep)
    c->light_lanes = 16;
    c->heavy_limit = 1024;
    c->heavy_chunk = 2048;
  } else if (S <= 4) {
    c->heavy_limit = 512;
    c->heavy_chunk = 2048;
  } else if (S <= 16) {
    c->heavy_limit = 256;
    c->heavy_chunk = 2048;
  } else {
    c->heavy_limit = 128;
    c->heavy_chunk = 2048;
  }
  c->pull_lanes = 16;
  if (const char *e = getenv("RWR_LIGHT_LANES")) c->light_lanes = atoi(e);
  if (const char *e = getenv("RWR_PULL_LANES")) c->pull_lanes = atoi(e);
  if (const char *e = getenv("RWR_HEAVY_LIMIT")) c->heavy_limit = atoi(e);
  if (const char *e = getenv("RWR_HEAVY_CHUNK")) c->heavy_chunk = atoi(e);
  if (const char *e = getenv("RWR_PULL_RATIO")) c->pull_ratio = atoi(e);
  if (const char *e = getenv("RWR_GRAPHS")) c->graphs = atoi(e) != 0;
  if (const char *e = getenv("RWR_HEAVY_FOLD")) c->fold_max = atoi(e);
  if (const char *e = getenv("RWR_CARRY")) c->carry_level = std::max(0, std::min(2, atoi(e)));
  if (const char *e = getenv("RWR_LOCKSTEP")) c->lockstep = atoi(e) != 0;
  if (const char *e = getenv("RWR_WS_PUSH")) c->ws.push_mode = atoi(e) != 0 ? 1 : 0;
  if (const char *e = getenv("RWR_SEED_SORT")) c->seed_sort_mode = atoi(e) != 0 ? 1 : 0;
  if (const char *e = getenv("RWR_REFINE_TARGET")) {
    const double t = atof(e);
    if (t > 0.0 && t < 1.0) c->refine_target = t;
  }
  if (c->cfg.pull_ratio > 0) c->pull_ratio = c->cfg.pull_ratio;
  // grids sized to the resident capacity: workgroups loop over their work
  c->grid_light = 4 * c->n_cu;
  c->grid_sparse = 4 * c->n_cu;
  // dense sweeps: the workgroups that fit on the chip at once (registers:
  // and LDS: five per CU for both the single-column and the vector sweep)
  c->grid_pull = (S == 1 ? 6 : S == 2 ? 8 : 5) * c->n_cu;
  if (const char *e = getenv("RWR_GRID_LIGHT")) c->grid_light = atoi(e);
  if (const char *e = getenv("RWR_GRID_SPARSE")) c->grid_sparse = atoi(e);
  if (const char *e = getenv("RWR_GRID_PULL")) c->grid_pull = atoi(e);
}

// Row partition of the single-column dense sweep over all n_cap rows (rows
// beyond n are empty): consecutive rows, at most WV_ROWS per wavefront item
// and about WV_EDGES light in-edges (rows above the heavy limit count as
// empty).
static rwr_status plan_partition(rwr_ctx *c) {
  Orientation &o = c->g[pull_orient(c)];
  std::vector<int32_t> len(c->n_cap);
  D2H(c, len.data(), o.v.len, sizeof(int32_t) * c->n_cap);
  std::vector<int32_t> rows;
  rows.reserve(c->n_cap / 64 + 2);
  rows.push_back(0);
  int64_t acc = 0;
  int cnt = 0;
  const int max_rows = WV_ROWS;
  const int64_t max_edges = WV_EDGES;
  for (int32_t v = 0; v < c->n_cap; ++v) {
    const int64_t l = len[v] > c->heavy_limit ? 0 : len[v];
    if (cnt > 0 && (cnt == max_rows || acc + l > max_edges)) {
      rows.push_back(v);
      acc = 0;
      cnt = 0;
    }
    acc += l;
    ++cnt;
  }
  rows.push_back(c->n_cap);
  dev_free(c, c->mp_rows);
  RWR_TRY(dev_alloc(c, (void **)&c->mp_rows, sizeof(int32_t) * rows.size()));
  H2D(c, c->mp_rows, rows.data(), sizeof(int32_t) * rows.size());
  c->n_mp = (int32_t)rows.size() - 1;
  return RWR_OK;
}

// Heavy rows of the pull orientation: flag them, split them into chunks.
// Order of the light in-rows for the multi-column sweep: every row once,
// by descending in-degree, so that the row groups sharing a wavefront get
// rows of about equal length.  Any permutation is correct; the order is
// renewed only when the node capacity changes.
static rwr_status plan_order(rwr_ctx *c) {
  Orientation &o = c->g[pull_orient(c)];
  std::vector<int32_t> len(c->n_cap);
  D2H(c, len.data(), o.v.len, sizeof(int32_t) * c->n_cap);
  const int32_t top = std::max(1, c->heavy_limit) + 1;
  std::vector<int64_t> start(top + 1, 0);
  for (int32_t v = 0; v < c->n_cap; ++v) ++start[top - std::min(len[v], top)];
  int64_t acc = 0;
  for (int32_t b = 0; b <= top; ++b) {
    const int64_t t = start[b];
    start[b] = acc;
    acc += t;
  }
  std::vector<int32_t> order(c->n_cap);
  for (int32_t v = 0; v < c->n_cap; ++v) order[start[top - std::min(len[v], top)]++] = v;
  dev_free(c, c->row_order);
  RWR_TRY(alloc_zero(c, &c->row_order, c->n_cap));
  H2D(c, c->row_order, order.data(), sizeof(int32_t) * c->n_cap);
  return RWR_OK;
}

static rwr_status plan_heavy(rwr_ctx *c, bool with_order = false) {
  Orientation &o = c->g[pull_orient(c)];
  HIP_TRY(c, hipMemsetAsync(c->sel_count, 0, sizeof(int32_t), c->stream));
  launch_mark_heavy(o.v.len, c->n, c->heavy_limit, o.v.heavy, c->sel, c->sel_count, c->stream);
  int32_t count = 0;
  HIP_TRY(c, hipMemcpyAsync(&count, c->sel_count, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::vector<int32_t> rows(count), lens(count);
  if (count > 0) {
    D2H(c, rows.data(), c->sel, sizeof(int32_t) * count);
    std::sort(rows.begin(), rows.end());
    H2D(c, c->sel, rows.data(), sizeof(int32_t) * count);
    launch_gather_i32(o.v.len, c->sel, count, c->sel + c->n_cap, c->stream);
    HIP_TRY(c, hipMemcpyAsync(lens.data(), c->sel + c->n_cap, sizeof(int32_t) * count, hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  std::vector<int32_t> item_row, item_chunk, nchunks(count), first(count);
  for (int32_t h = 0; h < count; ++h) {
    const int64_t planned = (int64_t)lens[h] + lens[h] / 4;
    const int32_t nch = (int32_t)std::max<int64_t>(1, (planned + c->heavy_chunk - 1) / c->heavy_chunk);
    nchunks[h] = nch;
    first[h] = (int32_t)item_row.size();
    for (int32_t k = 0; k < nch; ++k) {
      item_row.push_back(h);
      item_chunk.push_back(k);
    }
  }
  dev_free(c, c->h_item_row);
  dev_free(c, c->h_item_chunk);
  dev_free(c, c->h_rows);
  dev_free(c, c->h_nchunks);
  dev_free(c, c->h_first);
  dev_free(c, c->h_part);
  const int32_t items = (int32_t)item_row.size();
  RWR_TRY(alloc_zero(c, &c->h_item_row, std::max(1, items)));
  RWR_TRY(alloc_zero(c, &c->h_item_chunk, std::max(1, items)));
  RWR_TRY(alloc_zero(c, &c->h_rows, std::max(1, count)));
  RWR_TRY(alloc_zero(c, &c->h_nchunks, std::max(1, count)));
  RWR_TRY(alloc_zero(c, &c->h_first, std::max(1, count)));
  RWR_TRY(alloc_zero(c, &c->h_part, (size_t)std::max(1, items) * c->S));
  if (items > 0) {
    H2D(c, c->h_item_row, item_row.data(), sizeof(int32_t) * items);
    H2D(c, c->h_item_chunk, item_chunk.data(), sizeof(int32_t) * items);
    H2D(c, c->h_rows, rows.data(), sizeof(int32_t) * count);
    H2D(c, c->h_nchunks, nchunks.data(), sizeof(int32_t) * count);
    H2D(c, c->h_first, first.data(), sizeof(int32_t) * count);
  }
  c->h_items = items;
  c->h_nrows = count;
  if (c->S == 1) RWR_TRY(plan_partition(c));
  if (c->S >= 4 && (with_order || !c->row_order)) RWR_TRY(plan_order(c));
  return ensure_partials(c);
}

// Grow every per-node array to hold at least `need` nodes.
static rwr_status grow_nodes(rwr_ctx *c, int32_t need) {
  if (need <= c->n_cap) return RWR_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int32_t old_cap = c->n_cap;
  const int64_t want = std::max<int64_t>((int64_t)need + need / 8 + 1024, (int64_t)old_cap * 3 / 2);
  if (want >= INT32_MAX) {
    c->err = "node capacity overflow";
    return RWR_EINVAL;
  }
  const int32_t new_cap = (int32_t)want;
  auto regrow = [&](void **p, size_t elem, size_t per_node) -> rwr_status {
    void *np = nullptr;
    RWR_TRY(dev_alloc(c, &np, elem * per_node * new_cap));
    launch_zero_bytes(np, (elem * per_node * new_cap + 3) / 4 * 4, c->stream);
    if (*p) {
      hipError_t e = hipMemcpyAsync(np, *p, elem * per_node * old_cap, hipMemcpyDeviceToDevice, c->stream);
      if (e != hipSuccess) {
        c->err = hipGetErrorString(e);
        return RWR_EHIP;
      }
      (void)hipStreamSynchronize(c->stream);
      dev_free(c, *p);
    }
    *p = np;
    return RWR_OK;
  };
  const int no = c->undirected ? 1 : 2;
  for (int o = 0; o < no; ++o) {
    RWR_TRY(regrow((void **)&c->g[o].v.off, 4, 1));
    RWR_TRY(regrow((void **)&c->g[o].v.len, 4, 1));
    RWR_TRY(regrow((void **)&c->g[o].v.cap, 4, 1));
    RWR_TRY(regrow((void **)&c->g[o].v.heavy, 1, 1));
  }
  if (c->undirected) c->g[1] = c->g[0];
  const size_t xs = c->fp64 ? 8 : 4;
  RWR_TRY(regrow((void **)&c->r, 8, c->S));
  RWR_TRY(regrow((void **)&c->ybuf, 8, c->S));
  RWR_TRY(regrow((void **)&c->gbuf, 8, c->S));
  RWR_TRY(regrow((void **)&c->xres, 8, c->S));
  if (c->qmode) RWR_TRY(regrow((void **)&c->qvec, 8, c->S));
  RWR_TRY(regrow(&c->x[0], xs, c->S));
  RWR_TRY(regrow(&c->x[1], xs, c->S));
  RWR_TRY(regrow((void **)&c->stamp, 4, 1));
  RWR_TRY(regrow((void **)&c->fstamp, 4, 1));
  RWR_TRY(regrow((void **)&c->nmark, 4, 1));
  RWR_TRY(regrow((void **)&c->hfront, 4, 1));
  RWR_TRY(regrow((void **)&c->hbase, 4, 1));
  RWR_TRY(regrow((void **)&c->sel, 4, 2));
  RWR_TRY(regrow((void **)&c->perm, 4, 1));
  RWR_TRY(regrow((void **)&c->inv, 4, 1));
  launch_identity(c->perm, c->inv, old_cap, new_cap, c->stream);
  if (c->ws.alloc) {
    RWR_TRY(regrow((void **)&c->ws.hop1, 4, 1));
    RWR_TRY(regrow((void **)&c->ws.loc1, 4, 1));
    RWR_TRY(regrow((void **)&c->ws.wlist, 4, 1));
    RWR_TRY(regrow((void **)&c->ws.flags, 4, 1));
    RWR_TRY(regrow((void **)&c->ws.wbuf, 8, c->S));
    RWR_TRY(regrow((void **)&c->ws.sg, 1, c->S));
    RWR_TRY(regrow((void **)&c->ws.pbuf, 8, c->S));
    const size_t tb = ws_select_temp_bytes(new_cap);
    if (tb > c->ws.temp_bytes) {
      dev_free(c, c->ws.temp);
      c->ws.temp = nullptr;
      RWR_TRY(dev_alloc(c, &c->ws.temp, tb));
      c->ws.temp_bytes = tb;
    }
  }
  c->n_cap = new_cap;
  RWR_TRY(plan_heavy(c, true));
  RWR_TRY(ensure_partials(c));
  return RWR_OK;
}

// Move orientation o to a fresh layout with slack on every row and an arena of
// at least `arena_min` slots.
static rwr_status relayout(rwr_ctx *c, int o, int64_t arena_min) {
  Orientation &g = c->g[o];
  int32_t *new_off = nullptr, *new_capv = nullptr, *new_adj = nullptr;
  RWR_TRY(dev_alloc(c, (void **)&new_off, sizeof(int32_t) * c->n_cap));
  RWR_TRY(dev_alloc(c, (void **)&new_capv, sizeof(int32_t) * c->n_cap));
  launch_fill_i32(new_off, c->n_cap, 0, c->stream);
  launch_fill_i32(new_capv, c->n_cap, 0, c->stream);
  RWR_TRY(ensure_temp(c, build_temp_bytes(1, c->n_cap)));
  int64_t used = 0;
  HIP_TRY(c, relayout_offsets(g.v.len, c->n, new_capv, new_off, c->temp, c->temp_bytes, &used, c->stream));
  const int64_t arena = std::max<int64_t>({used / 4, arena_min, 65536});
  const int64_t e_cap = used + arena;
  if (e_cap >= INT32_MAX) {
    c->err = "adjacency capacity exceeds 2^31 slots";
    return RWR_ENOMEM;
  }
  RWR_TRY(dev_alloc(c, (void **)&new_adj, sizeof(int32_t) * e_cap));
  launch_copy_rows(g.v, new_off, new_adj, c->n, c->stream);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  dev_free(c, g.v.adj);
  dev_free(c, g.v.off);
  dev_free(c, g.v.cap);
  g.v.adj = new_adj;
  g.v.off = new_off;
  g.v.cap = new_capv;
  g.e_cap = e_cap;
  uint64_t tail = (uint64_t)used;
  H2D(c, &c->ctl->tail[o], &tail, sizeof(tail));
  if (c->undirected) c->g[1] = c->g[0];
  return RWR_OK;
}

// Build orientation o from rows/cols (device arrays of m entries).
static rwr_status build_orient(rwr_ctx *c, int o, const int32_t *rows, const int32_t *cols, int64_t m) {
  Orientation &g = c->g[o];
  RWR_TRY(alloc_zero(c, &g.v.off, c->n_cap));
  RWR_TRY(alloc_zero(c, &g.v.len, c->n_cap));
  RWR_TRY(alloc_zero(c, &g.v.cap, c->n_cap));
  RWR_TRY(alloc_zero(c, &g.v.heavy, c->n_cap));
  uint64_t *keys = nullptr, *keys_alt = nullptr;
  int32_t *sstart = nullptr;
  RWR_TRY(dev_alloc(c, (void **)&keys, sizeof(uint64_t) * std::max<int64_t>(1, m)));
  RWR_TRY(dev_alloc(c, (void **)&keys_alt, sizeof(uint64_t) * std::max<int64_t>(1, m)));
  RWR_TRY(dev_alloc(c, (void **)&sstart, sizeof(int32_t) * c->n_cap));
  RWR_TRY(ensure_temp(c, build_temp_bytes(std::max<int64_t>(1, m), c->n_cap)));
  int64_t used = 0;
  // rows beyond n are empty; build over all n_cap rows so offsets are defined
  HIP_TRY(c, build_phase1(rows, cols, m, c->n, g.v, c->temp, c->temp_bytes, keys, keys_alt, sstart, c->ctl, &used,
                          c->stream));
  RWR_TRY(read_ctl(c));
  if (c->ctl_h->err != 0) {
    dev_free(c, keys);
    dev_free(c, keys_alt);
    dev_free(c, sstart);
    c->err = "edge list has an id out of range or a repeated edge";
    return RWR_EINVAL;
  }
  const int64_t arena = std::max<int64_t>(used / 4, 65536);
  g.e_cap = used + arena;
  if (g.e_cap >= INT32_MAX) {
    c->err = "adjacency capacity exceeds 2^31 slots";
    return RWR_ENOMEM;
  }
  RWR_TRY(alloc_zero(c, &g.v.adj, g.e_cap));
  build_phase2(keys, m, g.v, sstart, c->stream);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  dev_free(c, keys);
  dev_free(c, keys_alt);
  dev_free(c, sstart);
  uint64_t tail = (uint64_t)used;
  H2D(c, &c->ctl->tail[o], &tail, sizeof(tail));
  return RWR_OK;
}

static void tune_begin(rwr_ctx *c) {
  rwr_ctx::Tune &t = c->tune;
  t.cand.clear();
  const int cu = c->n_cu;
  if (c->S == 1) {
    for (int g : {4, 5, 6}) t.cand.push_back({c->pull_lanes, g * cu});
  } else if (c->S == 2) {
    for (int g : {4, 6, 8}) t.cand.push_back({c->pull_lanes, g * cu});
  } else {
    for (int l : {16, 32, 64})
      for (int g : {5, 6, 7}) t.cand.push_back({l, g * cu});
  }
  t.ms.assign(t.cand.size(), {});
  t.launched = 0;
  t.limit = 4 * t.reps * (int)t.cand.size();
  t.on = true;
}

// Tuning cache (environment RWR_TUNE_CACHE = a text file): one line per
// tuned workload, "key lanes workgroups ms", the key naming the device
// (architecture and compute units), n, m, S, the propagation precision and
// a hash of the pull orientation's degree histogram (log2 buckets).  A build
// whose key is listed takes the listed shape instead of tuning.
static rwr_status tune_key(rwr_ctx *c, std::string *key) {
  hipDeviceProp_t prop{};
  HIP_TRY(c, hipGetDeviceProperties(&prop, c->device));
  std::vector<int32_t> len(c->n);
  D2H(c, len.data(), c->g[pull_orient(c)].v.len, sizeof(int32_t) * c->n);
  uint64_t hist[33] = {};
  for (int32_t d : len) {
    int b = 0;
    while (b < 32 && (1ll << b) <= d) ++b;
    ++hist[b];
  }
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the histogram counts
  for (uint64_t x : hist)
    for (int k = 0; k < 8; ++k) {
      h ^= (x >> (8 * k)) & 0xffu;
      h *= 1099511628211ull;
    }
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s/cu%d/n%d/m%lld/S%d/fp%d/deg%016llx", prop.gcnArchName, c->n_cu, c->n,
                (long long)c->m, c->S, c->fp64 ? 64 : 32, (unsigned long long)h);
  for (char *p = buf; *p; ++p)
    if (*p == ' ') *p = '_';
  *key = buf;
  return RWR_OK;
}

static bool tune_cache_find(const char *path, const std::string &key, int32_t *lanes, int32_t *grid, double *ms) {
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  char k[256];
  int l = 0, g = 0;
  double t = 0.0;
  bool found = false;
  while (std::fscanf(f, "%255s %d %d %lf", k, &l, &g, &t) == 4)
    if (key == k && l > 0 && g > 0) {
      *lanes = l;
      *grid = g;
      *ms = t;
      found = true;  // the last entry for the key wins
    }
  std::fclose(f);
  return found;
}

static void tune_cache_store(const char *path, const std::string &key, int32_t lanes, int32_t grid, double ms) {
  FILE *f = std::fopen(path, "a");
  if (!f) return;  // the cache is an optimisation: a read-only location only costs the tuning
  std::fprintf(f, "%s %d %d %.6f\n", key.c_str(), lanes, grid, ms);
  std::fclose(f);
}

static bool tune_done(const rwr_ctx::Tune &t) {
  for (const auto &v : t.ms)
    if ((int)v.size() < t.reps) return false;
  return true;
}

static void tune_finish(rwr_ctx *c) {
  rwr_ctx::Tune &t = c->tune;
  t.on = false;
  int best = -1;
  float bms = 0.0f;
  for (size_t i = 0; i < t.cand.size(); ++i) {
    std::vector<float> v = t.ms[i];
    if (v.empty()) continue;
    std::sort(v.begin(), v.end());
    const float med = v[v.size() / 2];
    if (best < 0 || med < bms) best = (int)i, bms = med;
  }
  if (best >= 0) {
    c->pull_lanes = t.cand[best].first;
    c->grid_pull = t.cand[best].second;
    t.best_ms = bms;
    if (!t.cache_path.empty()) tune_cache_store(t.cache_path.c_str(), t.cache_key, c->pull_lanes, c->grid_pull, bms);
  }
  t.cache_path.clear();
}

static void pair_graph_drop(rwr_ctx *c) {
  if (c->pair_exec) (void)hipGraphExecDestroy(c->pair_exec);
  c->pair_exec = nullptr;
}

// the pair graph for arguments a (captured on first use or when a changed)
static rwr_status pair_graph(rwr_ctx *c, const SlotArgs &a) {
  if (c->pair_exec && std::memcmp(&c->pair_args, &a, sizeof(SlotArgs)) == 0) return RWR_OK;
  pair_graph_drop(c);
  hipGraph_t g = nullptr;
  HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  launch_dense_slot(a, c->S, c->fp64, 2, c->stream);
  launch_dense_slot(a, c->S, c->fp64, 3, c->stream);
  const hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (e != hipSuccess || !g) {
    c->err = std::string("graph capture failed: ") + hipGetErrorString(e);
    return RWR_EHIP;
  }
  const hipError_t ei = hipGraphInstantiate(&c->pair_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    c->pair_exec = nullptr;
    c->err = std::string("graph instantiation failed: ") + hipGetErrorString(ei);
    return RWR_EHIP;
  }
  c->pair_args = a;
  return RWR_OK;
}

// Enqueue iteration slots until the device reports MODE_DONE.  The slot that
// computes x^(0) must already be enqueued; `mode` is the phase it leaves
// (sparse after an offset seed or a seed vector, dense after a residual).
// Only the kernels of the current phase are launched; the phase is re-read
// at every synchronisation (a switch mid-chunk turns the chunk's remaining
// sparse slots into no-ops, and the next chunk starts at the device's count).
static rwr_status run_slots(rwr_ctx *c, int mode, double init_norm = -1.0, double eps_hint = 0.0,
                           bool keep_tail = false, uint64_t inject = 0, int guard = -1) {
  const int max_it = guard > 0 ? guard : c->max_iters;
  const SlotArgs a = slot_args(c);
  int k = 1;
  // first chunk: predicted from the starting norm when it is known (a
  // refinement), else a few sparse slots
  int chunk = 3;
  if (init_norm > 0.0 && eps_hint > 0.0 && init_norm > eps_hint)
    chunk = std::max(1, std::min(64, (int)std::ceil(std::log(eps_hint / init_norm) / std::log(c->decay_ema))));
  // an update run: the first chunk holds the sparse slots recent update runs
  // needed.  (Enqueueing their predicted dense slots behind them as well, which
  // the slot guards allow, cost more in idle launches whenever a run stayed
  // sparse one slot longer than predicted than the host round trip it saved.)
  rwr_ctx::Tune &tn0 = c->tune;
  const bool update_run = mode == MODE_SPARSE && init_norm < 0.0 && c->built && !tn0.on;
  const int sparse_end = 1 << 30;
  if (update_run && c->update_runs >= 2) chunk = std::max(1, std::min(16, (int)std::lround(c->sparse_ema)));
  double prev = -1.0;
  int prev_iter = 0;
  int dense_launched = 0, dense_base = c->prof_used;
  rwr_ctx::Tune &tn = c->tune;
  while (true) {
    const int dense_before = c->ctl_h->dense_iters;
    tn.pending.clear();
    if (k > max_it + 1) {
      c->err = "iteration slots exhausted without completion";
      return RWR_EHIP;
    }
    const int kend = std::min(k + chunk, max_it + 2);
    for (; k < kend; ++k) {
      if (mode == MODE_DENSE || k >= sparse_end) {
        if (inject) {
          // pending vectors join the first dense sweep's input
          launch_inject(a, c->S, c->fp64, k, inject, c->stream);
          inject = 0;
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (tn.on && tn.launched < tn.limit) {
          // a tuning launch: the next candidate shape, timed
          const int ci = tn.launched++ % (int)tn.cand.size();
          const size_t q = 2 * tn.pending.size();
          while (tn.ev.size() < q + 2) {
            hipEvent_t e;
            HIP_TRY(c, timing_event(&e));
            tn.ev.push_back(e);
          }
          tn.pending.push_back(ci);
          SlotArgs at = a;
          at.pull_lanes = tn.cand[ci].first;
          at.grid_pull = tn.cand[ci].second;
          launch_dense_slot(at, c->S, c->fp64, k, c->stream, tn.ev[q], tn.ev[q + 1]);
        } else if (c->graphs && !c->prof_on && (k & 1) == 0 && k + 1 < kend) {
          // two dense slots (k even, k + 1) from the captured graph
          RWR_TRY(pair_graph(c, a));
          HIP_TRY(c, hipGraphLaunch(c->pair_exec, c->stream));
          ++c->graph_replays;
          ++k;
        } else {
          if (c->prof_on) RWR_TRY(prof_pair(c, &e0, &e1));
          launch_dense_slot(a, c->S, c->fp64, k, c->stream, e0, e1);
          ++dense_launched;
        }
      } else {
        launch_sparse_slot(a, c->S, c->fp64, k, c->stream);
      }
    }
    RWR_TRY(read_ctl(c));
    const Ctl &h = *c->ctl_h;
    if (!tn.pending.empty()) {
      // the first `real` tuning launches of the chunk swept; the rest were idle
      const int real = std::max(0, h.dense_iters - dense_before);
      for (int i = 0; i < (int)tn.pending.size() && i < real; ++i) {
        float ms = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&ms, tn.ev[2 * i], tn.ev[2 * i + 1]));
        tn.ms[tn.pending[i]].push_back(ms);
      }
      tn.pending.clear();
      if (tune_done(tn) || tn.launched >= tn.limit) tune_finish(c);
    }
    if (h.mode == MODE_DONE) break;
    mode = h.mode;
    k = h.iter;
    // predict the remaining iterations from the observed decay
    double cur = 0.0;
    for (int j = 0; j < c->n_seeds; ++j)
      if (h.active[j]) cur = std::max(cur, h.last_norm[j]);
    double decay = c->decay_ema;
    if (prev > 0.0 && cur > 0.0 && h.iter > prev_iter) {
      decay = std::pow(cur / prev, 1.0 / (h.iter - prev_iter));
      decay = std::min(std::max(decay, 0.3), 0.95);
    }
    int rem = 1;
    if (cur > h.eps && cur > 0.0) rem = std::max(1, (int)std::ceil(std::log(h.eps / cur) / std::log(decay)));
    chunk = mode == MODE_DENSE ? std::min(rem, 64) : std::max(2, std::min(rem, 16));
    prev = cur;
    prev_iter = h.iter;
  }
  if (c->prof_on) RWR_TRY(prof_collect(c, dense_base, dense_launched, c->ctl_h->dense_iters));
  if (update_run) {
    const Ctl &h = *c->ctl_h;
    const int dense = h.dense_iters, sparse = std::max(0, h.iter - 1 - dense);
    if (c->update_runs == 0) {
      c->sparse_ema = sparse;
      c->dense_ema = dense;
    } else {
      c->sparse_ema = 0.8 * c->sparse_ema + 0.2 * sparse;
      c->dense_ema = 0.8 * c->dense_ema + 0.2 * dense;
    }
    ++c->update_runs;
  }
  // a run that ended dense may leave its last iterate for the next update
  if (keep_tail && c->ctl_h->ended_dense && c->ctl_h->prop_err == 0) {
    c->tail_slot = (c->ctl_h->iter - 1) & 1;
    c->tail_cols = 0;
    for (int j = 0; j < c->n_seeds; ++j)
      if (c->ctl_h->last_it[j] == c->ctl_h->iter - 1) c->tail_cols |= 1ull << j;
    return RWR_OK;
  }
  launch_finish(a, c->S, c->fp64, c->stream);
  return RWR_OK;
}

static uint64_t all_cols_mask(int n_seeds) { return n_seeds >= 64 ? ~0ull : ((1ull << n_seeds) - 1ull); }

// frontier edges above which a run leaves the sparse push for dense pull
// sweeps; -1 (deterministic): dense from the first iteration, since the push
// scatters with floating-point atomics
static int64_t dense_thresh(const rwr_ctx *c) {
  if (c->det) return -1;
  return std::max<int64_t>(1, c->m / std::max(1, c->pull_ratio));
}

static double fp32_factor(const rwr_ctx *c) { return c->fp64 ? 0.0 : 8.0 * std::ldexp(1.0, -24); }

// Give up every carried vector (before a residual check, which supersedes
// them, or the learned warm start): each one's bound stays in the error bound
// (r - p has residual p, so r is within that bound), and the x buffers are
// cleared (every other run starts from zero buffers).
static void drop_carry(rwr_ctx *c) {
  if (c->tail_slot >= 0) {
    const size_t bytes = (size_t)c->n_cap * c->S * (c->fp64 ? 8 : 4);
    launch_zero_bytes(c->x[0], bytes, c->stream);
    launch_zero_bytes(c->x[1], bytes, c->stream);
  }
  c->tail_slot = -1;
  c->tail_cols = 0;
  c->pend = 0;
  for (int j = 0; j < RWR_MAX_COLS; ++j) c->pend_b[j] = 0.0;
}

// bookkeeping after a propagation run: per-column bound increments; returns
// the largest increment.  `reset`: the run started from exact scores (the
// bound restarts); `inj`: columns whose pending vector joined the run (its
// bound is replaced by the run's).  A column whose last iterate the run
// deferred records that iterate's bound and norm.
static double account_run(rwr_ctx *c, bool reset, uint64_t inj = 0) {
  const Ctl &h = *c->ctl_h;
  const int iters = std::max(0, h.iter - 1);
  c->last_iters = iters;
  c->hist_host_valid = false;
  const double cc = c->cfg.c;
  const int k0 = h.last_it[0];
  if (k0 >= 3) {
    // per-iteration decay between iteration 1 and column 0's last one
    const double n1 = h.norm1[0], nk = h.last_norm[0];
    if (n1 > 0.0 && nk > 0.0) {
      const double d = std::pow(nk / n1, 1.0 / (k0 - 1));
      if (d > 0.2 && d < 0.99) c->decay_ema = 0.8 * c->decay_ema + 0.2 * d;
    }
  }
  double inc = 0.0;
  for (int j = 0; j < c->n_seeds; ++j) {
    const double sum_norms = h.sum_norm[j];
    const double sig = std::fabs(h.sigma[j]) > 0 ? std::fabs(h.sigma[j]) : 1.0;
    const double tail = 2.0 * (1.0 - cc) / cc * h.last_norm[j] / sig;
    const double rnd = 2.0 * fp32_factor(c) * sum_norms / (cc * sig);
    const bool took = (inj >> j) & 1ull;
    const double base = reset ? 0.0 : c->err_bound[j] - (took ? c->pend_b[j] : 0.0);
    c->err_bound[j] = base + tail + rnd;
    if (took) c->pend_b[j] = 0.0;
    if ((c->tail_cols >> j) & 1ull) {
      c->pend_b[j] = tail;
      c->pend_l1[j] = h.last_norm[j];
    }
    inc = std::max(inc, tail + rnd);
  }
  return inc;
}

// Keep every column's error bound within the budget.  The running bound is
// the sum of the per-update truncation bounds (Theorem 3 applied to each
// update, doubled for the rescaling) plus an estimate of FP32 rounding.  When
// it exceeds the budget, the FP64 residual g = P r - r (seed entries zeroed)
// is evaluated: it certifies ||r/sigma - r*/sigma*||_1 <= 2 ||g||_1 / (c sigma).
// Columns whose certified error is still above the budget are refined: g is
// propagated (r += sum_i P^i g) down to a fraction of the budget (0.9 in
// updates: the next check comes sooner, but each refinement is short, which
// costs fewer sweeps per update overall).  `force`
// evaluates the residual regardless of the running bound, and refines above
// `refine_at` (a fraction of the budget).
static rwr_status check_and_refine(rwr_ctx *c, bool force, rwr_stats *st, double refine_at = 1.0,
                                   double target = -1.0) {
  double worst = 0.0, next = 0.0;
  for (int j = 0; j < c->n_seeds; ++j) {
    worst = std::max(worst, c->err_bound[j]);
    // a carried vector's bound is replaced by the next run's
    next = std::max(next, c->err_bound[j] - c->pend_b[j]);
  }
  // the residual carry (updates only): check now when the next update would
  // likely pass the budget, and carry the residual into it
  const bool carry = !force && c->carry_level >= 1;
  if (!force && worst <= c->budget && !(carry && c->tail_ema > 0.0 && next + c->tail_ema > c->budget))
    return RWR_OK;
  drop_carry(c);  // the residual supersedes the carried vectors
  const SlotArgs a = slot_args(c);
  launch_residual(a, c->S, c->stream);
  RWR_TRY(read_ctl(c));
  const double cc = c->cfg.c;
  uint64_t mask = 0;
  double resid = 0.0;
  for (int j = 0; j < c->n_seeds; ++j) {
    const double sig = std::fabs(c->ctl_h->sigma[j]);
    const double g = c->ctl_h->red_norm[j];
    if (!std::isfinite(g) || !std::isfinite(sig)) {
      c->stale = true;
      c->err = "non-finite residual or score sum";
      return RWR_ENUMERIC;
    }
    resid = std::max(resid, g);
    const double cert = 2.0 * g / (cc * sig);
    c->err_bound[j] = cert;
    if (cert > refine_at * c->budget) mask |= 1ull << j;
  }
  if (st) {
    st->checked = 1;
    st->residual_l1 = resid;
  }
  if (mask == 0) {
    if (carry) {
      // keep g as a pending vector: r += g (then r - g has residual g) and
      // sigma exactly; the certificate still bounds r + g
      launch_add_resid(a, c->S, c->stream);
      launch_sigma_exact(a, c->S, c->stream);
      c->pend = all_cols_mask(c->n_seeds);
      for (int j = 0; j < c->n_seeds; ++j) {
        c->pend_b[j] = c->err_bound[j];
        c->pend_l1[j] = c->ctl_h->red_norm[j];
      }
    }
    return RWR_OK;
  }
  double min_sig = 1e300;
  for (int j = 0; j < c->n_seeds; ++j) min_sig = std::min(min_sig, std::fabs(c->ctl_h->sigma[j]));
  // truncation bound of the refinement: 2 (1-c)/c * eps_ref / sigma = target * budget
  const double tgt = target > 0.0 ? target : c->refine_target;
  const double eps_ref = tgt * c->budget * cc * min_sig / (2.0 * (1.0 - cc));
  // in a stream the refinement's last iterate is left for the next update too
  // (otherwise its truncation, near the budget, pushes the next update's
  // bound over it and the refinements follow one another); its columns then
  // retire together so that every one of them leaves its last iterate
  const bool keep = carry && c->carry_level >= 2;
  launch_reset_run(c->ctl, c->S, mask, eps_ref, c->solve_iters, dense_thresh(c), c->n / 16 + 1, c->stream,
                   c->max_iters + 2, keep && c->lockstep ? 1 : 0);
  launch_refine_init(a, c->S, c->fp64, c->stream);
  RWR_TRY(run_slots(c, MODE_DENSE, resid * (1.0 - cc), eps_ref, keep, 0, c->solve_iters));
  if (c->ctl_h->prop_err != 0) {
    c->stale = true;
    c->err = "refinement did not converge";
    return (rwr_status)c->ctl_h->prop_err;
  }
  const double fpf = fp32_factor(c);
  for (int j = 0; j < c->n_seeds; ++j) {
    if (!((mask >> j) & 1ull)) continue;
    const double sig = std::fabs(c->ctl_h->sigma[j]);
    // truncation of the refinement + FP32 rounding of propagating g
    const double tail = 2.0 * (1.0 - cc) / cc * c->ctl_h->last_norm[j] / sig;
    c->err_bound[j] = tail + 8.0 * fpf * c->ctl_h->red_norm[j] / (cc * sig);
    if ((c->tail_cols >> j) & 1ull) {
      c->pend_b[j] = tail;
      c->pend_l1[j] = c->ctl_h->last_norm[j];
    }
  }
  if (st) {
    st->refined = 1;
    st->flushed = __builtin_popcountll(mask);
  }
  return RWR_OK;
}

// ---------------------------------------------------------- warm start
static void warm_free(rwr_ctx *c) {
  rwr_ctx::Warm &w = c->ws;
  dev_free(c, w.hop1);
  dev_free(c, w.loc1);
  dev_free(c, w.wlist);
  dev_free(c, w.flags);
  dev_free(c, w.R);
  dev_free(c, w.cnt);
  dev_free(c, w.lin_cnt);
  dev_free(c, w.lin_off);
  dev_free(c, w.lout_cnt);
  dev_free(c, w.lout_off);
  dev_free(c, w.lin_adj);
  dev_free(c, w.lout_adj);
  dev_free(c, w.items);
  dev_free(c, w.item_off);
  dev_free(c, w.lin_items);
  dev_free(c, w.lout_items);
  dev_free(c, w.gpart);
  dev_free(c, w.grow);
  w.gpart_cap = 0;
  dev_free(c, w.lin_item_row);
  dev_free(c, w.lout_item_row);
  w.item_row_cap = 0;
  for (int k = 0; k < 2; ++k) {
    dev_free(c, w.it_tmp[k]);
    dev_free(c, w.it_rit[k]);
    dev_free(c, w.it_irow[k]);
    dev_free(c, w.it_icnt[k]);
    dev_free(c, w.it_ioff[k]);
  }
  w.items_cap = 0;
  dev_free(c, w.lv);
  dev_free(c, w.kpart);
  dev_free(c, w.fa);
  w.ladj_cap = 0;
  dev_free(c, w.scan_temp);
  w.scan_temp = nullptr;
  w.scan_bytes = 0;
  dev_free(c, w.dinv);
  dev_free(c, w.xhat);
  dev_free(c, w.wbuf);
  dev_free(c, w.sg);
  dev_free(c, w.pbuf);
  dev_free(c, w.qn);
  dev_free(c, w.part);
  dev_free(c, w.sums);
  dev_free(c, w.temp);
  w.temp = nullptr;
  w.temp_bytes = 0;
  dev_free(c, w.net_mem);
  dev_free(c, w.mask_d);
  w.net = gnn::Net{};
  w.alloc = false;
  w.params = false;
}

// trainable-parameter mask of the warm-start network (host floats, null: all train)
static rwr_status warm_set_mask(rwr_ctx *c, const float *host) {
  rwr_ctx::Warm &w = c->ws;
  if (!host) {
    dev_free(c, w.mask_d);
    w.net.mask = nullptr;
    return RWR_OK;
  }
  if (!w.mask_d) RWR_TRY(dev_alloc(c, (void **)&w.mask_d, sizeof(float) * gnn::LAYOUT.total));
  H2D(c, w.mask_d, host, sizeof(float) * gnn::LAYOUT.total);
  w.net.mask = w.mask_d;
  return RWR_OK;
}

static rwr_status warm_alloc(rwr_ctx *c, int64_t max_rows) {
  rwr_ctx::Warm &w = c->ws;
  w.max_rows = std::max<int64_t>(max_rows, c->S);
  w.max_nodes = w.max_rows / c->S;
  const size_t nb = gnn::net_view(w.net, c->S, w.max_rows, nullptr, 0, gnn::NET_PART_CAP);
  RWR_TRY(dev_alloc(c, &w.net_mem, nb));
  if (gnn::net_view(w.net, c->S, w.max_rows, w.net_mem, nb, gnn::NET_PART_CAP) != nb) {
    c->err = "network buffers do not fit";
    return RWR_ENOMEM;
  }
  w.net.det = c->det ? 1 : 0;
  RWR_TRY(alloc_zero(c, &w.hop1, c->n_cap));
  RWR_TRY(alloc_zero(c, &w.loc1, c->n_cap));
  RWR_TRY(alloc_zero(c, &w.wlist, c->n_cap));
  RWR_TRY(alloc_zero(c, &w.flags, c->n_cap));
  RWR_TRY(alloc_zero(c, &w.wbuf, (size_t)c->n_cap * c->S));
  RWR_TRY(alloc_zero(c, &w.sg, (size_t)c->n_cap * c->S));
  RWR_TRY(alloc_zero(c, &w.pbuf, (size_t)c->n_cap * c->S));
  RWR_TRY(alloc_zero(c, &w.R, w.max_nodes));
  RWR_TRY(alloc_zero(c, &w.lin_cnt, w.max_nodes + 1));
  RWR_TRY(alloc_zero(c, &w.lin_off, w.max_nodes + 1));
  RWR_TRY(alloc_zero(c, &w.lout_cnt, w.max_nodes + 1));
  RWR_TRY(alloc_zero(c, &w.lout_off, w.max_nodes + 1));
  RWR_TRY(alloc_zero(c, &w.items, w.max_nodes + 1));
  RWR_TRY(alloc_zero(c, &w.lin_items, w.max_nodes + 1));
  RWR_TRY(alloc_zero(c, &w.lout_items, w.max_nodes + 1));
  RWR_TRY(alloc_zero(c, &w.item_off, w.max_nodes + 1));
  RWR_TRY(alloc_zero(c, &w.kpart, (size_t)WS_KPART_BLOCKS * RWR_MAX_COLS));
  RWR_TRY(alloc_zero(c, &w.fa, RWR_MAX_COLS));
  for (int k = 0; k < 2; ++k) {
    RWR_TRY(alloc_zero(c, &w.it_tmp[k], w.max_nodes + 1));
    RWR_TRY(alloc_zero(c, &w.it_rit[k], w.max_nodes + 1));
  }
  RWR_TRY(alloc_zero(c, &w.lv, 3 + WS_MAX_HOPS));
  w.scan_bytes = ws_scan_temp_bytes((int32_t)w.max_nodes);
  RWR_TRY(dev_alloc(c, &w.scan_temp, w.scan_bytes));
  RWR_TRY(alloc_zero(c, &w.dinv, w.max_nodes));
  RWR_TRY(alloc_zero(c, &w.xhat, w.max_rows));
  RWR_TRY(alloc_zero(c, &w.cnt, 4));
  RWR_TRY(alloc_zero(c, &w.qn, 2 * RWR_MAX_COLS));
  RWR_TRY(alloc_zero(c, &w.sums, 4 * RWR_MAX_COLS));
  RWR_TRY(alloc_zero(c, &w.part, (size_t)1024 * 2 * RWR_MAX_COLS));
  w.temp_bytes = ws_select_temp_bytes(c->n_cap);
  RWR_TRY(dev_alloc(c, &w.temp, w.temp_bytes));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  w.alloc = true;
  return RWR_OK;
}

// the network's view of the region: its own edges in local ids
static gnn::RegionView warm_view(rwr_ctx *c) {
  const rwr_ctx::Warm &w = c->ws;
  gnn::RegionView g{};
  g.in_off = w.lin_off;
  g.in_len = w.lin_cnt;
  g.in_adj = w.lin_adj;
  g.out_off = w.lout_off;
  g.out_len = w.lout_cnt;
  g.out_adj = w.lout_adj;
  g.in_items = w.lin_items;
  g.out_items = w.lout_items;
  g.n_in_items = w.n_in_items;
  g.n_out_items = w.n_out_items;
  g.in_item_row = w.lin_item_row;
  g.out_item_row = w.lout_item_row;
  g.loc = nullptr;
  g.nodes = nullptr;
  g.dinv = w.dinv;
  g.nR = w.nR;
  return g;
}

// row-item buffers for rows of up to max_nodes region nodes in the current
// graph (they grow with its edge count)
static rwr_status warm_items(rwr_ctx *c) {
  rwr_ctx::Warm &w = c->ws;
  const int64_t mi = ws_max_items((int32_t)w.max_nodes, c->m);
  if (mi <= w.items_cap) return RWR_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int64_t cap = std::max<int64_t>(mi, w.items_cap + w.items_cap / 2);
  if (cap >= INT32_MAX) {
    c->err = "warm-start row items exceed 2^31";
    return RWR_ENOMEM;
  }
  for (int k = 0; k < 2; ++k) {
    dev_free(c, w.it_irow[k]);
    dev_free(c, w.it_icnt[k]);
    dev_free(c, w.it_ioff[k]);
    RWR_TRY(alloc_zero(c, &w.it_irow[k], cap + 1));
    RWR_TRY(alloc_zero(c, &w.it_icnt[k], cap + 1));
    RWR_TRY(alloc_zero(c, &w.it_ioff[k], cap + 1));
  }
  w.items_cap = cap;
  const size_t sb = ws_scan_temp_bytes((int32_t)std::max<int64_t>(cap, w.max_nodes));
  if (sb > w.scan_bytes) {
    dev_free(c, w.scan_temp);
    w.scan_bytes = 0;
    RWR_TRY(dev_alloc(c, &w.scan_temp, sb));
    w.scan_bytes = sb;
  }
  return RWR_OK;
}

static WsItems items_set(rwr_ctx *c, int k) {
  rwr_ctx::Warm &w = c->ws;
  WsItems it{};
  it.tmp = w.it_tmp[k];
  it.rit = w.it_rit[k];
  it.irow = w.it_irow[k];
  it.icnt = w.it_icnt[k];
  it.ioff = w.it_ioff[k];
  it.max_items = (int32_t)w.items_cap;
  it.scan_temp = w.scan_temp;
  it.scan_bytes = w.scan_bytes;
  return it;
}

// local in- and out-rows of the region (after ws_loc): offsets and item
// counts of both orientations, one read of their totals, then the rows
static rwr_status warm_local_graph(rwr_ctx *c) {
  rwr_ctx::Warm &w = c->ws;
  const DevGraphView &in = c->g[pull_orient(c)].v;
  const DevGraphView &out = c->g[0].v;
  const WsItems A = items_set(c, 0), B = items_set(c, 1);
  HIP_TRY(c, ws_local_rows(w.R, w.lv, w.nR, in, w.loc1, A, w.lin_cnt, w.lin_off, c->stream));
  HIP_TRY(c, ws_local_rows(w.R, w.lv, w.nR, out, w.loc1, B, w.lout_cnt, w.lout_off, c->stream));
  HIP_TRY(c, ws_chunk_items(w.lin_cnt, w.nR, gnn::AGG_CHUNK, w.items, w.lin_items, w.scan_temp, w.scan_bytes,
                            c->stream));
  HIP_TRY(c, ws_chunk_items(w.lout_cnt, w.nR, gnn::AGG_CHUNK, w.items, w.lout_items, w.scan_temp, w.scan_bytes,
                            c->stream));
  int32_t tot[5] = {0, 0, 0, 0, 0};
  HIP_TRY(c, hipMemcpyAsync(&tot[0], w.lin_off + w.nR, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(&tot[1], w.lout_off + w.nR, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(&tot[2], w.lin_items + w.nR, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(&tot[3], w.lout_items + w.nR, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(&tot[4], B.rit + w.nR, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int32_t tin = tot[0], tout = tot[1];
  w.n_in_items = tot[2];
  w.n_out_items = tot[3];
  w.out_items = tot[4];
  const int64_t need = std::max<int64_t>(std::max(tin, tout), 1);
  if (need > w.ladj_cap) {
    dev_free(c, w.lin_adj);
    dev_free(c, w.lout_adj);
    const int64_t cap = std::max<int64_t>(need, 2 * w.ladj_cap);
    RWR_TRY(dev_alloc(c, (void **)&w.lin_adj, sizeof(int32_t) * cap));
    RWR_TRY(dev_alloc(c, (void **)&w.lout_adj, sizeof(int32_t) * cap));
    w.ladj_cap = cap;
  }
  ws_local_fill(w.R, w.lv, in, w.loc1, A, w.lin_adj, c->stream);
  ws_local_fill(w.R, w.lv, out, w.loc1, B, w.lout_adj, c->stream);
  const int64_t ni = std::max<int64_t>({w.n_in_items, w.n_out_items, 1});
  if (ni > w.item_row_cap) {
    dev_free(c, w.lin_item_row);
    dev_free(c, w.lout_item_row);
    const int64_t cap = std::max<int64_t>(ni, 2 * w.item_row_cap);
    RWR_TRY(dev_alloc(c, (void **)&w.lin_item_row, sizeof(int32_t) * cap));
    RWR_TRY(dev_alloc(c, (void **)&w.lout_item_row, sizeof(int32_t) * cap));
    w.item_row_cap = cap;
  }
  gnn::region_item_rows(w.lin_items, w.nR, w.lin_item_row, c->stream);
  gnn::region_item_rows(w.lout_items, w.nR, w.lout_item_row, c->stream);
  return RWR_OK;
}

// After the offset seed (q in ybuf, its support stamped) and the structural
// update: the region (offset support and the nodes within `hops` out-hops,
// level by level, a level that would exceed the capacity left out), the
// features, the forward pass, the prediction and its exact residual.
// Prediction on: the seed becomes the residual in every column where the
// residual is smaller, and the scores take the prediction.  Training on: one
// AdamW step on the loss sum_j ||rho_j||_1 / sum_j ||q_j||_1 of this
// prediction.
static rwr_status warm_prepare(rwr_ctx *c) {
  rwr_ctx::Warm &w = c->ws;
  const double t0 = now_ms();
  w.nR = 0;
  w.accepted = 0;
  w.fallback = 0;
  w.ratio = 1.0;
  w.loss = 0.0;
  w.trained = false;
  w.level_end.clear();
  const int S = c->S;
  const DevGraphView &in = c->g[pull_orient(c)].v;
  const DevGraphView &out = c->g[0].v;
  const int32_t st0 = c->ctl_h->stamp;
  RWR_TRY(warm_items(c));
  HIP_TRY(c, ws_region(c->stamp, st0, c->n, w.hops, (int32_t)w.max_nodes, out, w.hop1, w.flags, w.wlist, w.cnt,
                       w.R, w.lv, items_set(c, 0), w.temp, w.temp_bytes, c->stream));
  int32_t lvh[3 + WS_MAX_HOPS];
  D2H(c, lvh, w.lv, sizeof(int32_t) * (3 + w.hops));
  const int32_t nR = lvh[0];
  for (int h = 0; h <= w.hops && lvh[2 + h] >= 0; ++h) w.level_end.push_back(lvh[2 + h]);
  const int32_t n0 = w.level_end.empty() ? 0 : w.level_end[0];
  w.nR = nR;
  if (nR == 0 || n0 == 0) {
    ws_clear(w.R, nR, w.hop1, w.loc1, c->stream);
    w.nR = 0;
    w.ms = now_ms() - t0;
    return RWR_OK;
  }
  const int64_t rows = (int64_t)nR * S;
  const double c1 = 1.0 - c->cfg.c;
  ws_loc(w.R, nR, out, w.loc1, w.dinv, c->stream);
  RWR_TRY(warm_local_graph(c));
  ws_qnorm(w.R, n0, S, c->ybuf, w.part, w.qn, c->stream);
  ws_features(w.R, nR, S, w.hop1, in, out, c->ybuf, c->r, c->ctl, c->seeds_d, w.qn, c->n, w.net.F, c->stream);
  gnn::net_forward(w.net, warm_view(c), rows, c->stream);
  // prediction in wbuf (dense) and xhat (region rows)
  double *beta = w.sums + 2 * RWR_MAX_COLS;
  ws_predict(w.R, nR, S, out, w.net.o, w.qn, c1, w.xhat, w.wbuf, w.part, beta, w.fa, c->stream);
  // work items over the region's out-rows (the push and the gradient)
  const int64_t need = ((int64_t)nR + c->m / 1024 + 2) * S;
  if (need > w.gpart_cap) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    dev_free(c, w.gpart);
    dev_free(c, w.grow);
    w.gpart_cap = 0;
    RWR_TRY(dev_alloc(c, (void **)&w.gpart, sizeof(double) * need));
    RWR_TRY(dev_alloc(c, (void **)&w.grow, sizeof(int32_t) * (need / S)));
    w.gpart_cap = need;
  }
  HIP_TRY(c, ws_out_items(w.R, nR, out, w.items, w.item_off, w.grow, w.scan_temp, w.scan_bytes, c->stream));
  // rho = q - (I - (1-c) B~^T) xhat': from the region alone (a push over its
  // out-rows) when those rows hold less than a quarter of the graph's edges,
  // else by a pull over every in-row; the push adds with FP64 atomics, so
  // deterministic mode always pulls
  w.pushed = !c->det && (w.push_mode == 1 || (w.push_mode < 0 && (int64_t)w.out_items * 1024 * 4 < c->m));
  // (rho lives in pbuf, so that carried vectors in gbuf stay untouched)
  if (w.pushed) {
    ws_rho_push(w.R, nR, S, out, w.item_off, w.grow, w.xhat, c1, w.pbuf, w.hop1, c->n, c->ybuf, w.wbuf, w.sg,
                w.part, w.sums, c->stream);
  } else {
    SlotArgs a = slot_args(c);
    a.r = w.wbuf;
    a.gbuf = w.pbuf;
    a.zero_seed_rows = 0;
    launch_apply_p(a, S, c->stream);
    ws_rho(c->n, S, c->ybuf, w.pbuf, w.wbuf, w.sg, w.part, w.sums, c->stream);
  }
  std::vector<double> sums(2 * S);
  D2H(c, sums.data(), w.sums, sizeof(double) * 2 * S);
  w.qn_h.assign(S, 0.0);
  D2H(c, w.qn_h.data(), w.qn, sizeof(double) * S);
  uint64_t accept = 0;
  double num = 0.0, den = 0.0;
  int n_act = 0;
  std::vector<int32_t> act(RWR_MAX_COLS, 0);
  for (int j = 0; j < c->n_seeds; ++j) {
    const double q = w.qn_h[j], rho = sums[j];
    if (!(q > 0.0) || !std::isfinite(rho)) continue;
    act[j] = 1;
    ++n_act;
    den += q;
    num += rho;
    if ((w.mode & 1) && rho < q) {
      accept |= 1ull << j;
      ++w.accepted;
    } else if (w.mode & 1) {
      ++w.fallback;
    }
  }
  w.ratio = den > 0.0 ? num / den : 1.0;
  if ((w.mode & 2) && n_act > 0) {
    w.loss = num / den;
    H2D(c, w.net.active, act.data(), sizeof(int32_t) * RWR_MAX_COLS);
    HIP_TRY(c, ws_resid_grad(w.R, nR, S, out, c1, w.pbuf, w.sg, w.gpart, w.items, w.item_off, w.grow, w.scan_temp,
                             w.scan_bytes, w.net.active, den, w.net.o, w.qn, beta, w.fa, w.kpart,
                             w.sums + 3 * RWR_MAX_COLS, w.net.dout, c->stream));
    gnn::net_backward(w.net, warm_view(c), rows, c->stream);
    gnn::net_adamw(w.net, c->stream);
    w.trained = true;
  }
  if (w.pushed) {
    ws_apply_sparse(c->n, S, accept, w.hop1, c->ybuf, w.pbuf, c->r, w.wbuf, c->stamp, c->ctl, w.sums + S,
                    c->stream);
    ws_unmark_boundary(c->n, w.hop1, c->stream);
  } else {
    ws_apply(c->n, S, accept, c->ybuf, w.pbuf, c->r, w.wbuf, c->stamp, c->ctl, w.sums + S, c->stream);
  }
  ws_unscatter(w.R, nR, S, w.wbuf, c->stream);
  ws_clear(w.R, nR, w.hop1, w.loc1, c->stream);
  w.ms = now_ms() - t0;
  return RWR_OK;
}

static void fill_stats(rwr_ctx *c, rwr_stats *st) {
  if (!st) return;
  const Ctl &h = *c->ctl_h;
  st->iters = std::max(0, h.iter - 1);
  st->dense_iters = h.dense_iters;
  st->visited_edges = h.visited + (int64_t)h.dense_iters * c->m;
  st->touched_rows = h.nT[0];
  double q = 0.0, lx = 0.0;
  for (int j = 0; j < c->n_seeds; ++j) {
    q = std::max(q, h.norm0[j]);
    lx = std::max(lx, h.last_norm[j]);
  }
  st->q_off_l1 = q;
  st->last_x_l1 = lx;
  st->carry_l1 = c->last_carry_l1;
  double dr = 0.0;
  for (int j = 0; j < c->n_seeds; ++j)
    dr = std::max(dr, c->seed_sorted ? std::ldexp((double)h.dr_fix[j], -52) : h.dr_l1[j]);
  st->dr_l1 = dr;
}

// argument checks shared by rwr_gnn_eval and rwr_gnn_eval_noalloc
static rwr_status gnn_eval_check(const float *params, int32_t nR, int32_t S, const int32_t *in_off,
                                 const int32_t *in_len, const int32_t *in_adj, int64_t n_in, const int32_t *out_off,
                                 const int32_t *out_len, const int32_t *out_adj, int64_t n_out, const float *dinv,
                                 const float *feats, const float *target, const int32_t *active, float *grad,
                                 double *loss, float *params_after) {
  if (!params || nR <= 0 || S < 1 || S > RWR_MAX_COLS || !in_off || !in_len || (n_in > 0 && !in_adj) ||
      !out_off || !out_len || (n_out > 0 && !out_adj) || !dinv || !feats || n_in < 0 || n_out < 0) {
    g_build_error = "invalid arguments";
    return RWR_EINVAL;
  }
  if ((target == nullptr) != (active == nullptr) || ((grad || loss || params_after) && !target)) {
    g_build_error = "gradients need a target and active columns";
    return RWR_EINVAL;
  }
  for (int32_t i = 0; i < nR; ++i) {
    if (in_len[i] < 0 || out_len[i] < 0 || in_off[i] < 0 || out_off[i] < 0 || in_off[i] + (int64_t)in_len[i] > n_in ||
        out_off[i] + (int64_t)out_len[i] > n_out) {
      g_build_error = "region rows out of range";
      return RWR_EINVAL;
    }
  }
  for (int64_t e = 0; e < n_in; ++e)
    if (in_adj[e] < 0 || in_adj[e] >= nR) {
      g_build_error = "region adjacency id out of range";
      return RWR_EINVAL;
    }
  for (int64_t e = 0; e < n_out; ++e)
    if (out_adj[e] < 0 || out_adj[e] >= nR) {
      g_build_error = "region adjacency id out of range";
      return RWR_EINVAL;
    }
  return RWR_OK;
}

// --------------------------------------------- evaluation without allocation
// rwr_gnn_eval_noalloc runs the network in one fixed file-scope device array
// instead of memory it allocates: regions of at most NA_MAX_ROWS (node,
// column) rows and NA_MAX_EDGES edges per orientation.  Each device holds its
// own copy of the array until the process ends; host code reaches it only
// through the address hipGetSymbolAddress gives on that device (the array's
// name on the host is a stand-in, not a device address).
#define NA_MAX_ROWS 8192
#define NA_MAX_EDGES 131072
#define NA_BYTES (24u << 20)
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

static std::mutex g_na_mu;
static void *g_na_ptr[64] = {};

// the array's device address on the current device (looked up once per device)
static rwr_status noalloc_scratch(void **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    g_build_error = "no usable current device";
    return RWR_EHIP;
  }
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (!g_na_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      g_build_error = std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(e);
      return RWR_EHIP;
    }
    g_na_ptr[dev] = ptr;
  }
  *out = g_na_ptr[dev];
  return RWR_OK;
}

// items[i] = sum over k < i of ceil(len[k] / chunk), i = 0 .. nR (one
// workgroup of NA_SCAN threads: per-thread ranges, then a scan of their sums)
#define NA_SCAN 1024
__global__ __launch_bounds__(NA_SCAN) void k_na_items(const int32_t *__restrict__ len, int32_t nR, int32_t chunk,
                                                      int32_t *__restrict__ items) {
  __shared__ int32_t tot[NA_SCAN];
  const int t = threadIdx.x;
  const int32_t per = (nR + NA_SCAN - 1) / NA_SCAN;
  const int32_t lo = min(nR, t * per), hi = min(nR, lo + per);
  int32_t s = 0;
  for (int32_t i = lo; i < hi; ++i) s += (len[i] + chunk - 1) / chunk;
  tot[t] = s;
  __syncthreads();
  for (int off = 1; off < NA_SCAN; off <<= 1) {
    const int32_t v = t >= off ? tot[t - off] : 0;
    __syncthreads();
    tot[t] += v;
    __syncthreads();
  }
  int32_t acc = tot[t] - s;  // exclusive prefix of this thread's range
  for (int32_t i = lo; i < hi; ++i) {
    items[i] = acc;
    acc += (len[i] + chunk - 1) / chunk;
  }
  if (t == NA_SCAN - 1) items[nR] = tot[t];
}

// ------------------------------------------------------------------ ABI
extern "C" {

rwr_status rwr_config_default(rwr_config *cfg) {
  if (!cfg) return RWR_EINVAL;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->c = 0.15;
  cfg->eps = 1e-9;
  cfg->err_budget = 0.0;
  cfg->build_tol = 0.0;
  cfg->precision = RWR_PROP_FP32;
  cfg->undirected = 0;
  cfg->max_iters = 10000;
  cfg->pull_ratio = 0;
  cfg->reorder = 1;
  cfg->autotune = 1;
  cfg->stream = nullptr;
  return RWR_OK;
}

static rwr_status build_impl(rwr_ctx *c, int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                             int32_t n_seeds, const int32_t *seeds, int32_t on_device, const double *q = nullptr) {
  HIP_TRY(c, hipGetDevice(&c->device));
  HIP_TRY(c, hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device));
  if (c->cfg.stream) {
    c->stream = (hipStream_t)c->cfg.stream;
  } else {
    HIP_TRY(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
  }
  c->undirected = c->cfg.undirected != 0;
  c->fp64 = c->cfg.precision == RWR_PROP_FP64;
  c->max_iters = c->cfg.max_iters > 0 ? c->cfg.max_iters : 10000;
  // builds and refinements start from a norm of at most about 1 and stop
  // above 1e-16: Theorem 2 bounds their iterations by log_{1-c}(1e-16)
  c->solve_iters = std::max<int32_t>(c->max_iters, (int32_t)std::ceil(std::log(1e-16) / std::log(1.0 - c->cfg.c)) + 64);
  c->rows_only = c->cfg.node_deletion == 1 && !c->cfg.undirected;
  c->det = c->cfg.deterministic != 0;
  c->n = n;
  c->n_cap = (int32_t)std::min<int64_t>((int64_t)n + std::max<int64_t>(1024, n / 16), INT32_MAX - 1);
  c->n_seeds = n_seeds;
  c->S = next_pow2_cols(n_seeds);
  c->budget = c->cfg.err_budget > 0 ? c->cfg.err_budget : 2.0 * c->cfg.eps / c->cfg.c;
  c->qmode = q != nullptr;
  if (seeds) c->seeds_h.assign(seeds, seeds + n_seeds);
  tune_defaults(c);

  HIP_TRY(c, hipHostMalloc((void **)&c->ctl_h, sizeof(Ctl), hipHostMallocDefault));
  std::memset(c->ctl_h, 0, sizeof(Ctl));
  RWR_TRY(alloc_zero(c, &c->ctl, 1));
  {
    Ctl init{};
    init.stamp = 1;
    H2D(c, c->ctl, &init, sizeof(Ctl));
  }
  RWR_TRY(alloc_zero(c, &c->seeds_d, RWR_MAX_COLS));

  // edge list on the device, both directions for undirected graphs
  int32_t *src_d = nullptr, *dst_d = nullptr;
  int64_t m2 = m;
  if (c->undirected) {
    std::vector<int32_t> hs(m), hd(m);
    if (m > 0) {
      if (on_device) {
        D2H(c, hs.data(), src, sizeof(int32_t) * m);
        D2H(c, hd.data(), dst, sizeof(int32_t) * m);
      } else {
        std::memcpy(hs.data(), src, sizeof(int32_t) * m);
        std::memcpy(hd.data(), dst, sizeof(int32_t) * m);
      }
    }
    std::vector<int32_t> s2, d2;
    s2.reserve(2 * m);
    d2.reserve(2 * m);
    for (int64_t i = 0; i < m; ++i) {
      s2.push_back(hs[i]);
      d2.push_back(hd[i]);
      if (hs[i] != hd[i]) {
        s2.push_back(hd[i]);
        d2.push_back(hs[i]);
      }
    }
    m2 = (int64_t)s2.size();
    RWR_TRY(dev_alloc(c, (void **)&src_d, sizeof(int32_t) * std::max<int64_t>(1, m2)));
    RWR_TRY(dev_alloc(c, (void **)&dst_d, sizeof(int32_t) * std::max<int64_t>(1, m2)));
    if (m2 > 0) {
      H2D(c, src_d, s2.data(), sizeof(int32_t) * m2);
      H2D(c, dst_d, d2.data(), sizeof(int32_t) * m2);
    }
  } else if (on_device) {
    src_d = const_cast<int32_t *>(src);
    dst_d = const_cast<int32_t *>(dst);
  } else {
    RWR_TRY(dev_alloc(c, (void **)&src_d, sizeof(int32_t) * std::max<int64_t>(1, m)));
    RWR_TRY(dev_alloc(c, (void **)&dst_d, sizeof(int32_t) * std::max<int64_t>(1, m)));
    if (m > 0) {
      H2D(c, src_d, src, sizeof(int32_t) * m);
      H2D(c, dst_d, dst, sizeof(int32_t) * m);
    }
  }
  const bool own_edges = c->undirected || !on_device;
  // internal numbering: descending out-degree, or the caller's order
  RWR_TRY(alloc_zero(c, &c->perm, c->n_cap));
  RWR_TRY(alloc_zero(c, &c->inv, c->n_cap));
  int32_t *msrc = nullptr, *mdst = nullptr;
  RWR_TRY(dev_alloc(c, (void **)&msrc, sizeof(int32_t) * std::max<int64_t>(1, m2)));
  RWR_TRY(dev_alloc(c, (void **)&mdst, sizeof(int32_t) * std::max<int64_t>(1, m2)));
  if (c->cfg.reorder) {
    uint64_t *k1 = nullptr, *k2 = nullptr;
    int32_t *deg = nullptr;
    RWR_TRY(dev_alloc(c, (void **)&k1, sizeof(uint64_t) * c->n_cap));
    RWR_TRY(dev_alloc(c, (void **)&k2, sizeof(uint64_t) * c->n_cap));
    RWR_TRY(dev_alloc(c, (void **)&deg, sizeof(int32_t) * c->n_cap));
    RWR_TRY(ensure_temp(c, build_temp_bytes(std::max<int64_t>(m2, c->n_cap), c->n_cap)));
    HIP_TRY(c, build_relabel(src_d, m2, n, c->n_cap, c->perm, c->inv, deg, k1, k2, c->temp, c->temp_bytes,
                             c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    dev_free(c, k1);
    dev_free(c, k2);
    dev_free(c, deg);
  } else {
    launch_identity(c->perm, c->inv, 0, c->n_cap, c->stream);
  }
  launch_map_ids(src_d, m2, n, c->perm, msrc, c->stream);
  launch_map_ids(dst_d, m2, n, c->perm, mdst, c->stream);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (own_edges) {
    dev_free(c, src_d);
    dev_free(c, dst_d);
  }
  rwr_status s = build_orient(c, 0, msrc, mdst, m2);
  if (s == RWR_OK && !c->undirected) s = build_orient(c, 1, mdst, msrc, m2);
  dev_free(c, msrc);
  dev_free(c, mdst);
  if (s == RWR_OK && c->qmode) {
    // seed vectors in internal ids (no seed nodes)
    launch_fill_i32(c->seeds_d, RWR_MAX_COLS, -1, c->stream);
    std::vector<int32_t> perm(n);
    D2H(c, perm.data(), c->perm, sizeof(int32_t) * n);
    std::vector<double> qi((size_t)c->n_cap * c->S, 0.0);
    for (int32_t v = 0; v < n; ++v)
      for (int32_t j = 0; j < n_seeds; ++j) qi[(size_t)perm[v] * c->S + j] = q[(size_t)v * n_seeds + j];
    RWR_TRY(dev_alloc(c, (void **)&c->qvec, sizeof(double) * qi.size()));
    H2D(c, c->qvec, qi.data(), sizeof(double) * qi.size());
  } else if (s == RWR_OK) {
    // seeds in internal ids
    int32_t *tmp = nullptr;
    RWR_TRY(dev_alloc(c, (void **)&tmp, sizeof(int32_t) * RWR_MAX_COLS));
    H2D(c, tmp, seeds, sizeof(int32_t) * n_seeds);
    launch_fill_i32(c->seeds_d, RWR_MAX_COLS, -1, c->stream);  // padding columns name no node
    launch_map_ids(tmp, n_seeds, n, c->perm, c->seeds_d, c->stream);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    dev_free(c, tmp);
  }
  if (s != RWR_OK) return s;
  if (c->undirected) c->g[1] = c->g[0];
  c->m = m2;

  // score and propagation state
  const size_t nS = (size_t)c->n_cap * c->S;
  RWR_TRY(alloc_zero(c, &c->r, nS));
  RWR_TRY(alloc_zero(c, &c->ybuf, nS));
  RWR_TRY(alloc_zero(c, &c->gbuf, nS));
  RWR_TRY(alloc_zero(c, &c->xres, nS));
  const size_t xs = c->fp64 ? 8 : 4;
  RWR_TRY(dev_alloc(c, &c->x[0], xs * nS));
  RWR_TRY(dev_alloc(c, &c->x[1], xs * nS));
  launch_zero_bytes(c->x[0], xs * nS, c->stream);
  launch_zero_bytes(c->x[1], xs * nS, c->stream);
  RWR_TRY(alloc_zero(c, &c->stamp, c->n_cap));
  RWR_TRY(alloc_zero(c, &c->fstamp, c->n_cap));
  RWR_TRY(alloc_zero(c, &c->nmark, c->n_cap));
  RWR_TRY(alloc_zero(c, &c->hfront, c->n_cap));
  RWR_TRY(alloc_zero(c, &c->hbase, c->n_cap));
  RWR_TRY(alloc_zero(c, &c->sel, (size_t)c->n_cap * 2));
  RWR_TRY(alloc_zero(c, &c->sel_count, 1));
  // norms of the update runs (max_iters + 2 rows), then of the build and
  // refinement runs (solve_iters + 2 rows)
  RWR_TRY(alloc_zero(c, &c->hist, (size_t)(c->max_iters + 2 + c->solve_iters + 2) * c->S));
  RWR_TRY(plan_heavy(c, true));
  RWR_TRY(ensure_partials(c));

  // static scores: CPI from c*e_s (Section 2.2), then residual refinement.
  // Its first dense sweeps also choose the sweep shape (unless fixed by the
  // caller's configuration or the environment).
  // (not in deterministic mode: the shape sets each row's summation order)
  const char *cache = getenv("RWR_TUNE_CACHE");
  std::string tkey;
  bool cached = false;
  if (c->cfg.autotune && !c->det && !getenv("RWR_PULL_LANES") && !getenv("RWR_GRID_PULL") && cache && *cache) {
    RWR_TRY(tune_key(c, &tkey));
    int32_t l = 0, g = 0;
    double ms = 0.0;
    if (tune_cache_find(cache, tkey, &l, &g, &ms)) {
      c->pull_lanes = l;
      c->grid_pull = g;
      c->tune.best_ms = ms;
      c->tune.cached = true;
      cached = true;
      RWR_TRY(ensure_partials(c));
    }
  }
  if (c->cfg.autotune && !c->det && !cached && !getenv("RWR_PULL_LANES") && !getenv("RWR_GRID_PULL")) {
    tune_begin(c);
    if (!tkey.empty()) {
      c->tune.cache_path = cache;
      c->tune.cache_key = tkey;
    }
    int32_t gmax = 0;
    for (const auto &cd : c->tune.cand) gmax = std::max(gmax, cd.second);
    const int32_t keep = c->grid_pull;
    c->grid_pull = std::max(c->grid_pull, gmax);
    RWR_TRY(ensure_partials(c));
    c->grid_pull = keep;
  }
  const double build_tol = c->cfg.build_tol > 0 ? c->cfg.build_tol : 0.25 * c->budget;
  const double cc = c->cfg.c;
  const double eps0 = std::min(c->cfg.eps, build_tol * cc / (4.0 * (1.0 - cc)));
  const SlotArgs a = slot_args(c);
  launch_reset_run(c->ctl, c->S, all_cols_mask(n_seeds), eps0, c->solve_iters, dense_thresh(c), c->n / 16 + 1,
                   c->stream);
  if (c->qmode)
    launch_seed_init_q(a, c->S, c->stream);
  else
    launch_seed_init(a, c->S, c->stream);
  launch_slot0_epilogue(a, c->S, c->fp64, c->stream);
  RWR_TRY(run_slots(c, MODE_SPARSE, -1.0, 0.0, false, 0, c->solve_iters));
  RWR_TRY(read_ctl(c));
  if (c->ctl_h->prop_err != 0) {
    c->err = "initial solve did not converge";
    return (rwr_status)c->ctl_h->prop_err;
  }
  account_run(c, true);
  // certify (and refine) until the build tolerance holds
  const double saved = c->budget;
  c->budget = build_tol;
  for (int round = 0; round < 8; ++round) {
    rwr_stats st{};
    RWR_TRY(check_and_refine(c, true, &st));
    if (!st.refined) break;
  }
  c->budget = saved;
  if (c->tune.on) tune_finish(c);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return RWR_OK;
}

rwr_status rwr_build(const rwr_config *cfg, int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                     int32_t n_seeds, const int32_t *seeds, int32_t edges_on_device, rwr_ctx **out) {
  if (!out) return RWR_EINVAL;
  *out = nullptr;
  rwr_config def;
  rwr_config_default(&def);
  const rwr_config &cf = cfg ? *cfg : def;
  if (n <= 0 || m < 0 || (m > 0 && (!src || !dst)) || n_seeds < 1 || n_seeds > RWR_MAX_COLS || !seeds ||
      !(cf.c > 0.0 && cf.c < 1.0) || !(cf.eps > 0.0) || n >= INT32_MAX - 1024) {
    g_build_error = "invalid argument";
    return RWR_EINVAL;
  }
  for (int i = 0; i < n_seeds; ++i) {
    if (seeds[i] < 0 || seeds[i] >= n) {
      g_build_error = "seed id out of range";
      return RWR_EINVAL;
    }
    for (int k = 0; k < i; ++k)
      if (seeds[k] == seeds[i]) {
        g_build_error = "repeated seed";
        return RWR_EINVAL;
      }
  }
  if ((cf.dev_alloc == nullptr) != (cf.dev_free == nullptr)) {
    g_build_error = "dev_alloc and dev_free must be given together";
    return RWR_EINVAL;
  }
  rwr_ctx *c = new rwr_ctx();
  c->cfg = cf;
  rwr_status s = build_impl(c, n, m, src, dst, n_seeds, seeds, edges_on_device);
  if (s != RWR_OK) {
    g_build_error = c->err;
    rwr_destroy(c);
    return s;
  }
  c->built = true;
  *out = c;
  return RWR_OK;
}

rwr_status rwr_build_vectors(const rwr_config *cfg, int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                             int32_t n_cols, const double *q, int32_t edges_on_device, rwr_ctx **out) {
  if (!out) return RWR_EINVAL;
  *out = nullptr;
  rwr_config def;
  rwr_config_default(&def);
  const rwr_config &cf = cfg ? *cfg : def;
  if (n <= 0 || m < 0 || (m > 0 && (!src || !dst)) || n_cols < 1 || n_cols > RWR_MAX_COLS || !q ||
      !(cf.c > 0.0 && cf.c < 1.0) || !(cf.eps > 0.0) || n >= INT32_MAX - 1024) {
    g_build_error = "invalid argument";
    return RWR_EINVAL;
  }
  for (int32_t j = 0; j < n_cols; ++j) {
    double sum = 0.0;
    for (int32_t v = 0; v < n; ++v) {
      const double x = q[(size_t)v * n_cols + j];
      if (!(x >= 0.0) || !std::isfinite(x)) {
        g_build_error = "seed vector entry negative or not finite";
        return RWR_EINVAL;
      }
      sum += x;
    }
    if (std::fabs(sum - 1.0) > 1e-9) {
      g_build_error = "seed vector does not sum to 1";
      return RWR_EINVAL;
    }
  }
  if ((cf.dev_alloc == nullptr) != (cf.dev_free == nullptr)) {
    g_build_error = "dev_alloc and dev_free must be given together";
    return RWR_EINVAL;
  }
  rwr_ctx *c = new rwr_ctx();
  c->cfg = cf;
  rwr_status s = build_impl(c, n, m, src, dst, n_cols, nullptr, edges_on_device, q);
  if (s != RWR_OK) {
    g_build_error = c->err;
    rwr_destroy(c);
    return s;
  }
  c->built = true;
  *out = c;
  return RWR_OK;
}

static rwr_status ensure_batch(rwr_ctx *c, int64_t nkeys, int64_t nints) {
  if (nkeys > c->bcap) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int64_t cap = std::max<int64_t>(nkeys, 2 * c->bcap);
    for (int o = 0; o < 2; ++o) {
      dev_free(c, c->keys[o]);
      dev_free(c, c->seg[o]);
      dev_free(c, c->row[o]);
      dev_free(c, c->t_dold[o]);
      dev_free(c, c->t_dnew[o]);
      RWR_TRY(alloc_zero(c, &c->keys[o], cap));
      RWR_TRY(alloc_zero(c, &c->seg[o], cap + 1));
      RWR_TRY(alloc_zero(c, &c->row[o], cap + 1));
      RWR_TRY(alloc_zero(c, &c->t_dold[o], cap + 1));
      RWR_TRY(alloc_zero(c, &c->t_dnew[o], cap + 1));
    }
    dev_free(c, c->keys_alt);
    dev_free(c, c->flags);
    dev_free(c, c->pos);
    dev_free(c, c->sdcnt);
    dev_free(c, c->sroff);
    dev_free(c, c->bigv);
    dev_free(c, c->biga);
    RWR_TRY(alloc_zero(c, &c->keys_alt, cap));
    RWR_TRY(alloc_zero(c, &c->bigv, 2 * (cap + 1)));
    RWR_TRY(alloc_zero(c, &c->biga, 2 * (cap + 1)));
    RWR_TRY(alloc_zero(c, &c->flags, cap + 1));
    RWR_TRY(alloc_zero(c, &c->pos, cap + 1));
    RWR_TRY(alloc_zero(c, &c->sdcnt, cap + 1));
    RWR_TRY(alloc_zero(c, &c->sroff, cap + 1));
    RWR_TRY(ensure_temp(c, std::max(sort_temp_bytes((int32_t)cap), seed_scan_temp_bytes((int32_t)cap))));
    c->bcap = cap;
  }
  if (nints > c->b_host_cap) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->b_host) (void)hipHostFree(c->b_host);
    dev_free(c, c->b_dev);
    const int64_t cap = std::max<int64_t>(nints, 2 * c->b_host_cap);
    HIP_TRY(c, hipHostMalloc((void **)&c->b_host, sizeof(int32_t) * cap, hipHostMallocDefault));
    RWR_TRY(dev_alloc(c, (void **)&c->b_dev, sizeof(int32_t) * cap));
    c->b_host_cap = cap;
  }
  return RWR_OK;
}

// record buffers of the sorted offset seed for n_rec records
static rwr_status ensure_seed_recs(rwr_ctx *c, int64_t n_rec) {
  if (n_rec > c->srec_cap) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int64_t cap = std::min<int64_t>(INT32_MAX, std::max<int64_t>(n_rec, 2 * c->srec_cap));
    for (int i = 0; i < 2; ++i) {
      dev_free(c, c->srec[i]);
      c->srec[i] = nullptr;
    }
    dev_free(c, c->spart);
    c->spart = nullptr;
    c->srec_cap = 0;
    for (int i = 0; i < 2; ++i) RWR_TRY(dev_alloc(c, (void **)&c->srec[i], sizeof(uint64_t) * cap));
    RWR_TRY(dev_alloc(c, (void **)&c->spart, sizeof(double) * 2 * seed_part_len(cap, c->S)));
    c->srec_cap = cap;
  }
  return ensure_temp(c, seed_sort_temp_bytes(c->srec_cap));
}

// whether an update may take the sorted offset seed (it then needs the
// record count that validation sums)
static bool seed_sort_possible(const rwr_ctx *c) {
  return c->det || c->seed_sort_mode == 1 || (c->seed_sort_mode < 0 && c->S >= SEED_SORT_MIN_S);
}

// per-orientation arguments of the batch kernels (check: the out orientation
// tests the batch against the graph)
static OrientPair orient_pair(const rwr_ctx *c, bool check) {
  OrientPair P{};
  const int po = pull_orient(c);
  for (int o = 0; o < 2; ++o) {
    OrientArgs &q = P.o[o];
    q.keys = c->keys[o];
    q.seg = c->seg[o];
    q.row = c->row[o];
    q.g = c->g[o].v;
    q.t_dold = c->t_dold[o];
    q.t_dnew = c->t_dnew[o];
    q.orient = o;
    q.check = (check && o == 0) ? 1 : 0;
    q.heavy_limit = o == po ? c->heavy_limit : 0;
    q.e_cap = c->g[o].e_cap;
  }
  P.bigv = c->bigv;
  P.biga = c->biga;
  P.big = c->big_batch ? 1 : 0;
  P.recs = seed_sort_possible(c) ? 1 : 0;
  return P;
}

// phase-timing event i on the context's stream (config phase_timing)
static rwr_status phase_mark(rwr_ctx *c, int i) {
  if (!c->cfg.phase_timing) return RWR_OK;
  if (!c->ph_ev[i]) HIP_TRY(c, timing_event(&c->ph_ev[i]));
  HIP_TRY(c, hipEventRecord(c->ph_ev[i], c->stream));
  return RWR_OK;
}

static double phase_ms(rwr_ctx *c, int a, int b) {
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, c->ph_ev[a], c->ph_ev[b]) != hipSuccess) return 0.0;
  return ms;
}

rwr_status rwr_update(rwr_ctx *c, const rwr_batch *b, rwr_stats *st) {
  if (!c || !b) return RWR_EINVAL;
  const double t0 = now_ms();
  if (st) std::memset(st, 0, sizeof(*st));
  if (c->stale) {
    c->err = "context is stale (an earlier update did not converge); call rwr_refine";
    return RWR_ESTATE;
  }
  RWR_TRY(phase_mark(c, 0));
  if (b->n_ins < 0 || b->n_del < 0 || b->n_new_nodes < 0 || b->n_del_nodes < 0 ||
      (b->n_ins > 0 && (!b->ins_src || !b->ins_dst)) || (b->n_del > 0 && (!b->del_src || !b->del_dst))) {
    c->err = "invalid batch";
    return RWR_EINVAL;
  }
  if (b->n_del_nodes > 0 && !b->del_nodes) {
    c->err = "invalid batch";
    return RWR_EINVAL;
  }
  // node deletions are checked on the host: ids of existing nodes, distinct,
  // no seed (the walk restarts there)
  const int32_t nd = b->n_del_nodes;
  std::vector<int32_t> dn(nd);
  if (nd > 0) {
    if (b->on_device)
      D2H(c, dn.data(), b->del_nodes, sizeof(int32_t) * nd);
    else
      std::memcpy(dn.data(), b->del_nodes, sizeof(int32_t) * nd);
    std::vector<int32_t> sorted = dn;
    std::sort(sorted.begin(), sorted.end());
    for (int32_t i = 0; i < nd; ++i) {
      if (sorted[i] < 0 || sorted[i] >= c->n || (i > 0 && sorted[i] == sorted[i - 1])) {
        c->err = "node deletion names an id out of range or twice";
        return RWR_EINVAL;
      }
    }
    for (int32_t sd : c->seeds_h) {
      if (std::binary_search(sorted.begin(), sorted.end(), sd)) {
        c->err = "a seed node cannot be deleted";
        return RWR_EINVAL;
      }
    }
  }
  const int64_t n_new64 = (int64_t)c->n + b->n_new_nodes;
  if (n_new64 >= INT32_MAX - 1024) {
    c->err = "node count overflow";
    return RWR_EINVAL;
  }
  const int32_t n_new = (int32_t)n_new64;
  RWR_TRY(grow_nodes(c, n_new));
  const int64_t N = b->n_ins + b->n_del;
  const int64_t nints = 2 * N + nd;
  RWR_TRY(ensure_batch(c, 1, std::max<int64_t>(nints, 1)));
  const int32_t *ins_s = b->ins_src, *ins_d = b->ins_dst, *del_s = b->del_src, *del_d = b->del_dst;
  int32_t *dn_dev = c->b_dev + 2 * N;
  if (nints > 0) {
    int32_t *h = c->b_host;
    if (!b->on_device) {
      std::memcpy(h, b->ins_src, sizeof(int32_t) * b->n_ins);
      std::memcpy(h + b->n_ins, b->ins_dst, sizeof(int32_t) * b->n_ins);
      std::memcpy(h + 2 * b->n_ins, b->del_src, sizeof(int32_t) * b->n_del);
      std::memcpy(h + 2 * b->n_ins + b->n_del, b->del_dst, sizeof(int32_t) * b->n_del);
    }
    if (nd > 0) std::memcpy(h + 2 * N, dn.data(), sizeof(int32_t) * nd);
    const int64_t lo = b->on_device ? 2 * N : 0;
    if (nints > lo)
      HIP_TRY(c, hipMemcpyAsync(c->b_dev + lo, h + lo, sizeof(int32_t) * (nints - lo), hipMemcpyHostToDevice,
                                c->stream));
    if (!b->on_device) {
      ins_s = c->b_dev;
      ins_d = c->b_dev + b->n_ins;
      del_s = c->b_dev + 2 * b->n_ins;
      del_d = c->b_dev + 2 * b->n_ins + b->n_del;
    }
  }
  // entries contributed by node deletions (exact count known after marking)
  int64_t T = 0;
  if (nd > 0) {
    if (nd + 1 > c->ndel_cap) {
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      dev_free(c, c->ndel);
      RWR_TRY(alloc_zero(c, &c->ndel, 2 * (int64_t)nd + 2));
      c->ndel_cap = 2 * (int64_t)nd + 2;
    }
    launch_node_mark(dn_dev, nd, c->perm, c->g[0].v, c->g[1].v, c->undirected ? 1 : 0, c->rows_only ? 1 : 0,
                     c->nmark, c->ndel, c->stream);
    std::vector<int64_t> cnt(nd), off(nd);
    D2H(c, cnt.data(), c->ndel, sizeof(int64_t) * nd);
    for (int32_t i = 0; i < nd; ++i) {
      off[i] = T;
      T += cnt[i];
    }
    H2D(c, c->ndel, off.data(), sizeof(int64_t) * nd);
  }
  const int64_t nkeys = c->undirected ? 2 * (N + T) : N + T;
  if (nkeys >= INT32_MAX) {
    if (nd > 0) launch_node_unmark(dn_dev, nd, c->perm, c->nmark, c->stream);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->err = "batch too large";
    return RWR_EINVAL;
  }
  RWR_TRY(ensure_batch(c, std::max<int64_t>(nkeys, 1), std::max<int64_t>(nints, 1)));
  c->big_batch = nkeys >= BIG_BATCH;
  const int b1 = bits_for(std::max(1, n_new - 1)) + 1;
  launch_reset_batch(c->ctl, 0, c->stream);

  const int norient = c->undirected ? 1 : 2;
  if (nkeys > 0) {
    launch_make_keys(ins_s, ins_d, b->n_ins, del_s, del_d, b->n_del, n_new, b1, c->undirected ? 1 : 0, c->perm,
                     nd > 0 ? c->nmark : nullptr, c->keys[0], c->keys[1], c->ctl, c->stream);
    if (nd > 0)
      launch_node_keys(dn_dev, nd, c->ndel, N, c->perm, c->g[0].v, c->g[1].v, c->undirected ? 1 : 0,
                       c->rows_only ? 1 : 0, c->nmark, b1, c->keys[0], c->keys[1], c->ctl, c->stream);
    if (nkeys <= SMALL_SORT_MAX) {
      launch_sort_segment_small(c->keys[0], c->keys[1], (int32_t)nkeys, b1, c->seg[0], c->row[0], c->seg[1],
                                c->row[1], norient, c->ctl, c->stream);
    } else {
      for (int o = 0; o < norient; ++o)
        HIP_TRY(c, sort_segment_large(c->keys[o], c->keys_alt, (int32_t)nkeys, b1, c->flags, c->pos, c->seg[o],
                                      c->row[o], c->temp, c->temp_bytes, c->ctl, o, c->stream));
    }
    launch_validate_plan(orient_pair(c, true), norient, b1, c->ctl, (int32_t)nkeys, c->stream);
  }
  if (nd > 0) launch_node_unmark(dn_dev, nd, c->perm, c->nmark, c->stream);
  RWR_TRY(read_ctl(c));
  if (c->ctl_h->err != 0) {
    const int e = c->ctl_h->err;
    c->err = e == ERR_EEXIST   ? "batch inserts an edge that exists"
             : e == ERR_ENOENT ? "batch deletes an edge that does not exist"
                               : "batch has an id out of range or a repeated entry";
    return (rwr_status)e;
  }
  // arena space for relocated rows; after a relayout the demand is recomputed
  // on the new layout (capacities changed)
  for (int round = 0;; ++round) {
    bool again = false;
    for (int o = 0; o < norient; ++o) {
      const int64_t need = (int64_t)c->ctl_h->tail[o] + c->ctl_h->demand[o];
      if (need > c->g[o].e_cap) {
        if (round > 0) {
          c->err = "relocation arena too small after relayout";
          return RWR_ENOMEM;
        }
        RWR_TRY(relayout(c, o, 2 * c->ctl_h->demand[o] + 65536));
        again = true;
      }
    }
    if (!again) break;
    launch_reset_batch(c->ctl, 1, c->stream);
    launch_validate_plan(orient_pair(c, false), norient, b1, c->ctl, (int32_t)nkeys, c->stream);
    RWR_TRY(read_ctl(c));
  }
  // the offset seed: scattered with FP64 atomics, or written as records that
  // are sorted and summed per node in a fixed order (deterministic mode, and
  // batches with many terms of many columns, where it is also faster: the
  // scatter issues S atomics per term, the sort moves one key)
  int64_t n_rec = 0;
  if (nkeys > 0 && seed_sort_possible(c)) {
    n_rec = nkeys;
    for (int i = 0; i < 32; ++i) n_rec += c->ctl_h->seed_recs[i];
  }
  c->seed_sorted = n_rec > 0 && (c->det || c->seed_sort_mode == 1 || n_rec >= SEED_SORT_MIN);
  if (c->seed_sorted && n_rec >= INT32_MAX) {
    if (c->det) {
      c->err = "batch too large for the deterministic offset seed (2^31 terms)";
      return RWR_EINVAL;
    }
    c->seed_sorted = false;
  }
  if (c->seed_sorted) RWR_TRY(ensure_seed_recs(c, n_rec));
  // the batch is valid: commit the node count and apply
  RWR_TRY(phase_mark(c, 1));
  c->n = n_new;
  const SlotArgs a = slot_args(c);
  const bool warm = c->ws.alloc && c->ws.mode != 0 && nkeys > 0;
  // a run that may leave its last iterate for the next update: its columns
  // retire together, so that every column leaves one (a column that stopped
  // earlier would otherwise spend its truncation bound)
  const bool keep = c->carry_level >= 2;
  launch_reset_run(c->ctl, c->S, all_cols_mask(c->n_seeds), c->cfg.eps, c->max_iters, dense_thresh(c),
                   c->n / 16 + 1, c->stream, 0, keep && c->lockstep ? 1 : 0);
  // carried vectors into gbuf (deferred last iterates unscaled with the
  // degrees before the batch; normally done at the end of the previous
  // update); the offset seed is that of r - p
  if (c->tail_slot >= 0) {
    const uint64_t tails = c->tail_slot >= 0 ? c->tail_cols : 0;
    launch_carry_prepare(a, c->S, c->fp64, c->tail_slot, tails, c->pend & ~tails, c->stream);
    c->pend |= tails;
    c->tail_slot = -1;
    c->tail_cols = 0;
  }
  // the offset seed of r - p
  const double *rsub = c->pend ? c->gbuf : nullptr;
  if (nkeys > 0)
    HIP_TRY(c, launch_offset_seed(c->S, c->keys[0], c->seg[0], c->row[0], c->t_dold[0], c->t_dnew[0], c->g[0].v,
                                  c->r, rsub, c->pend, c->seed_sorted ? nullptr : c->ybuf, c->stamp, c->ctl, b1,
                                  1.0 - c->cfg.c, (int32_t)nkeys, c->flags, c->pos,
                                  c->seed_sorted ? c->srec[0] : nullptr, c->sdcnt, c->sroff, c->temp,
                                  c->temp_bytes, 4 * c->n_cu, c->stream));
  if (c->seed_sorted) {
    const int64_t pl = seed_part_len(n_rec, c->S);
    HIP_TRY(c, launch_seed_sort_reduce(c->S, c->srec[0], c->srec[1], (int32_t)n_rec, (int32_t)nkeys, c->n, c->sroff,
                                       c->seg[0], c->row[0], c->t_dold[0], c->t_dnew[0], c->r, rsub, c->pend,
                                       1.0 - c->cfg.c,
                                       c->ybuf, c->spart, c->spart + pl, c->temp, c->temp_bytes, c->ctl,
                                       8 * c->n_cu, c->stream));
  }
  RWR_TRY(phase_mark(c, 2));
  if (nkeys > 0)
    launch_apply(orient_pair(c, false), norient, b1, c->ctl, (int32_t)nkeys, c->ctl_h->nbig_a, c->stream);
  RWR_TRY(phase_mark(c, 3));
  // stored edge count (an undirected self-loop is stored once; the count only
  // steers the sparse/dense switch and the visited-edge statistic)
  c->m += (b->n_ins - b->n_del) * (c->undirected ? 2 : 1) - c->ctl_h->node_dels;
  if (warm) RWR_TRY(warm_prepare(c));
  RWR_TRY(phase_mark(c, 4));
  launch_slot0_epilogue(a, c->S, c->fp64, c->stream);
  RWR_TRY(run_slots(c, MODE_SPARSE, -1.0, 0.0, keep, c->pend));
  RWR_TRY(phase_mark(c, 5));
  // columns whose pending vector joined the run (it reached the dense phase)
  uint64_t inj = 0;
  double cl = 0.0;
  for (int j = 0; j < c->n_seeds; ++j)
    if (((c->pend >> j) & 1ull) && c->ctl_h->inj[j]) {
      inj |= 1ull << j;
      cl = std::max(cl, c->pend_l1[j]);
    }
  c->last_carry_l1 = cl;
  c->pend &= ~inj;
  const double inc = account_run(c, false, inj);
  c->tail_ema = c->tail_ema < 0.0 ? inc : std::max(inc, 0.5 * (c->tail_ema + inc));
  fill_stats(c, st);
  if (st && warm) {
    st->ws_region = c->ws.nR;
    st->ws_accepted = c->ws.accepted;
    st->ws_resid_ratio = c->ws.ratio;
    st->fallback = c->ws.fallback;
    st->ws_loss = c->ws.loss;
    st->ms_warm = c->ws.ms;
  }
  rwr_status ret = RWR_OK;
  if (c->ctl_h->prop_err != 0) {
    c->stale = true;
    ret = (rwr_status)c->ctl_h->prop_err;
    c->err = ret == RWR_ENOCONV ? "max_iters reached before convergence" : "non-finite values during propagation";
  } else {
    RWR_TRY(check_and_refine(c, false, st));
  }
  if (c->ctl_h->heavy_stale > 0) RWR_TRY(plan_heavy(c));
  RWR_TRY(phase_mark(c, 6));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (st) {
    double worst = 0.0;
    for (int j = 0; j < c->n_seeds; ++j) worst = std::max(worst, c->err_bound[j]);
    st->err_bound = worst;
    st->ms_total = now_ms() - t0;
    if (c->cfg.phase_timing) {
      st->ms_delta = phase_ms(c, 0, 1) + phase_ms(c, 2, 3);
      st->ms_seed = phase_ms(c, 1, 2);
      st->ms_model = phase_ms(c, 3, 4);
      st->ms_prop = phase_ms(c, 4, 5);
      st->ms_merge = phase_ms(c, 5, 6);
    }
  }
  // A last iterate left in x is unscaled into gbuf now, with the degrees the
  // next batch starts from, so that this pass runs while the host prepares
  // the next call (it is not waited for here).
  if (ret == RWR_OK && c->tail_slot >= 0) {
    const SlotArgs an = slot_args(c);
    launch_carry_prepare(an, c->S, c->fp64, c->tail_slot, c->tail_cols, c->pend & ~c->tail_cols, c->stream);
    c->pend |= c->tail_cols;
    c->tail_slot = -1;
    c->tail_cols = 0;
  }
  return ret;
}

rwr_status rwr_refine(rwr_ctx *c, rwr_stats *st) {
  if (!c) return RWR_EINVAL;
  if (st) std::memset(st, 0, sizeof(*st));
  const double t0 = now_ms();
  c->stale = false;
  rwr_status s = check_and_refine(c, true, st, 0.125, 0.125);
  if (s != RWR_OK) return s;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (st) {
    double worst = 0.0;
    for (int j = 0; j < c->n_seeds; ++j) worst = std::max(worst, c->err_bound[j]);
    st->err_bound = worst;
    st->ms_total = now_ms() - t0;
  }
  return RWR_OK;
}

rwr_status rwr_scores(rwr_ctx *c, int32_t j, double *out, int64_t cap, int32_t out_on_device) {
  if (!c || !out || j < 0 || j >= c->n_seeds) return RWR_EINVAL;
  if (cap < c->n) {
    c->err = "output capacity below the node count";
    return RWR_EINVAL;
  }
  // staged in the residual sweep's scratch (gbuf may hold a carried residual)
  double *dst = out_on_device ? out : c->xres;
  launch_scores(c->r, c->ctl, c->perm, c->S, j, c->n, dst, c->stream);
  if (!out_on_device) HIP_TRY(c, hipMemcpyAsync(out, c->xres, sizeof(double) * c->n, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return RWR_OK;
}

rwr_status rwr_scores_set(rwr_ctx *c, int32_t j, const double *in, int64_t n, int32_t in_on_device) {
  if (!c || !in || j < 0 || j >= c->n_seeds) return RWR_EINVAL;
  if (n != c->n) {
    c->err = "score count differs from the node count";
    return RWR_EINVAL;
  }
  // the carried vectors belong to the scores being replaced
  drop_carry(c);
  const double *src = in;
  if (!in_on_device) {
    // staged in the residual sweep's scratch (free between calls)
    HIP_TRY(c, hipMemcpyAsync(c->xres, in, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    src = c->xres;
  }
  launch_set_scores(src, c->perm, c->S, j, c->n, c->r, c->stream);
  launch_sigma_exact(slot_args(c), c->S, c->stream);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->err_bound[j] = HUGE_VAL;
  return RWR_OK;
}

rwr_status rwr_graph_size(const rwr_ctx *c, int32_t *n, int64_t *m) {
  if (!c) return RWR_EINVAL;
  if (n) *n = c->n;
  if (m) *m = c->m;
  return RWR_OK;
}

rwr_status rwr_graph_export(rwr_ctx *c, int32_t *src, int32_t *dst, int64_t cap, int64_t *m_out, int32_t *deg_out) {
  if (!c) return RWR_EINVAL;
  std::vector<int32_t> len(c->n), perm(c->n);
  D2H(c, len.data(), c->g[0].v.len, sizeof(int32_t) * c->n);
  D2H(c, perm.data(), c->perm, sizeof(int32_t) * c->n);
  int64_t m = 0;
  for (int32_t v = 0; v < c->n; ++v) m += len[v];
  c->m = m;
  if (m_out) *m_out = m;
  if (deg_out)
    for (int32_t v = 0; v < c->n; ++v) deg_out[v] = len[perm[v]];
  if (!src || !dst) return RWR_OK;
  if (cap < m) {
    c->err = "export capacity below the edge count";
    return RWR_EINVAL;
  }
  int32_t *ds = nullptr, *dd = nullptr, *pos = nullptr;
  RWR_TRY(dev_alloc(c, (void **)&ds, sizeof(int32_t) * std::max<int64_t>(1, m)));
  RWR_TRY(dev_alloc(c, (void **)&dd, sizeof(int32_t) * std::max<int64_t>(1, m)));
  RWR_TRY(dev_alloc(c, (void **)&pos, sizeof(int32_t) * c->n_cap));
  RWR_TRY(ensure_temp(c, build_temp_bytes(1, c->n_cap)));
  HIP_TRY(c, export_rows(c->g[0].v, c->n, c->inv, ds, dd, pos, c->temp, c->temp_bytes, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  D2H(c, src, ds, sizeof(int32_t) * m);
  D2H(c, dst, dd, sizeof(int32_t) * m);
  dev_free(c, ds);
  dev_free(c, dd);
  dev_free(c, pos);
  return RWR_OK;
}

rwr_status rwr_last_norms(rwr_ctx *c, int32_t j, double *out, int32_t cap, int32_t *len) {
  if (!c || j < 0 || j >= c->n_seeds || !len) return RWR_EINVAL;
  const int32_t total = c->last_iters + 1;
  if (!c->hist_host_valid) {
    // the device history of the last run, copied on first request
    c->last_hist.assign((size_t)total * c->S, 0.0);
    HIP_TRY(c, hipMemcpyAsync(c->last_hist.data(), c->hist, sizeof(double) * c->last_hist.size(),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->hist_host_valid = true;
  }
  const int32_t k = std::min(cap, total);
  for (int32_t i = 0; i < k && out; ++i) out[i] = c->last_hist[(size_t)i * c->S + j];
  *len = total;
  return RWR_OK;
}

void rwr_destroy(rwr_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  warm_free(c);
  const int no = c->undirected ? 1 : 2;
  for (int o = 0; o < no; ++o) {
    dev_free(c, c->g[o].v.off);
    dev_free(c, c->g[o].v.len);
    dev_free(c, c->g[o].v.cap);
    dev_free(c, c->g[o].v.adj);
    dev_free(c, c->g[o].v.heavy);
  }
  dev_free(c, c->r);
  dev_free(c, c->ybuf);
  dev_free(c, c->gbuf);
  dev_free(c, c->xres);
  dev_free(c, c->qvec);
  dev_free(c, c->x[0]);
  dev_free(c, c->x[1]);
  dev_free(c, c->stamp);
  dev_free(c, c->fstamp);
  dev_free(c, c->nmark);
  dev_free(c, c->srec[0]);
  dev_free(c, c->srec[1]);
  dev_free(c, c->spart);
  dev_free(c, c->sdcnt);
  dev_free(c, c->sroff);
  dev_free(c, c->bigv);
  dev_free(c, c->biga);
  dev_free(c, c->ndel);
  dev_free(c, c->row_order);
  dev_free(c, c->hfront);
  dev_free(c, c->hbase);
  dev_free(c, c->ctl);
  dev_free(c, c->hist);
  dev_free(c, c->part);
  dev_free(c, c->part_i);
  dev_free(c, c->h_item_row);
  dev_free(c, c->h_item_chunk);
  dev_free(c, c->h_rows);
  dev_free(c, c->h_nchunks);
  dev_free(c, c->h_first);
  dev_free(c, c->h_part);
  dev_free(c, c->sel);
  dev_free(c, c->sel_count);
  dev_free(c, c->mp_rows);
  dev_free(c, c->seeds_d);
  dev_free(c, c->perm);
  dev_free(c, c->inv);
  dev_free(c, c->b_dev);
  for (int o = 0; o < 2; ++o) {
    dev_free(c, c->keys[o]);
    dev_free(c, c->seg[o]);
    dev_free(c, c->row[o]);
    dev_free(c, c->t_dold[o]);
    dev_free(c, c->t_dnew[o]);
  }
  dev_free(c, c->keys_alt);
  dev_free(c, c->flags);
  dev_free(c, c->pos);
  dev_free(c, c->temp);
  if (c->b_host) (void)hipHostFree(c->b_host);
  if (c->ctl_h) (void)hipHostFree(c->ctl_h);
  for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->tune.ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ph_ev)
    if (e) (void)hipEventDestroy(e);
  pair_graph_drop(c);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

rwr_status rwr_profile(rwr_ctx *c, int32_t enable) {
  if (!c) return RWR_EINVAL;
  c->prof_on = enable != 0;
  return RWR_OK;
}

rwr_status rwr_profile_read(rwr_ctx *c, double *dense_ms, int64_t *dense_sweeps, int64_t *idle_launches,
                            int32_t reset) {
  if (!c) return RWR_EINVAL;
  if (dense_ms) *dense_ms = c->prof_dense_ms;
  if (dense_sweeps) *dense_sweeps = c->prof_dense_sweeps;
  if (idle_launches) *idle_launches = c->prof_idle;
  if (reset) {
    c->prof_dense_ms = 0.0;
    c->prof_dense_sweeps = 0;
    c->prof_idle = 0;
  }
  return RWR_OK;
}

const char *rwr_last_error(const rwr_ctx *c) { return c ? c->err.c_str() : g_build_error.c_str(); }

rwr_status rwr_context_info(const rwr_ctx *c, rwr_config *cfg, int32_t *n_seeds, int32_t *seeds) {
  if (!c) return RWR_EINVAL;
  if (cfg) *cfg = c->cfg;
  if (n_seeds) *n_seeds = c->n_seeds;
  if (seeds) {
    for (int32_t j = 0; j < c->n_seeds; ++j) seeds[j] = c->qmode ? -1 : c->seeds_h[j];
  }
  return RWR_OK;
}

// ------------------------------------------------------------------ checkpoint
// A checkpoint holds what the next update reads, in the context's internal
// layout: node numbering, each row's entries in storage order, the heavy-row,
// row-order and partition plans and the sweep shape, so that a loaded context
// repeats the saved one's arithmetic exactly.  Native byte order: CkptHead,
// then the sections in the order rwr_save writes them.
namespace {
constexpr char CKPT_MAGIC[8] = {'R', 'W', 'R', 'C', 'K', 'P', 'T', '1'};
constexpr uint32_t CKPT_VERSION = 1;
struct CkptHead {
  char magic[8];
  uint32_t version, head_bytes, cfg_bytes, ctl_bytes;
  rwr_config cfg;  // runtime fields (stream, allocator hooks, user pointer) cleared
  int32_t n, n_cap, n_seeds, S, max_iters, solve_iters;
  int64_t m;
  int64_t m_o[2];  // stored entries per orientation
  int32_t undirected, fp64, rows_only, det, qmode, stale, lockstep, carry_level;
  int32_t tail_slot, update_runs, last_iters, pad0;
  uint64_t pend, tail_cols;
  double budget, refine_target, decay_ema, sparse_ema, dense_ema, last_carry_l1, tail_ema;
  double err_bound[RWR_MAX_COLS], pend_b[RWR_MAX_COLS], pend_l1[RWR_MAX_COLS];
  int32_t grid_sparse, grid_light, grid_pull, light_lanes, pull_lanes, pull_ratio;
  int32_t heavy_limit, heavy_chunk, fold_max, h_items, h_nrows, n_mp, has_order, pad1;
  // learned warm start
  int32_t ws_alloc, ws_params, ws_mode, ws_hops, ws_warmup, ws_has_mask;
  int64_t ws_max_rows, ws_step;
  float ws_lr, ws_wd;
};

struct File {
  FILE *f = nullptr;
  ~File() {
    if (f) std::fclose(f);
  }
};
}  // namespace

#define CK_IO(c, ok, what)               \
  do {                                   \
    if (!(ok)) {                         \
      (c)->err = std::string(what);      \
      return RWR_EIO;                    \
    }                                    \
  } while (0)

// device range -> file (staged through host memory)
static rwr_status ck_put_dev(rwr_ctx *c, FILE *f, const void *dev, size_t bytes) {
  if (bytes == 0) return RWR_OK;
  std::vector<char> h(bytes);
  D2H(c, h.data(), dev, bytes);
  CK_IO(c, std::fwrite(h.data(), 1, bytes, f) == bytes, "checkpoint write failed");
  return RWR_OK;
}

static rwr_status ck_get_dev(rwr_ctx *c, FILE *f, void *dev, size_t bytes) {
  if (bytes == 0) return RWR_OK;
  std::vector<char> h(bytes);
  CK_IO(c, std::fread(h.data(), 1, bytes, f) == bytes, "checkpoint truncated");
  H2D(c, dev, h.data(), bytes);
  return RWR_OK;
}

rwr_status rwr_save(rwr_ctx *c, const char *path) {
  if (!c || !path) return RWR_EINVAL;
  if (!c->built) {
    c->err = "context not built";
    return RWR_ESTATE;
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  RWR_TRY(read_ctl(c));
  const int no = c->undirected ? 1 : 2;
  const size_t nS = (size_t)c->n * c->S;
  const size_t xs = c->fp64 ? 8 : 4;
  // rows of each orientation, compacted in storage order
  std::vector<std::vector<int32_t>> lens(no), adjs(no);
  for (int o = 0; o < no; ++o) {
    lens[o].resize(c->n);
    D2H(c, lens[o].data(), c->g[o].v.len, sizeof(int32_t) * c->n);
    std::vector<int32_t> coff(std::max(1, c->n));
    int64_t acc = 0;
    for (int32_t v = 0; v < c->n; ++v) {
      coff[v] = (int32_t)acc;
      acc += lens[o][v];
    }
    adjs[o].resize(acc);
    if (acc > 0) {
      int32_t *doff = nullptr, *dadj = nullptr;
      RWR_TRY(dev_alloc(c, (void **)&doff, sizeof(int32_t) * coff.size()));
      rwr_status s = dev_alloc(c, (void **)&dadj, sizeof(int32_t) * acc);
      if (s == RWR_OK) s = copy_sync(c, doff, coff.data(), sizeof(int32_t) * coff.size(), hipMemcpyHostToDevice);
      if (s == RWR_OK) {
        launch_copy_rows(c->g[o].v, doff, dadj, c->n, c->stream);
        s = copy_sync(c, adjs[o].data(), dadj, sizeof(int32_t) * acc, hipMemcpyDeviceToHost);
      }
      dev_free(c, doff);
      dev_free(c, dadj);
      RWR_TRY(s);
    }
  }
  CkptHead h{};
  std::memcpy(h.magic, CKPT_MAGIC, 8);
  h.version = CKPT_VERSION;
  h.head_bytes = sizeof(CkptHead);
  h.cfg_bytes = sizeof(rwr_config);
  h.ctl_bytes = sizeof(Ctl);
  h.cfg = c->cfg;
  h.cfg.stream = nullptr;
  h.cfg.dev_alloc = nullptr;
  h.cfg.dev_free = nullptr;
  h.cfg.alloc_user = nullptr;
  h.n = c->n;
  h.n_cap = c->n_cap;
  h.n_seeds = c->n_seeds;
  h.S = c->S;
  h.max_iters = c->max_iters;
  h.solve_iters = c->solve_iters;
  h.m = c->m;
  for (int o = 0; o < no; ++o) h.m_o[o] = (int64_t)adjs[o].size();
  h.undirected = c->undirected;
  h.fp64 = c->fp64;
  h.rows_only = c->rows_only;
  h.det = c->det;
  h.qmode = c->qmode;
  h.stale = c->stale;
  h.lockstep = c->lockstep;
  h.carry_level = c->carry_level;
  h.tail_slot = c->tail_slot;
  h.update_runs = c->update_runs;
  h.last_iters = c->last_iters;
  h.pend = c->pend;
  h.tail_cols = c->tail_cols;
  h.budget = c->budget;
  h.refine_target = c->refine_target;
  h.decay_ema = c->decay_ema;
  h.sparse_ema = c->sparse_ema;
  h.dense_ema = c->dense_ema;
  h.last_carry_l1 = c->last_carry_l1;
  h.tail_ema = c->tail_ema;
  std::memcpy(h.err_bound, c->err_bound, sizeof(h.err_bound));
  std::memcpy(h.pend_b, c->pend_b, sizeof(h.pend_b));
  std::memcpy(h.pend_l1, c->pend_l1, sizeof(h.pend_l1));
  h.grid_sparse = c->grid_sparse;
  h.grid_light = c->grid_light;
  h.grid_pull = c->grid_pull;
  h.light_lanes = c->light_lanes;
  h.pull_lanes = c->pull_lanes;
  h.pull_ratio = c->pull_ratio;
  h.heavy_limit = c->heavy_limit;
  h.heavy_chunk = c->heavy_chunk;
  h.fold_max = c->fold_max;
  h.h_items = c->h_items;
  h.h_nrows = c->h_nrows;
  h.n_mp = c->mp_rows ? c->n_mp : -1;
  h.has_order = c->row_order ? 1 : 0;
  const rwr_ctx::Warm &w = c->ws;
  h.ws_alloc = w.alloc;
  h.ws_params = w.params;
  h.ws_mode = w.mode;
  h.ws_hops = w.hops;
  h.ws_warmup = w.warmup;
  h.ws_has_mask = !w.mask_h.empty();
  h.ws_max_rows = w.max_rows;
  h.ws_step = w.net.step;
  h.ws_lr = w.net.lr;
  h.ws_wd = w.net.wd;

  const std::string tmp = std::string(path) + ".part";
  File F;
  F.f = std::fopen(tmp.c_str(), "wb");
  CK_IO(c, F.f, "cannot open " + tmp + " for writing");
  FILE *f = F.f;
  auto put = [&](const void *p, size_t bytes) { return bytes == 0 || std::fwrite(p, 1, bytes, f) == bytes; };
  CK_IO(c, put(&h, sizeof(h)), "checkpoint write failed");
  CK_IO(c, put(c->seeds_h.data(), sizeof(int32_t) * c->seeds_h.size()), "checkpoint write failed");
  CK_IO(c, put(c->ctl_h, sizeof(Ctl)), "checkpoint write failed");
  RWR_TRY(ck_put_dev(c, f, c->seeds_d, sizeof(int32_t) * RWR_MAX_COLS));
  RWR_TRY(ck_put_dev(c, f, c->perm, sizeof(int32_t) * c->n_cap));
  RWR_TRY(ck_put_dev(c, f, c->inv, sizeof(int32_t) * c->n_cap));
  RWR_TRY(ck_put_dev(c, f, c->r, sizeof(double) * nS));
  RWR_TRY(ck_put_dev(c, f, c->gbuf, sizeof(double) * nS));
  if (c->qmode) RWR_TRY(ck_put_dev(c, f, c->qvec, sizeof(double) * nS));
  if (c->tail_slot >= 0) RWR_TRY(ck_put_dev(c, f, c->x[c->tail_slot], xs * nS));
  for (int o = 0; o < no; ++o) {
    CK_IO(c, put(lens[o].data(), sizeof(int32_t) * lens[o].size()), "checkpoint write failed");
    CK_IO(c, put(adjs[o].data(), sizeof(int32_t) * adjs[o].size()), "checkpoint write failed");
    RWR_TRY(ck_put_dev(c, f, c->g[o].v.heavy, c->n_cap));
  }
  RWR_TRY(ck_put_dev(c, f, c->h_item_row, sizeof(int32_t) * c->h_items));
  RWR_TRY(ck_put_dev(c, f, c->h_item_chunk, sizeof(int32_t) * c->h_items));
  RWR_TRY(ck_put_dev(c, f, c->h_rows, sizeof(int32_t) * c->h_nrows));
  RWR_TRY(ck_put_dev(c, f, c->h_nchunks, sizeof(int32_t) * c->h_nrows));
  RWR_TRY(ck_put_dev(c, f, c->h_first, sizeof(int32_t) * c->h_nrows));
  if (h.has_order) RWR_TRY(ck_put_dev(c, f, c->row_order, sizeof(int32_t) * c->n_cap));
  if (h.n_mp >= 0) RWR_TRY(ck_put_dev(c, f, c->mp_rows, sizeof(int32_t) * (c->n_mp + 1)));
  if (w.alloc && w.params) {
    const size_t P = sizeof(float) * gnn::LAYOUT.total;
    RWR_TRY(ck_put_dev(c, f, w.net.theta, P));
    RWR_TRY(ck_put_dev(c, f, w.net.m1, P));
    RWR_TRY(ck_put_dev(c, f, w.net.m2, P));
  }
  if (h.ws_has_mask) CK_IO(c, put(w.mask_h.data(), sizeof(float) * w.mask_h.size()), "checkpoint write failed");
  CK_IO(c, std::fflush(f) == 0, "checkpoint write failed");
  std::fclose(F.f);
  F.f = nullptr;
  CK_IO(c, std::rename(tmp.c_str(), path) == 0, "cannot rename " + tmp + " to " + path);
  return RWR_OK;
}

static rwr_status load_impl(rwr_ctx *c, FILE *f, const CkptHead &h) {
  auto get = [&](void *p, size_t bytes) { return bytes == 0 || std::fread(p, 1, bytes, f) == bytes; };
  HIP_TRY(c, hipGetDevice(&c->device));
  HIP_TRY(c, hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device));
  if (c->cfg.stream) {
    c->stream = (hipStream_t)c->cfg.stream;
  } else {
    HIP_TRY(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
  }
  c->n = h.n;
  c->n_cap = h.n_cap;
  c->m = h.m;
  c->n_seeds = h.n_seeds;
  c->S = h.S;
  c->max_iters = h.max_iters;
  c->solve_iters = h.solve_iters;
  c->undirected = h.undirected;
  c->fp64 = h.fp64;
  c->rows_only = h.rows_only;
  c->det = h.det;
  c->qmode = h.qmode;
  c->stale = h.stale;
  c->lockstep = h.lockstep;
  c->carry_level = h.carry_level;
  c->tail_slot = h.tail_slot;
  c->update_runs = h.update_runs;
  c->last_iters = h.last_iters;
  c->pend = h.pend;
  c->tail_cols = h.tail_cols;
  c->budget = h.budget;
  c->refine_target = h.refine_target;
  c->decay_ema = h.decay_ema;
  c->sparse_ema = h.sparse_ema;
  c->dense_ema = h.dense_ema;
  c->last_carry_l1 = h.last_carry_l1;
  c->tail_ema = h.tail_ema;
  std::memcpy(c->err_bound, h.err_bound, sizeof(h.err_bound));
  std::memcpy(c->pend_b, h.pend_b, sizeof(h.pend_b));
  std::memcpy(c->pend_l1, h.pend_l1, sizeof(h.pend_l1));
  tune_defaults(c);  // settings that only the environment sets (graph replay, ...)
  c->grid_sparse = h.grid_sparse;
  c->grid_light = h.grid_light;
  c->grid_pull = h.grid_pull;
  c->light_lanes = h.light_lanes;
  c->pull_lanes = h.pull_lanes;
  c->pull_ratio = h.pull_ratio;
  c->heavy_limit = h.heavy_limit;
  c->heavy_chunk = h.heavy_chunk;
  c->fold_max = h.fold_max;
  c->lockstep = h.lockstep;
  c->carry_level = h.carry_level;
  c->refine_target = h.refine_target;
  const int no = c->undirected ? 1 : 2;
  const size_t nS = (size_t)c->n * c->S, nSc = (size_t)c->n_cap * c->S;
  const size_t xs = c->fp64 ? 8 : 4;

  c->seeds_h.resize(h.n_seeds);
  CK_IO(c, get(c->seeds_h.data(), sizeof(int32_t) * h.n_seeds), "checkpoint truncated");
  HIP_TRY(c, hipHostMalloc((void **)&c->ctl_h, sizeof(Ctl), hipHostMallocDefault));
  CK_IO(c, get(c->ctl_h, sizeof(Ctl)), "checkpoint truncated");
  RWR_TRY(alloc_zero(c, &c->ctl, 1));
  RWR_TRY(alloc_zero(c, &c->seeds_d, RWR_MAX_COLS));
  RWR_TRY(ck_get_dev(c, f, c->seeds_d, sizeof(int32_t) * RWR_MAX_COLS));
  RWR_TRY(alloc_zero(c, &c->perm, c->n_cap));
  RWR_TRY(alloc_zero(c, &c->inv, c->n_cap));
  RWR_TRY(ck_get_dev(c, f, c->perm, sizeof(int32_t) * c->n_cap));
  RWR_TRY(ck_get_dev(c, f, c->inv, sizeof(int32_t) * c->n_cap));
  RWR_TRY(alloc_zero(c, &c->r, nSc));
  RWR_TRY(alloc_zero(c, &c->ybuf, nSc));
  RWR_TRY(alloc_zero(c, &c->gbuf, nSc));
  RWR_TRY(alloc_zero(c, &c->xres, nSc));
  RWR_TRY(ck_get_dev(c, f, c->r, sizeof(double) * nS));
  RWR_TRY(ck_get_dev(c, f, c->gbuf, sizeof(double) * nS));
  if (c->qmode) {
    RWR_TRY(alloc_zero(c, &c->qvec, nSc));
    RWR_TRY(ck_get_dev(c, f, c->qvec, sizeof(double) * nS));
  }
  RWR_TRY(dev_alloc(c, &c->x[0], xs * nSc));
  RWR_TRY(dev_alloc(c, &c->x[1], xs * nSc));
  launch_zero_bytes(c->x[0], xs * nSc, c->stream);
  launch_zero_bytes(c->x[1], xs * nSc, c->stream);
  if (c->tail_slot >= 0) RWR_TRY(ck_get_dev(c, f, c->x[c->tail_slot], xs * nS));

  // graph: each orientation laid out afresh (slack per row and an arena, as
  // a relayout makes them) with the saved row contents
  RWR_TRY(ensure_temp(c, build_temp_bytes(1, c->n_cap)));
  for (int o = 0; o < no; ++o) {
    Orientation &g = c->g[o];
    RWR_TRY(alloc_zero(c, &g.v.off, c->n_cap));
    RWR_TRY(alloc_zero(c, &g.v.len, c->n_cap));
    RWR_TRY(alloc_zero(c, &g.v.cap, c->n_cap));
    RWR_TRY(alloc_zero(c, &g.v.heavy, c->n_cap));
    std::vector<int32_t> len(c->n), adj(h.m_o[o]);
    CK_IO(c, get(len.data(), sizeof(int32_t) * len.size()), "checkpoint truncated");
    CK_IO(c, get(adj.data(), sizeof(int32_t) * adj.size()), "checkpoint truncated");
    std::vector<int32_t> coff(std::max(1, c->n));
    int64_t acc = 0;
    for (int32_t v = 0; v < c->n; ++v) {
      if (len[v] < 0) CK_IO(c, false, "checkpoint corrupt (row length)");
      coff[v] = (int32_t)acc;
      acc += len[v];
    }
    CK_IO(c, acc == h.m_o[o], "checkpoint corrupt (edge count)");
    for (int32_t x : adj) CK_IO(c, x >= 0 && x < c->n, "checkpoint corrupt (node id)");
    H2D(c, g.v.len, len.data(), sizeof(int32_t) * c->n);
    int64_t used = 0;
    HIP_TRY(c, relayout_offsets(g.v.len, c->n, g.v.cap, g.v.off, c->temp, c->temp_bytes, &used, c->stream));
    g.e_cap = used + std::max<int64_t>(used / 4, 65536);
    if (g.e_cap >= INT32_MAX) {
      c->err = "adjacency capacity exceeds 2^31 slots";
      return RWR_ENOMEM;
    }
    RWR_TRY(dev_alloc(c, (void **)&g.v.adj, sizeof(int32_t) * g.e_cap));
    if (acc > 0) {
      int32_t *doff = nullptr, *dadj = nullptr;
      RWR_TRY(dev_alloc(c, (void **)&doff, sizeof(int32_t) * coff.size()));
      rwr_status s = dev_alloc(c, (void **)&dadj, sizeof(int32_t) * acc);
      if (s == RWR_OK) s = copy_sync(c, doff, coff.data(), sizeof(int32_t) * coff.size(), hipMemcpyHostToDevice);
      if (s == RWR_OK) s = copy_sync(c, dadj, adj.data(), sizeof(int32_t) * acc, hipMemcpyHostToDevice);
      if (s == RWR_OK) {
        DevGraphView src = g.v;
        src.off = doff;
        src.adj = dadj;
        launch_copy_rows(src, g.v.off, g.v.adj, c->n, c->stream);
        if (hipStreamSynchronize(c->stream) != hipSuccess) s = RWR_EHIP;
      }
      dev_free(c, doff);
      dev_free(c, dadj);
      RWR_TRY(s);
    }
    RWR_TRY(ck_get_dev(c, f, g.v.heavy, c->n_cap));
    c->ctl_h->tail[o] = (uint64_t)used;
  }
  if (c->undirected) c->g[1] = c->g[0];
  Ctl ctl = *c->ctl_h;
  ctl.err = 0;
  ctl.done_blocks = 0;
  H2D(c, c->ctl, &ctl, sizeof(Ctl));

  RWR_TRY(alloc_zero(c, &c->stamp, c->n_cap));
  RWR_TRY(alloc_zero(c, &c->fstamp, c->n_cap));
  RWR_TRY(alloc_zero(c, &c->nmark, c->n_cap));
  RWR_TRY(alloc_zero(c, &c->hfront, c->n_cap));
  RWR_TRY(alloc_zero(c, &c->hbase, c->n_cap));
  RWR_TRY(alloc_zero(c, &c->sel, (size_t)c->n_cap * 2));
  RWR_TRY(alloc_zero(c, &c->sel_count, 1));
  RWR_TRY(alloc_zero(c, &c->hist, (size_t)(c->max_iters + 2 + c->solve_iters + 2) * c->S));

  // plans as saved
  c->h_items = h.h_items;
  c->h_nrows = h.h_nrows;
  RWR_TRY(alloc_zero(c, &c->h_item_row, std::max(1, h.h_items)));
  RWR_TRY(alloc_zero(c, &c->h_item_chunk, std::max(1, h.h_items)));
  RWR_TRY(alloc_zero(c, &c->h_rows, std::max(1, h.h_nrows)));
  RWR_TRY(alloc_zero(c, &c->h_nchunks, std::max(1, h.h_nrows)));
  RWR_TRY(alloc_zero(c, &c->h_first, std::max(1, h.h_nrows)));
  RWR_TRY(alloc_zero(c, &c->h_part, (size_t)std::max(1, h.h_items) * c->S));
  RWR_TRY(ck_get_dev(c, f, c->h_item_row, sizeof(int32_t) * h.h_items));
  RWR_TRY(ck_get_dev(c, f, c->h_item_chunk, sizeof(int32_t) * h.h_items));
  RWR_TRY(ck_get_dev(c, f, c->h_rows, sizeof(int32_t) * h.h_nrows));
  RWR_TRY(ck_get_dev(c, f, c->h_nchunks, sizeof(int32_t) * h.h_nrows));
  RWR_TRY(ck_get_dev(c, f, c->h_first, sizeof(int32_t) * h.h_nrows));
  if (h.has_order) {
    RWR_TRY(alloc_zero(c, &c->row_order, c->n_cap));
    RWR_TRY(ck_get_dev(c, f, c->row_order, sizeof(int32_t) * c->n_cap));
  }
  if (h.n_mp >= 0) {
    c->n_mp = h.n_mp;
    RWR_TRY(dev_alloc(c, (void **)&c->mp_rows, sizeof(int32_t) * (h.n_mp + 1)));
    RWR_TRY(ck_get_dev(c, f, c->mp_rows, sizeof(int32_t) * (h.n_mp + 1)));
  }
  RWR_TRY(ensure_partials(c));

  // learned warm start
  if (h.ws_alloc) {
    RWR_TRY(warm_alloc(c, h.ws_max_rows));
    rwr_ctx::Warm &w = c->ws;
    if (h.ws_params) {
      const int64_t P = gnn::LAYOUT.total;
      std::vector<float> th(P);
      CK_IO(c, get(th.data(), sizeof(float) * P), "checkpoint truncated");
      HIP_TRY(c, gnn::net_set_params(w.net, th.data(), c->stream));
      RWR_TRY(ck_get_dev(c, f, w.net.m1, sizeof(float) * P));
      RWR_TRY(ck_get_dev(c, f, w.net.m2, sizeof(float) * P));
      w.net.step = h.ws_step;
      w.params = true;
    }
    w.mode = h.ws_mode;
    w.hops = h.ws_hops;
    w.warmup = h.ws_warmup;
    w.net.warmup = h.ws_warmup;
    w.net.lr = h.ws_lr;
    w.net.wd = h.ws_wd;
  }
  if (h.ws_has_mask) {
    c->ws.mask_h.resize(gnn::LAYOUT.total);
    CK_IO(c, get(c->ws.mask_h.data(), sizeof(float) * gnn::LAYOUT.total), "checkpoint truncated");
    if (c->ws.alloc) RWR_TRY(warm_set_mask(c, c->ws.mask_h.data()));
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return RWR_OK;
}

rwr_status rwr_load(const char *path, const rwr_config *runtime, rwr_ctx **out) {
  if (!path || !out) return RWR_EINVAL;
  *out = nullptr;
  g_build_error.clear();
  if (runtime && ((runtime->dev_alloc == nullptr) != (runtime->dev_free == nullptr))) {
    g_build_error = "dev_alloc and dev_free must be given together";
    return RWR_EINVAL;
  }
  File F;
  F.f = std::fopen(path, "rb");
  if (!F.f) {
    g_build_error = std::string("cannot open ") + path;
    return RWR_EIO;
  }
  CkptHead h{};
  if (std::fread(&h, 1, sizeof(h), F.f) != sizeof(h) || std::memcmp(h.magic, CKPT_MAGIC, 8) != 0 ||
      h.version != CKPT_VERSION || h.head_bytes != sizeof(CkptHead) || h.cfg_bytes != sizeof(rwr_config) ||
      h.ctl_bytes != sizeof(Ctl)) {
    g_build_error = std::string(path) + " is not a checkpoint of this library version";
    return RWR_EIO;
  }
  if (h.n <= 0 || h.n > h.n_cap || h.n_seeds < 1 || h.n_seeds > RWR_MAX_COLS || h.S < h.n_seeds ||
      h.S > RWR_MAX_COLS || h.m_o[0] < 0 || h.m_o[1] < 0 || h.h_items < 0 || h.h_nrows < 0 ||
      h.m_o[0] > INT32_MAX || h.m_o[1] > INT32_MAX || h.tail_slot < -1 || h.tail_slot > 1) {
    g_build_error = std::string(path) + ": corrupt header";
    return RWR_EIO;
  }
  rwr_ctx *c = new rwr_ctx();
  c->cfg = h.cfg;
  if (runtime) {
    c->cfg.stream = runtime->stream;
    c->cfg.dev_alloc = runtime->dev_alloc;
    c->cfg.dev_free = runtime->dev_free;
    c->cfg.alloc_user = runtime->alloc_user;
    c->cfg.phase_timing = runtime->phase_timing;
  }
  rwr_status s = load_impl(c, F.f, h);
  if (s != RWR_OK) {
    g_build_error = c->err;
    rwr_destroy(c);
    return s;
  }
  c->built = true;
  *out = c;
  return RWR_OK;
}

rwr_status rwr_sweep_shape(const rwr_ctx *c, int32_t *lanes_per_row, int32_t *workgroups, double *tuned_ms) {
  if (!c) return RWR_EINVAL;
  if (lanes_per_row) *lanes_per_row = c->pull_lanes;
  if (workgroups) *workgroups = c->grid_pull;
  if (tuned_ms) *tuned_ms = c->tune.best_ms;
  return RWR_OK;
}

int64_t rwr_gnn_num_params(void) { return gnn::LAYOUT.total; }

rwr_status rwr_warm_start(rwr_ctx *c, int32_t mode, int32_t hops, int64_t max_rows, float lr, float weight_decay) {
  if (!c) return RWR_EINVAL;
  if (mode < 0 || mode > 3 || hops < 0 || hops > 8 || max_rows < 0 || !(lr >= 0.0f) || !(weight_decay >= 0.0f)) {
    c->err = "invalid warm-start settings";
    return RWR_EINVAL;
  }
  if (mode == 0) {
    c->ws.mode = 0;
    return RWR_OK;
  }
  if (c->qmode) {
    c->err = "the learned warm start needs seed nodes (its features mark them)";
    return RWR_ESTATE;
  }
  const int64_t rows = max_rows > 0 ? max_rows : ((int64_t)1 << 21);
  if (c->ws.alloc && rows != c->ws.max_rows) {
    std::vector<float> keep;
    if (c->ws.params) {
      keep.resize(gnn::LAYOUT.total);
      HIP_TRY(c, gnn::net_get_params(c->ws.net, keep.data(), c->stream));
    }
    std::vector<float> mask = c->ws.mask_h;
    const int32_t warmup = c->ws.warmup;
    warm_free(c);
    RWR_TRY(warm_alloc(c, rows));
    if (!keep.empty()) {
      HIP_TRY(c, gnn::net_set_params(c->ws.net, keep.data(), c->stream));
      c->ws.params = true;
    }
    c->ws.mask_h = mask;
    c->ws.warmup = warmup;
    c->ws.net.warmup = warmup;
    if (!mask.empty()) RWR_TRY(warm_set_mask(c, mask.data()));
  } else if (!c->ws.alloc) {
    RWR_TRY(warm_alloc(c, rows));
  }
  if (!c->ws.params) {
    c->err = "warm start needs parameters (rwr_model_set) first";
    c->ws.mode = 0;
    return RWR_ESTATE;
  }
  c->ws.mode = mode;
  c->ws.hops = hops;
  c->ws.net.lr = lr;
  c->ws.net.wd = weight_decay;
  return RWR_OK;
}

rwr_status rwr_model_set(rwr_ctx *c, const float *params, int64_t n) {
  if (!c || !params || n != gnn::LAYOUT.total) return RWR_EINVAL;
  if (!c->ws.alloc) RWR_TRY(warm_alloc(c, (int64_t)1 << 21));
  HIP_TRY(c, gnn::net_set_params(c->ws.net, params, c->stream));
  c->ws.params = true;
  return RWR_OK;
}

rwr_status rwr_model_trainable(rwr_ctx *c, const float *mask, int64_t n, int32_t warmup_steps) {
  if (!c || (mask && n != gnn::LAYOUT.total) || warmup_steps < 0) return RWR_EINVAL;
  if (!c->ws.alloc) RWR_TRY(warm_alloc(c, (int64_t)1 << 21));
  if (mask)
    c->ws.mask_h.assign(mask, mask + n);
  else
    c->ws.mask_h.clear();
  c->ws.warmup = warmup_steps;
  c->ws.net.warmup = warmup_steps;
  RWR_TRY(warm_set_mask(c, mask ? c->ws.mask_h.data() : nullptr));
  return RWR_OK;
}

rwr_status rwr_model_get(rwr_ctx *c, float *params, int64_t cap) {
  if (!c || !params || cap < gnn::LAYOUT.total) return RWR_EINVAL;
  if (!c->ws.params) {
    c->err = "no model parameters set";
    return RWR_ESTATE;
  }
  HIP_TRY(c, gnn::net_get_params(c->ws.net, params, c->stream));
  return RWR_OK;
}

rwr_status rwr_warm_inspect(rwr_ctx *c, int32_t *nodes, int32_t *hops, float *o, float *dout, float *grad,
                            int64_t cap, int32_t *n_region, int32_t *row_cols) {
  if (!c || !n_region) return RWR_EINVAL;
  const rwr_ctx::Warm &w = c->ws;
  *n_region = w.alloc ? w.nR : 0;
  if (row_cols) *row_cols = c->S;
  if (!w.alloc || w.nR == 0) return RWR_OK;
  if ((dout || grad) && !w.trained) {
    c->err = "the last update took no training step";
    return RWR_ESTATE;
  }
  if ((nodes || hops || o || dout) && cap < w.nR) {
    c->err = "inspection capacity below the region size";
    return RWR_EINVAL;
  }
  const int64_t rows = (int64_t)w.nR * c->S;
  if (nodes) {
    // region rows in caller ids (wlist is free between updates)
    launch_gather_i32(c->inv, w.R, w.nR, w.wlist, c->stream);
    D2H(c, nodes, w.wlist, sizeof(int32_t) * w.nR);
  }
  if (hops) {
    int32_t h = 0;
    for (int32_t i = 0; i < w.nR; ++i) {
      while (h < (int32_t)w.level_end.size() && i >= w.level_end[h]) ++h;
      hops[i] = h;
    }
  }
  if (o) D2H(c, o, w.net.o, sizeof(float) * rows);
  if (dout) D2H(c, dout, w.net.dout, sizeof(float) * rows);
  if (grad) D2H(c, grad, w.net.grad, sizeof(float) * gnn::LAYOUT.total);
  return RWR_OK;
}

rwr_status rwr_gnn_eval_noalloc(const float *params, int32_t nR, int32_t S, const int32_t *in_off,
                                const int32_t *in_len, const int32_t *in_adj, int64_t n_in, const int32_t *out_off,
                                const int32_t *out_len, const int32_t *out_adj, int64_t n_out, const float *dinv,
                                const float *feats, const float *target, const int32_t *active, float *out,
                                float *grad, double *loss, float *params_after, void *stream) {
  g_build_error.clear();
  RWR_TRY(gnn_eval_check(params, nR, S, in_off, in_len, in_adj, n_in, out_off, out_len, out_adj, n_out, dinv, feats,
                         target, active, grad, loss, params_after));
  const int64_t rows = (int64_t)nR * S;
  if (rows > NA_MAX_ROWS || n_in > NA_MAX_EDGES || n_out > NA_MAX_EDGES) {
    g_build_error = "region exceeds the fixed scratch of rwr_gnn_eval_noalloc (" + std::to_string(NA_MAX_ROWS) +
                    " rows, " + std::to_string(NA_MAX_EDGES) + " edges per orientation)";
    return RWR_EINVAL;
  }
  void *base = nullptr;
  RWR_TRY(noalloc_scratch(&base));
  const hipStream_t st = (hipStream_t)stream;
  // the network's buffers, then the region arrays, carved from the scratch
  gnn::Net net;
  size_t used = gnn::net_view(net, S, NA_MAX_ROWS, base, NA_BYTES);
  char *p = static_cast<char *>(base);
  auto take = [&](size_t bytes) -> void * {
    const size_t b = (bytes + 255) / 256 * 256;
    if (used == 0 || used + b > NA_BYTES) {
      used = 0;
      return nullptr;
    }
    void *q = p + used;
    used += b;
    return q;
  };
  int32_t *d_in_off = (int32_t *)take(sizeof(int32_t) * NA_MAX_ROWS);
  int32_t *d_in_len = (int32_t *)take(sizeof(int32_t) * NA_MAX_ROWS);
  int32_t *d_out_off = (int32_t *)take(sizeof(int32_t) * NA_MAX_ROWS);
  int32_t *d_out_len = (int32_t *)take(sizeof(int32_t) * NA_MAX_ROWS);
  int32_t *d_in_items = (int32_t *)take(sizeof(int32_t) * (NA_MAX_ROWS + 1));
  int32_t *d_out_items = (int32_t *)take(sizeof(int32_t) * (NA_MAX_ROWS + 1));
  int32_t *d_in_adj = (int32_t *)take(sizeof(int32_t) * NA_MAX_EDGES);
  int32_t *d_out_adj = (int32_t *)take(sizeof(int32_t) * NA_MAX_EDGES);
  float *d_dinv = (float *)take(sizeof(float) * NA_MAX_ROWS);
  if (used == 0) {
    g_build_error = "scratch layout does not fit";
    return RWR_ENOMEM;
  }
#define NA_TRY(expr)                                                  \
  do {                                                                \
    const hipError_t _e = (expr);                                     \
    if (_e != hipSuccess) {                                           \
      g_build_error = std::string(#expr) + ": " + hipGetErrorString(_e); \
      return RWR_EHIP;                                                \
    }                                                                 \
  } while (0)
  const int64_t P = gnn::LAYOUT.total;
  // parameters; the optimiser starts from zero moments (the scratch keeps
  // the previous call's contents)
  NA_TRY(hipMemcpyAsync(net.theta, params, sizeof(float) * P, hipMemcpyHostToDevice, st));
  launch_zero_bytes(net.m1, sizeof(float) * P, st);
  launch_zero_bytes(net.m2, sizeof(float) * P, st);
  net.step = 0;
  gnn::net_prepare_weights(net, st);
  NA_TRY(hipMemcpyAsync(d_in_off, in_off, sizeof(int32_t) * nR, hipMemcpyHostToDevice, st));
  NA_TRY(hipMemcpyAsync(d_in_len, in_len, sizeof(int32_t) * nR, hipMemcpyHostToDevice, st));
  NA_TRY(hipMemcpyAsync(d_out_off, out_off, sizeof(int32_t) * nR, hipMemcpyHostToDevice, st));
  NA_TRY(hipMemcpyAsync(d_out_len, out_len, sizeof(int32_t) * nR, hipMemcpyHostToDevice, st));
  if (n_in > 0) NA_TRY(hipMemcpyAsync(d_in_adj, in_adj, sizeof(int32_t) * n_in, hipMemcpyHostToDevice, st));
  if (n_out > 0) NA_TRY(hipMemcpyAsync(d_out_adj, out_adj, sizeof(int32_t) * n_out, hipMemcpyHostToDevice, st));
  NA_TRY(hipMemcpyAsync(d_dinv, dinv, sizeof(float) * nR, hipMemcpyHostToDevice, st));
  NA_TRY(hipMemcpyAsync(net.F, feats, sizeof(float) * rows * gnn::FEAT, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_na_items, dim3(1), dim3(NA_SCAN), 0, st, d_in_len, nR, (int32_t)gnn::AGG_CHUNK, d_in_items);
  hipLaunchKernelGGL(k_na_items, dim3(1), dim3(NA_SCAN), 0, st, d_out_len, nR, (int32_t)gnn::AGG_CHUNK, d_out_items);
  int64_t ni = 0, no = 0;
  for (int32_t i = 0; i < nR; ++i) {
    ni += (in_len[i] + gnn::AGG_CHUNK - 1) / gnn::AGG_CHUNK;
    no += (out_len[i] + gnn::AGG_CHUNK - 1) / gnn::AGG_CHUNK;
  }
  gnn::RegionView g{};
  g.in_off = d_in_off;
  g.in_len = d_in_len;
  g.in_adj = d_in_adj;
  g.out_off = d_out_off;
  g.out_len = d_out_len;
  g.out_adj = d_out_adj;
  g.in_items = d_in_items;
  g.out_items = d_out_items;
  g.n_in_items = (int32_t)ni;
  g.n_out_items = (int32_t)no;
  g.loc = nullptr;
  g.nodes = nullptr;
  g.dinv = d_dinv;
  g.nR = nR;
  gnn::net_forward(net, g, rows, st);
  if (target) {
    int32_t act[RWR_MAX_COLS] = {};
    int n_act = 0;
    for (int j = 0; j < S; ++j) n_act += (act[j] = active[j] ? 1 : 0);
    NA_TRY(hipMemcpyAsync(net.t, target, sizeof(float) * rows, hipMemcpyHostToDevice, st));
    NA_TRY(hipMemcpyAsync(net.active, act, sizeof(int32_t) * RWR_MAX_COLS, hipMemcpyHostToDevice, st));
    gnn::net_loss(net, rows, n_act, st);
    gnn::net_backward(net, g, rows, st);
    if (params_after) gnn::net_adamw(net, st);
    // act lives on this stack frame: the copy must finish before return
    NA_TRY(hipStreamSynchronize(st));
  }
  if (out) NA_TRY(hipMemcpyAsync(out, net.o, sizeof(float) * rows, hipMemcpyDeviceToHost, st));
  if (grad) NA_TRY(hipMemcpyAsync(grad, net.grad, sizeof(float) * P, hipMemcpyDeviceToHost, st));
  if (loss) NA_TRY(hipMemcpyAsync(loss, net.loss, sizeof(double), hipMemcpyDeviceToHost, st));
  if (params_after) NA_TRY(hipMemcpyAsync(params_after, net.theta, sizeof(float) * P, hipMemcpyDeviceToHost, st));
  NA_TRY(hipStreamSynchronize(st));
#undef NA_TRY
  return RWR_OK;
}

rwr_status rwr_gnn_eval(const float *params, int32_t nR, int32_t S, const int32_t *in_off, const int32_t *in_len,
                        const int32_t *in_adj, int64_t n_in, const int32_t *out_off, const int32_t *out_len,
                        const int32_t *out_adj, int64_t n_out, const float *dinv, const float *feats,
                        const float *target, const int32_t *active, float *out, float *grad, double *loss,
                        float *params_after) {
  g_build_error.clear();
  RWR_TRY(gnn_eval_check(params, nR, S, in_off, in_len, in_adj, n_in, out_off, out_len, out_adj, n_out, dinv, feats,
                         target, active, grad, loss, params_after));
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    g_build_error = "hipStreamCreate failed";
    return RWR_EHIP;
  }
  const int64_t rows = (int64_t)nR * S;
  gnn::Net net;
  std::vector<void *> tmp;
  rwr_status ret = RWR_OK;
  auto up = [&](const void *h, size_t bytes) -> void * {
    void *d = nullptr;
    if (hipMalloc(&d, std::max<size_t>(bytes, 4)) != hipSuccess) return nullptr;
    tmp.push_back(d);
    if (bytes && hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st) != hipSuccess) return nullptr;
    return d;
  };
  do {
    if (gnn::net_alloc(net, S, rows) != hipSuccess || gnn::net_set_params(net, params, st) != hipSuccess) {
      ret = RWR_ENOMEM;
      break;
    }
    gnn::RegionView g{};
    g.in_off = (const int32_t *)up(in_off, sizeof(int32_t) * nR);
    g.in_len = (const int32_t *)up(in_len, sizeof(int32_t) * nR);
    g.in_adj = (const int32_t *)up(in_adj, sizeof(int32_t) * n_in);
    g.out_off = (const int32_t *)up(out_off, sizeof(int32_t) * nR);
    g.out_len = (const int32_t *)up(out_len, sizeof(int32_t) * nR);
    g.out_adj = (const int32_t *)up(out_adj, sizeof(int32_t) * n_out);
    g.dinv = (const float *)up(dinv, sizeof(float) * nR);
    std::vector<int32_t> ii(nR + 1, 0), oi(nR + 1, 0);
    for (int32_t i = 0; i < nR; ++i) {
      ii[i + 1] = ii[i] + (in_len[i] + gnn::AGG_CHUNK - 1) / gnn::AGG_CHUNK;
      oi[i + 1] = oi[i] + (out_len[i] + gnn::AGG_CHUNK - 1) / gnn::AGG_CHUNK;
    }
    g.in_items = (const int32_t *)up(ii.data(), sizeof(int32_t) * (nR + 1));
    g.out_items = (const int32_t *)up(oi.data(), sizeof(int32_t) * (nR + 1));
    g.n_in_items = ii[nR];
    g.n_out_items = oi[nR];
    g.loc = nullptr;
    g.nodes = nullptr;
    g.nR = nR;
    if (!g.in_off || !g.in_len || !g.in_adj || !g.out_off || !g.out_len || !g.out_adj || !g.dinv || !g.in_items ||
        !g.out_items ||
        hipMemcpyAsync(net.F, feats, sizeof(float) * rows * gnn::FEAT, hipMemcpyHostToDevice, st) != hipSuccess) {
      ret = RWR_ENOMEM;
      break;
    }
    gnn::net_forward(net, g, rows, st);
    if (target) {
      int n_act = 0;
      std::vector<int32_t> act(RWR_MAX_COLS, 0);
      for (int j = 0; j < S; ++j) n_act += (act[j] = active[j] ? 1 : 0);
      if (hipMemcpyAsync(net.t, target, sizeof(float) * rows, hipMemcpyHostToDevice, st) != hipSuccess ||
          hipMemcpyAsync(net.active, act.data(), sizeof(int32_t) * RWR_MAX_COLS, hipMemcpyHostToDevice, st) !=
              hipSuccess) {
        ret = RWR_EHIP;
        break;
      }
      gnn::net_loss(net, rows, n_act, st);
      gnn::net_backward(net, g, rows, st);
      if (params_after) gnn::net_adamw(net, st);
    }
    if (hipStreamSynchronize(st) != hipSuccess) {
      ret = RWR_EHIP;
      break;
    }
    if (out && hipMemcpy(out, net.o, sizeof(float) * rows, hipMemcpyDeviceToHost) != hipSuccess) ret = RWR_EHIP;
    if (grad && hipMemcpy(grad, net.grad, sizeof(float) * gnn::LAYOUT.total, hipMemcpyDeviceToHost) != hipSuccess)
      ret = RWR_EHIP;
    if (loss && hipMemcpy(loss, net.loss, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) ret = RWR_EHIP;
    if (params_after && gnn::net_get_params(net, params_after, st) != hipSuccess) ret = RWR_EHIP;
  } while (false);
  (void)hipStreamSynchronize(st);
  for (void *p : tmp) (void)hipFree(p);
  gnn::net_free(net);
  (void)hipStreamDestroy(st);
  if (ret != RWR_OK && g_build_error.empty()) g_build_error = "device error in rwr_gnn_eval";
  return ret;
}

}  // extern "C"
