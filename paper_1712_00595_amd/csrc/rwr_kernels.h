// Launch interface of the HIP kernels (host side).  Each launcher enqueues
// on the given stream and returns immediately.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "rwr_common.h"

#define SMALL_SORT_MAX 4096

// one orientation of the slack adjacency structure
struct DevGraphView {
  int32_t *off;
  int32_t *len;
  int32_t *cap;
  int32_t *adj;
  uint8_t *heavy;
};

// heavy-row schedule of the dense pull: rows whose in-degree exceeds the
// light limit are split into chunks, each handled by a whole workgroup; the
// chunk sums are combined by a follow-up kernel
struct HeavyView {
  const int32_t *item_row;   // work item -> heavy row index h
  const int32_t *item_chunk; // work item -> chunk number within the row
  const int32_t *rows;       // h -> node id
  const int32_t *nchunks;    // h -> chunks planned for the row
  const int32_t *first;      // h -> first work item of the row
  double *part;              // item*S + j -> chunk sum
  int32_t n_items;
  int32_t n_rows;
  int32_t chunk;
};

// everything an iteration slot needs
struct SlotArgs {
  DevGraphView out;  // rows of A~ (push, out-degrees)
  DevGraphView in;   // columns of A~ (pull)
  HeavyView heavy;
  double *r;
  double *ybuf;
  double *gbuf;
  double *xres;  // r / d_out per node and column (residual sweep gathers)
  void *x[2];
  int32_t *stamp;    // node touched in the current slot (slot stamp)
  int32_t *fstamp;   // node in the frontier of x^(i) (stamp of slot i)
  int32_t *hfront;   // frontier nodes routed to the chunked push
  int32_t *hbase;    // first chunk number of each of them
  const int32_t *seeds;
  Ctl *ctl;
  double *hist;
  double *part;      // per-workgroup partials, then per-group partials
  int64_t *part_i;
  int32_t n;
  int32_t n_seeds;
  double c;
  int32_t grid_sparse;
  int32_t grid_light;
  int32_t grid_pull;  // workgroups of a dense sweep (each loops over items)
  int32_t light_lanes;  // lanes per row of the light push
  int32_t pull_lanes;   // lanes per in-row of the dense sweep for S >= 4 (16, 32 or 64)
  int32_t fold_max;     // heavy row-columns at most that the decision kernel finishes itself
  int32_t zero_seed_rows;   // residual sweep: 1 zeroes the seed row of each column (the restart term)
  const double *qvec;       // seed vectors (node-major, S per node) or null; when set, the residual
                            // check adds their restart term c q after the sweep
  const int32_t *row_order;  // order of the in-rows in that sweep (a permutation of 0 .. n_cap-1)
  int32_t n_order;           // its length (n_cap)
  const int32_t *mp_rows;  // row partition of the single-column dense sweep (wavefront items)
  int32_t n_mp;            // items of that partition
};

// The host fills these structures and the kernels read them as by-value
// arguments: their layout is pinned here, so that the host and the device
// compilation of every source agree on it (plain pointers and 32/64-bit
// scalars only).
static_assert(sizeof(DevGraphView) == 40 && sizeof(HeavyView) == 64, "view layout");
static_assert(sizeof(SlotArgs) == 352 && offsetof(SlotArgs, r) == 144 && offsetof(SlotArgs, x) == 176 &&
                  offsetof(SlotArgs, ctl) == 232 && offsetof(SlotArgs, n) == 264 && offsetof(SlotArgs, c) == 272 &&
                  offsetof(SlotArgs, zero_seed_rows) == 304 && offsetof(SlotArgs, qvec) == 312 &&
                  offsetof(SlotArgs, n_mp) == 344,
              "slot argument layout");

#define WV_ROWS 64      // rows per wave item of the wave-granular single-column sweep
#define WV_EDGES 512    // light in-edges per wave item (one round of the wavefront)

// ---- delta (k_delta.hip)
void launch_make_keys(const int32_t *ins_s, const int32_t *ins_d, int64_t n_ins, const int32_t *del_s,
                      const int32_t *del_d, int64_t n_del, int32_t n_nodes, int b1, int undirected,
                      const int32_t *perm, const int32_t *mark, uint64_t *k_out, uint64_t *k_in, Ctl *ctl,
                      hipStream_t st);
// node deletions: mark the nodes and count their adjacency entries; write
// their incident edges (rows_only: their out-edges only) as deletion keys
// from entry `first` on; clear marks
void launch_node_mark(const int32_t *del_nodes, int32_t n_del, const int32_t *perm, const DevGraphView &out,
                      const DevGraphView &in, int undirected, int rows_only, int32_t *mark, int64_t *cnt,
                      hipStream_t st);
void launch_node_keys(const int32_t *del_nodes, int32_t n_del, const int64_t *off, int64_t first,
                      const int32_t *perm, const DevGraphView &out, const DevGraphView &in, int undirected,
                      int rows_only, const int32_t *mark, int b1, uint64_t *k_out, uint64_t *k_in, Ctl *ctl,
                      hipStream_t st);
// scores of column j from caller values (caller ids): r[perm[v]*S + j] = in[v]
void launch_set_scores(const double *in, const int32_t *perm, int S, int j, int32_t n, double *r, hipStream_t st);
void launch_node_unmark(const int32_t *del_nodes, int32_t n_del, const int32_t *perm, int32_t *mark,
                        hipStream_t st);
void launch_sort_segment_small(uint64_t *k0, uint64_t *k1, int32_t n_keys, int b1, int32_t *seg0, int32_t *row0,
                               int32_t *seg1, int32_t *row1, int orientations, Ctl *ctl, hipStream_t st);
hipError_t sort_segment_large(uint64_t *keys, uint64_t *keys_alt, int32_t n_keys, int b1, int32_t *flags,
                              int32_t *pos, int32_t *seg, int32_t *row, void *temp, size_t temp_bytes, Ctl *ctl,
                              int orient, hipStream_t st);
size_t sort_temp_bytes(int32_t n_keys);
// per-orientation arguments of the batch check and the structural apply;
// one launch serves both orientations (o[0..norient-1])
struct OrientArgs {
  const uint64_t *keys;
  const int32_t *seg;
  const int32_t *row;
  DevGraphView g;
  int32_t *t_dold;
  int32_t *t_dnew;
  int32_t orient;
  int32_t check;        // test inserted/deleted entries against the graph
  int32_t heavy_limit;  // count rows that become heavy (pull orientation)
  int64_t e_cap;        // arena capacity
};
// Rows above BIG_ROW entries are checked and rewritten by a whole workgroup
// when `big` is set (lists bigv: checked rows of the out orientation, biga:
// orient << 31 | t of rows to compact or move; 2 (max_rows + 1) ints each);
// otherwise every row takes one wavefront.
constexpr int32_t BIG_ROW = 4096;
struct OrientPair {
  OrientArgs o[2];
  int32_t *bigv;
  int32_t *biga;
  int32_t big;
  int32_t recs;  // sum the touched rows' old degrees (Ctl::seed_recs) for the sorted offset seed
};
static_assert(sizeof(OrientArgs) == 104 && sizeof(OrientPair) == 232 && offsetof(OrientPair, recs) == 228,
              "batch argument layout");
void launch_validate_plan(const OrientPair &P, int norient, int b1, Ctl *ctl, int32_t max_rows, hipStream_t st);
// q_offset of r - rsub (rsub may be null; subtracted in the columns of
// rmask only) into ybuf (atomically; ybuf null:
// the support stamps and cost-model sums only); touched rows cut into chunks
// (items, item_off: max_rows + 1 ints, temp: seed_scan_temp_bytes(max_rows)).
// rec (optional): the seed's records for launch_seed_sort_reduce, one slot per
// old neighbour and batch key of each touched row (ctl->seed_recs + the number
// of keys, read back after validation), with dcnt, rec_off: max_rows + 1 ints
hipError_t launch_offset_seed(int S, const uint64_t *keys, const int32_t *seg, const int32_t *row,
                              const int32_t *t_dold, const int32_t *t_dnew, const DevGraphView &g, const double *r,
                              const double *rsub, uint64_t rmask, double *ybuf, int32_t *stamp, Ctl *ctl, int b1,
                              double c1, int32_t max_rows, int32_t *items, int32_t *item_off, uint64_t *rec,
                              int32_t *dcnt, int32_t *rec_off, void *temp, size_t temp_bytes, int grid,
                              hipStream_t st);
size_t seed_scan_temp_bytes(int32_t max_rows);
// workgroups of the heavy-row epilogue (one (row, column) pair per thread);
// its partials follow the sweep's, so partial buffers hold this many more
constexpr int HEAVY_EPI_MAX_GRID = 2048;
// big_rows: the count of biga read back after validation (0: no launch)
void launch_apply(const OrientPair &P, int norient, int b1, Ctl *ctl, int32_t max_rows, int32_t big_rows,
                  hipStream_t st);
// the offset seed summed in a fixed order (no atomics) from the records that
// launch_offset_seed wrote into rec (n_rec slots; those past the last touched
// row's, located by rec_off and seg, become pads): sorted into
// rec_alt, each node's terms added in sorted order and stored into ybuf
// (plain stores; zero elsewhere).  hpart, tpart: seed_part_len(n_rec, S)
// doubles each; temp: seed_sort_temp_bytes(n_rec)
hipError_t launch_seed_sort_reduce(int S, uint64_t *rec, uint64_t *rec_alt, int32_t n_rec, int32_t max_rows,
                                   int32_t n_nodes, const int32_t *rec_off, const int32_t *seg,
                                   const int32_t *row, const int32_t *t_dold, const int32_t *t_dnew,
                                   const double *r, const double *rsub, uint64_t rmask, double c1, double *ybuf,
                                   double *hpart, double *tpart, void *temp, size_t temp_bytes, const Ctl *ctl,
                                   int grid, hipStream_t st);
int64_t seed_part_len(int64_t n_rec, int S);
size_t seed_sort_temp_bytes(int64_t n_rec);

// ---- propagation (k_prop.hip); fp64 selects the propagation type
// hist_base: first row of the norm history this run writes (0 for update
// runs; refinements write after them, so the update's norms stay readable).
// lockstep: a column that passes the stop test keeps propagating until every
// column of the run has passed it, and then all retire at once (their last
// iterates then sit in the same x buffer, so a run's tail can be carried for
// every column; the extra iterations only shrink the converged columns'
// truncation, and the dense sweep reads every column of a gathered row
// anyway).  0: each column retires at its own stop test (Algorithm 1 per
// seed).
void launch_reset_run(Ctl *ctl, int32_t S, uint64_t active_mask, double eps, int32_t max_iters, int64_t dense_thresh,
                      int64_t dense_nodes, hipStream_t st, int32_t hist_base = 0, int32_t lockstep = 0);
void launch_seed_init(const SlotArgs &a, int S, hipStream_t st);
void launch_seed_init_q(const SlotArgs &a, int S, hipStream_t st);
// carried vectors in gbuf before an update: d_out * x[last] for tail_mask
// columns (last = -1: none), the pending vector for keep_mask columns, 0
// elsewhere; clears both x buffers
void launch_carry_prepare(const SlotArgs &a, int S, bool fp64, int last, uint64_t tail_mask, uint64_t keep_mask,
                          hipStream_t st);
// before the first dense slot k of a run: x^(k-1) += gbuf / d_out for the
// active columns in mask (ctl->inj records them)
void launch_inject(const SlotArgs &a, int S, bool fp64, int k, uint64_t mask, hipStream_t st);
// r += gbuf over the seed columns
void launch_add_resid(const SlotArgs &a, int S, hipStream_t st);
void launch_slot0_epilogue(const SlotArgs &a, int S, bool fp64, hipStream_t st);
// iteration slot k (computes x^(k)): sparse = push + epilogue, dense = pull
void launch_sparse_slot(const SlotArgs &a, int S, bool fp64, int k, hipStream_t st);
// ev0/ev1 (optional) are recorded on st right before and after the sweep
// kernel itself, not around the epilogue and decision kernels.
void launch_dense_slot(const SlotArgs &a, int S, bool fp64, int k, hipStream_t st, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr);
void launch_finish(const SlotArgs &a, int S, bool fp64, hipStream_t st);
void launch_residual(const SlotArgs &a, int S, hipStream_t st);
// g = (1-c) B~^T (r / d_out) - r over every node (the residual sweep on the
// vector in a.r, written to a.gbuf), without the decision kernel
void launch_apply_p(const SlotArgs &a, int S, hipStream_t st);
void launch_refine_init(const SlotArgs &a, int S, bool fp64, hipStream_t st);
void launch_scores(const double *r, const Ctl *ctl, const int32_t *perm, int S, int j, int32_t n, double *out,
                   hipStream_t st);
void launch_sigma_exact(const SlotArgs &a, int S, hipStream_t st);

// ---- graph (k_graph.hip)
void launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t st);
void launch_zero_bytes(void *p, size_t bytes, hipStream_t st);
size_t build_temp_bytes(int64_t m, int32_t n);
hipError_t build_phase1(const int32_t *rows, const int32_t *cols, int64_t m, int32_t n, DevGraphView g, void *temp,
                        size_t temp_bytes, uint64_t *keys, uint64_t *keys_alt, int32_t *sstart, Ctl *ctl,
                        int64_t *used, hipStream_t st);
void build_phase2(const uint64_t *keys, int64_t m, DevGraphView g, const int32_t *sstart, hipStream_t st);
hipError_t relayout_offsets(const int32_t *len, int32_t n, int32_t *new_cap, int32_t *new_off, void *temp,
                            size_t temp_bytes, int64_t *used, hipStream_t st);
void launch_copy_rows(const DevGraphView &g, const int32_t *new_off, int32_t *new_adj, int32_t n, hipStream_t st);
hipError_t export_rows(const DevGraphView &g, int32_t n, const int32_t *inv, int32_t *out_src, int32_t *out_dst,
                       int32_t *pos, void *temp, size_t temp_bytes, hipStream_t st);
hipError_t build_relabel(const int32_t *src, int64_t m, int32_t n, int32_t n_cap, int32_t *perm, int32_t *inv,
                         int32_t *deg_tmp, uint64_t *keys, uint64_t *keys_alt, void *temp, size_t temp_bytes,
                         hipStream_t st);
void launch_identity(int32_t *perm, int32_t *inv, int32_t from, int32_t to, hipStream_t st);
void launch_map_ids(const int32_t *in, int64_t m, int32_t n, const int32_t *perm, int32_t *out, hipStream_t st);
void launch_mark_heavy(const int32_t *len, int32_t n, int32_t limit, uint8_t *flags, int32_t *sel,
                       int32_t *sel_count, hipStream_t st);
void launch_gather_i32(const int32_t *src, const int32_t *idx, int32_t count, int32_t *out, hipStream_t st);
void launch_reset_batch(Ctl *ctl, int demand_only, hipStream_t st);
