// Host launchers of the learned warm start inside an update (k_warm.hip).
//
// Inputs of the network for (region node v, seed column j), in order:
//   0  log(1 + d_in(v)) / 8          1  log(1 + d_out(v)) / 8
//   2  q_offset(v, j) / ||q_j||_1    3  |input 2|
//   4  log(1 + n * r_old(v, j) / sigma_j) / 8 (0 when negative)
//   5..8  hop distance from the offset support: 0, 1, 2, >= 3 (one-hot)
//   9  1 for a dead end              10 1 when v is seed j
//   11 1/d_out(v) (0 for a dead end) 12 1/d_in(v) (0 without in-edges)
//   13 input 3 * input 0             14 input 3 * input 1
//   15 input 2 * input 0
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rwr_common.h"
#include "rwr_kernels.h"

size_t ws_select_temp_bytes(int32_t n);
// out = indices v < n with flags[v] != 0, in increasing order; *count (device) their number
hipError_t ws_select(const int32_t *flags, int32_t n, int32_t *out, int32_t *count, void *temp, size_t temp_bytes,
                     hipStream_t s);
void ws_loc(const int32_t *R, int32_t nR, const DevGraphView &out, int32_t *loc1, float *dinv, hipStream_t s);
size_t ws_scan_temp_bytes(int32_t n);

// Rows of a node list cut into fixed-size edge items (one wavefront each):
// tmp and rit hold max_nodes + 1 ints, irow, icnt and ioff max_items + 1;
// scan_temp covers an exclusive sum of max(max_nodes, max_items) + 1 ints.
#define WS_MAX_HOPS 8
struct WsItems {
  int32_t *tmp, *rit, *irow, *icnt, *ioff;
  int32_t max_items;
  void *scan_temp;
  size_t scan_bytes;
};
// items needed for rows of up to max_nodes nodes in a graph of m stored edges
int64_t ws_max_items(int32_t max_nodes, int64_t m);
// The region on the device: level 0 = the stamped offset support, level h =
// unvisited out-neighbours of level h - 1 (h <= hops), each level in
// increasing node order, a level that would pass max_nodes left out and the
// search stopped there.  R holds the nodes level by level; lv (2 + hops + 1
// ints) receives lv[0] = |R|, lv[1] = 1 once stopped, lv[2 + h] = end of level
// h in R (-1 for levels not taken).  hop1 marks the nodes taken.
hipError_t ws_region(const int32_t *stamp, int32_t st, int32_t n, int32_t hops, int32_t max_nodes,
                     const DevGraphView &out, int32_t *hop1, int32_t *flags, int32_t *wlist, int32_t *kcnt,
                     int32_t *R, int32_t *lv, const WsItems &it, void *sel_temp, size_t sel_bytes, hipStream_t s);
// Local rows of the region (nR = lv[0] nodes, known to the caller) in
// orientation gv: cnt[i] = neighbours of R[i] inside the region, off =
// exclusive prefix (nR + 1 entries, off[nR] = total); then (ws_local_fill,
// with the same items, before they are reused) the rows in local ids.
hipError_t ws_local_rows(const int32_t *R, const int32_t *lv, int32_t nR, const DevGraphView &gv,
                         const int32_t *loc1, const WsItems &it, int32_t *cnt, int32_t *off, hipStream_t s);
void ws_local_fill(const int32_t *R, const int32_t *lv, const DevGraphView &gv, const int32_t *loc1,
                   const WsItems &it, int32_t *adj, hipStream_t s);
// items = exclusive prefix of ceil(cnt[i] / chunk) (nR + 1 entries; tmp is
// scratch of nR + 1 ints)
hipError_t ws_chunk_items(const int32_t *cnt, int32_t nR, int32_t chunk, int32_t *tmp, int32_t *items, void *temp,
                          size_t temp_bytes, hipStream_t s);
void ws_clear(const int32_t *R, int32_t nR, int32_t *hop1, int32_t *loc1, hipStream_t s);
void ws_features(const int32_t *R, int32_t nR, int S, const int32_t *hop1, const DevGraphView &in,
                 const DevGraphView &out, const double *ybuf, const double *r, const Ctl *ctl, const int32_t *seeds,
                 const double *qn, int32_t n_total, float *F, hipStream_t s);
// qn[j] = ||q_j||_1 and qn[S + j] = sum of q_j over the offset support
void ws_qnorm(const int32_t *R, int32_t n0, int S, const double *ybuf, double *part, double *qn, hipStream_t s);
// xhat = ||q|| o, corrected so that the residual has a zero sum, and
// scattered into the dense FP64 vector w (zero outside the region).  part
// holds at least 512 * 4 * S doubles, beta and fa S doubles each (the
// correction's beta and f(|xhat|) per column).
void ws_predict(const int32_t *R, int32_t nR, int S, const DevGraphView &out, const float *o, const double *qn,
                double c1, double *xhat, double *w, double *part, double *beta, double *fa, hipStream_t s);
void ws_unscatter(const int32_t *R, int32_t nR, int S, double *w, hipStream_t s);
// pbuf holds g = (1-c) B~^T xhat - xhat on every node; rho = q + g replaces
// it and its signs go to sg (n * S bytes); sums[j] = ||rho_j||_1, sums[S + j]
// = sum of xhat_j
void ws_rho(int32_t n, int S, const double *ybuf, double *pbuf, const double *w, int8_t *sg, double *part,
            double *sums, hipStream_t s);
// accepted columns: ybuf = rho, r += xhat, sigma += sum xhat, stamps; pbuf
// (rho) cleared
void ws_apply(int32_t n, int S, uint64_t accept, double *ybuf, double *pbuf, double *r, const double *w,
              int32_t *stamp, Ctl *ctl, const double *xsum, hipStream_t s);
// Work items over the region's out-rows (GRAD_CHUNK = 1024 edges each):
// items is scratch of nR + 1 ints, item_off[i] = first item of row i (nR + 1
// entries, item_off[nR] = their number), item_row the row of each item.
hipError_t ws_out_items(const int32_t *R, int32_t nR, const DevGraphView &out, int32_t *items, int32_t *item_off,
                        int32_t *item_row, void *temp, size_t temp_bytes, hipStream_t s);
// The residual from the region alone (for regions whose out-rows are a small
// part of the graph): rho = q - xhat' + (1-c) B~^T xhat' on the region and its
// out-neighbours (marked in hop1 until ws_unmark_boundary), by a push of the
// rows of xhat (region-row order) into pbuf (FP64, zero at rest and left
// zero at rest).  Outputs as ws_rho (rho in pbuf and its signs in sg only on
// those nodes).
void ws_rho_push(const int32_t *R, int32_t nR, int S, const DevGraphView &out, const int32_t *item_off,
                 const int32_t *item_row, const double *xhat, double c1, double *pbuf, int32_t *hop1, int32_t n,
                 const double *ybuf, const double *w, int8_t *sg, double *part, double *sums, hipStream_t s);
// ws_apply for the residual of ws_rho_push (only the marked nodes; pbuf back
// to zero there)
void ws_apply_sparse(int32_t n, int S, uint64_t accept, const int32_t *hop1, double *ybuf, double *pbuf, double *r,
                     const double *w, int32_t *stamp, Ctl *ctl, const double *xsum, hipStream_t s);
void ws_unmark_boundary(int32_t n, int32_t *hop1, hipStream_t s);
// dL/do of the residual loss through the mass correction (see
// k_ws_grad_fixed / k_ws_grad_corr) into dout (rows nR * S); gpart holds one
// double per (gradient item, column): at least (nR + edges of the region's
// out-rows / 1024 + 1) * S; item_off and item_row from ws_out_items;
// kpart WS_KPART_BLOCKS * S doubles, corr S doubles.  Fixed-order sums only.
#define WS_KPART_BLOCKS 1024
hipError_t ws_resid_grad(const int32_t *R, int32_t nR, int S, const DevGraphView &out, double c1, const double *rho,
                         const int8_t *sg, double *gpart, int32_t *items, int32_t *item_off, int32_t *item_row,
                         void *temp,
                         size_t temp_bytes, const int32_t *active, double q_active, const float *o, const double *qn,
                         const double *beta, const double *fa, double *kpart, double *corr, float *dout,
                         hipStream_t s);
