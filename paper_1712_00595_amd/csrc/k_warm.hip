// Learned warm start inside an update: the region around the offset seed,
// the network's input features, the prediction xhat, the exact residual
//   rho = q_offset - (I - (1-c) B~^T) xhat
// that replaces the offset seed, and the training target r_offset / ||q||.
//
// Node marks kept between updates (all zero when no update runs):
//   hop1[v] = hop distance + 1 of a region node (0 outside the region),
//   loc1[v] = local index + 1 of a region node.
// The dense FP64 vector w holds the prediction on the region rows during an
// update and is zero otherwise.
#include <hipcub/hipcub.hpp>

#include "gnn.h"
#include "rwr_common.h"
#include "rwr_kernels.h"
#include "warm.h"

#define WB 256
// edges per work item over the region's out-rows (push and gradient)
#define GRAD_CHUNK 1024

__device__ __forceinline__ uint64_t lanemask_below(int lane) { return lane == 0 ? 0ull : (~0ull >> (64 - lane)); }

// ------------------------------------------------------------ region
// flags[v] = 1 when v belongs to level h: the stamped offset support for
// h = 0 (marked hop 1), else the nodes marked h + 1 by the expansion
__global__ void k_ws_level_flags(const int32_t *__restrict__ stamp, int32_t st, int32_t n, int32_t h,
                                 int32_t *__restrict__ hop1, int32_t *__restrict__ flags) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    int f = 0;
    if (h == 0) {
      if (stamp[v] == st) {
        hop1[v] = 1;
        f = 1;
      }
    } else {
      f = hop1[v] == h + 1;
    }
    flags[v] = f;
  }
}

// Region levels on the device.  lv[0] = region nodes so far (nR), lv[1] = 1
// once the search has stopped (a level came out empty or would pass the
// capacity), lv[2 + h] = end of level h in R (-1 while not accepted).  The
// rows of a list (a level, or the whole region) are cut into WS_ROW_CHUNK-edge
// items, one wavefront each, so that rows of hubs spread over the chip.
#define WS_ROW_CHUNK 1024

struct ListRef {
  const int32_t *R;
  const int32_t *lv;
  int level;  // level of R to take; -1: the whole region
  __device__ __forceinline__ int32_t start() const { return level <= 0 ? 0 : lv[2 + level - 1]; }
  __device__ __forceinline__ int32_t end() const {
    if (level < 0) return lv[0];
    const int32_t e = lv[2 + level];
    return e < 0 ? start() : e;
  }
};

// tmp[i] = items of row i of the list (0 past its end), i <= cap
__global__ void k_ws_row_chunks(ListRef L, int32_t cap, DevGraphView gv, int32_t *__restrict__ tmp) {
  const int32_t b = L.start(), k = L.end() - b;
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= cap; i += gridDim.x * blockDim.x)
    tmp[i] = i < k ? (gv.len[L.R[b + i]] + WS_ROW_CHUNK - 1) / WS_ROW_CHUNK : 0;
}

__global__ void k_ws_item_rows(ListRef L, const int32_t *__restrict__ rit, int32_t *__restrict__ irow) {
  const int32_t k = L.end() - L.start();
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x)
    for (int32_t it = rit[i]; it < rit[i + 1]; ++it) irow[it] = i;
}

// mark the unvisited out-neighbours of level h - 1 with h + 1
__global__ void k_ws_expand(ListRef L, const int32_t *__restrict__ rit, const int32_t *__restrict__ irow,
                            DevGraphView out, int32_t h, int32_t *__restrict__ hop1) {
  if (L.lv[1]) return;
  const int32_t b = L.start(), k = L.end() - b;
  const int32_t total = rit[k];
  const int lane = threadIdx.x % RWR_WAVE;
  for (int32_t it = (blockIdx.x * blockDim.x + threadIdx.x) / RWR_WAVE; it < total;
       it += gridDim.x * blockDim.x / RWR_WAVE) {
    const int32_t i = irow[it];
    const int u = L.R[b + i];
    const int o = out.off[u], d = out.len[u];
    const int e1 = min(d, (it - rit[i] + 1) * WS_ROW_CHUNK);
    for (int e = (it - rit[i]) * WS_ROW_CHUNK + lane; e < e1; e += RWR_WAVE) {
      const int v = out.adj[o + e];
      if (hop1[v] == 0) hop1[v] = h + 1;  // every writer stores the same value
    }
  }
}

// level h (k = *kcnt nodes in wlist) joins the region unless the search has
// stopped or it would pass the capacity (then its marks are removed)
__global__ void k_ws_append(const int32_t *__restrict__ wlist, const int32_t *__restrict__ kcnt,
                            int32_t *__restrict__ R, const int32_t *__restrict__ lv, int32_t max_nodes,
                            int32_t *__restrict__ hop1) {
  if (lv[1]) return;
  const int32_t k = *kcnt, nR = lv[0];
  const bool fits = (int64_t)nR + k <= max_nodes;
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    if (fits)
      R[nR + i] = wlist[i];
    else
      hop1[wlist[i]] = 0;
  }
}

__global__ void k_ws_append_fin(const int32_t *__restrict__ kcnt, int32_t *__restrict__ lv, int32_t h,
                                int32_t max_nodes) {
  if (lv[1]) return;
  const int32_t k = *kcnt, nR = lv[0];
  if (k == 0 || (int64_t)nR + k > max_nodes) {
    lv[1] = 1;
    return;
  }
  lv[0] = nR + k;
  lv[2 + h] = nR + k;
}

__global__ void k_ws_lv_init(int32_t *__restrict__ lv, int32_t n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) lv[i] = i < 2 ? 0 : -1;
}

__global__ void k_ws_loc(const int32_t *__restrict__ R, int32_t nR, const DevGraphView out,
                         int32_t *__restrict__ loc1, float *__restrict__ dinv) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nR; i += gridDim.x * blockDim.x) {
    const int v = R[i];
    loc1[v] = i + 1;
    const int d = out.len[v];
    dinv[i] = d ? 1.0f / (float)d : 0.0f;
  }
}

__global__ void k_ws_clear(const int32_t *__restrict__ R, int32_t nR, int32_t *__restrict__ hop1,
                           int32_t *__restrict__ loc1) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nR; i += gridDim.x * blockDim.x) {
    hop1[R[i]] = 0;
    loc1[R[i]] = 0;
  }
}

// ------------------------------------------------------------ local region graph
// The region's own edges in local ids, so that the network's aggregations
// touch only them: rows of the region nodes in one orientation of the device
// graph, filtered to neighbours inside the region, in row order.  Row items
// (see ListRef) count their neighbours inside the region; the exclusive sum
// of the item counts places each item's entries, so a row's entries follow
// its edge order.
__global__ void k_ws_count_items(ListRef L, const int32_t *__restrict__ rit, const int32_t *__restrict__ irow,
                                 int32_t max_items, DevGraphView gv, const int32_t *__restrict__ loc1,
                                 int32_t *__restrict__ icnt) {
  const int32_t b = L.start(), k = L.end() - b;
  const int32_t total = rit[k];
  const int lane = threadIdx.x % RWR_WAVE;
  for (int32_t it = (blockIdx.x * blockDim.x + threadIdx.x) / RWR_WAVE; it <= max_items;
       it += gridDim.x * blockDim.x / RWR_WAVE) {
    int c = 0;
    if (it < total) {
      const int32_t i = irow[it];
      const int v = L.R[b + i];
      const int o = gv.off[v], d = gv.len[v];
      const int e1 = min(d, (it - rit[i] + 1) * WS_ROW_CHUNK);
      for (int e = (it - rit[i]) * WS_ROW_CHUNK + lane; e < e1; e += RWR_WAVE) c += loc1[gv.adj[o + e]] > 0;
      for (int off = 1; off < RWR_WAVE; off <<= 1) c += __shfl_xor(c, off, RWR_WAVE);
    }
    if (lane == 0) icnt[it] = c;
  }
}

// off[i] (nR + 1 entries) and cnt[i] of each row from the item offsets
__global__ void k_ws_row_off(const int32_t *__restrict__ rit, const int32_t *__restrict__ ioff, int32_t nR,
                             int32_t *__restrict__ off, int32_t *__restrict__ cnt) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= nR; i += gridDim.x * blockDim.x) {
    off[i] = ioff[rit[i]];
    if (i < nR) cnt[i] = ioff[rit[i + 1]] - ioff[rit[i]];
  }
}

__global__ void k_ws_fill_items(ListRef L, const int32_t *__restrict__ rit, const int32_t *__restrict__ irow,
                                DevGraphView gv, const int32_t *__restrict__ loc1, const int32_t *__restrict__ ioff,
                                int32_t *__restrict__ adj) {
  const int32_t b = L.start(), k = L.end() - b;
  const int32_t total = rit[k];
  const int lane = threadIdx.x % RWR_WAVE;
  for (int32_t it = (blockIdx.x * blockDim.x + threadIdx.x) / RWR_WAVE; it < total;
       it += gridDim.x * blockDim.x / RWR_WAVE) {
    const int32_t i = irow[it];
    const int v = L.R[b + i];
    const int o = gv.off[v], d = gv.len[v];
    const int e0 = (it - rit[i]) * WS_ROW_CHUNK, e1 = min(d, e0 + WS_ROW_CHUNK);
    int base = ioff[it];
    for (int eb = e0; eb < e1; eb += RWR_WAVE) {
      const int e = eb + lane;
      const int l = e < e1 ? loc1[gv.adj[o + e]] : 0;
      const uint64_t m = __ballot(l > 0);
      if (l > 0) adj[base + __popcll(m & lanemask_below(lane))] = l - 1;
      base += __popcll(m);
    }
  }
}

// ------------------------------------------------------------ features
// per-workgroup partials over the level-0 nodes (q sits in ybuf) of
// ||q_j||_1 (entries j) and of the signed sum of q_j (entries S + j)
__global__ __launch_bounds__(WB) void k_ws_qnorm(const int32_t *__restrict__ R, int32_t n0, int S,
                                                 const double *__restrict__ ybuf, double *__restrict__ part) {
  __shared__ double red[WB], sgn[WB];
  const int j = threadIdx.x % S, rl = threadIdx.x / S, RPB = WB / S;
  double s = 0.0, t = 0.0;
  for (int i = blockIdx.x * RPB + rl; i < n0; i += gridDim.x * RPB) {
    const double q = ybuf[col_index(R[i], S, j)];
    s += fabs(q);
    t += q;
  }
  red[threadIdx.x] = s;
  sgn[threadIdx.x] = t;
  __syncthreads();
  if (threadIdx.x < S) {
    double a = 0.0, b = 0.0;
    for (int q = 0; q < RPB; ++q) a += red[q * S + threadIdx.x], b += sgn[q * S + threadIdx.x];
    part[(int64_t)blockIdx.x * 2 * S + threadIdx.x] = a;
    part[(int64_t)blockIdx.x * 2 * S + S + threadIdx.x] = b;
  }
}

// out[j] = sum over b of part[b * S + j] (S entries per partial), one
// workgroup per entry: thread t sums partials t, t + WB, ..., then the thread
// sums are added in thread order
__global__ __launch_bounds__(WB) void k_ws_sum_parts(const double *__restrict__ part, int nb, int S,
                                                     double *__restrict__ out) {
  __shared__ double red[WB];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += WB) s += part[(int64_t)b * S + j];
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < WB; ++q) t += red[q];
    out[j] = t;
  }
}

// The sixteen inputs of a (node, column) row; see warm.h for the list.
__global__ void k_ws_features(const int32_t *__restrict__ R, int32_t nR, int S, const int32_t *__restrict__ hop1,
                              DevGraphView in, DevGraphView out, const double *__restrict__ ybuf,
                              const double *__restrict__ r, const Ctl *__restrict__ ctl,
                              const int32_t *__restrict__ seeds, const double *__restrict__ qn, int32_t n_total,
                              float *__restrict__ F) {
  const int64_t rows = (int64_t)nR * S;
  for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < rows;
       row += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(row / S), j = (int)(row % S);
    const int v = R[i];
    const int64_t kk = col_index(v, S, j);
    const double q = qn[j] > 0.0 ? ybuf[kk] / qn[j] : 0.0;
    const double sig = ctl->sigma[j];
    const double rn = sig != 0.0 ? r[kk] / sig : 0.0;
    const int din = in.len[v], dout = out.len[v];
    const int hp = hop1[v] - 1;
    float f[16];
    f[0] = log1pf((float)din) * 0.125f;
    f[1] = log1pf((float)dout) * 0.125f;
    f[2] = (float)q;
    f[3] = fabsf((float)q);
    f[4] = log1pf(fmaxf(0.0f, (float)(rn * (double)n_total))) * 0.125f;
    f[5] = hp == 0 ? 1.0f : 0.0f;
    f[6] = hp == 1 ? 1.0f : 0.0f;
    f[7] = hp == 2 ? 1.0f : 0.0f;
    f[8] = hp >= 3 ? 1.0f : 0.0f;
    f[9] = dout == 0 ? 1.0f : 0.0f;
    f[10] = (j < RWR_MAX_COLS && seeds[j] == v) ? 1.0f : 0.0f;
    f[11] = dout ? 1.0f / (float)dout : 0.0f;
    f[12] = din ? 1.0f / (float)din : 0.0f;
    // the degree inputs scaled by the offset seed (they grow with it, as
    // the prediction must)
    f[13] = f[3] * f[0];
    f[14] = f[3] * f[1];
    f[15] = f[2] * f[0];
    float4 *dst = reinterpret_cast<float4 *>(F + row * 16);
    dst[0] = float4{f[0], f[1], f[2], f[3]};
    dst[1] = float4{f[4], f[5], f[6], f[7]};
    dst[2] = float4{f[8], f[9], f[10], f[11]};
    dst[3] = float4{f[12], f[13], f[14], f[15]};
  }
}

// ------------------------------------------------------------ prediction and residual
// xhat = ||q_j|| o (FP64)
__global__ void k_ws_predict(int32_t nR, int S, const float *__restrict__ o, const double *__restrict__ qn,
                             double *__restrict__ xhat) {
  const int64_t rows = (int64_t)nR * S;
  for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < rows;
       row += (int64_t)gridDim.x * blockDim.x)
    xhat[row] = qn[row % S] * (double)o[row];
}

// Mass of the prediction.  For any xhat, sum(rho) = sum(q) - f(xhat) with
// f(x) = sum(x) - (1-c) sum over non-dead-end nodes of x (the column sums of
// I - (1-c) B~^T), and f(r_offset) = sum(q) exactly.  A residual with a
// non-zero sum decays no faster than (1-c) per iteration (the all-ones
// vector is a left eigenvector of (1-c) B~^T without dead ends), so the
// prediction is corrected to f(xhat') = sum(q):
//   xhat' = xhat - beta |xhat|,  beta = (f(xhat) - sum(q)) / f(|xhat|).
// Partials per column: [xhat, xhat on non-dead ends, |xhat|, |xhat| on
// non-dead ends] at entries [0, S, 2S, 3S) + j.
__global__ __launch_bounds__(WB) void k_ws_mass(const int32_t *__restrict__ R, int32_t nR, int S,
                                                const DevGraphView out, const double *__restrict__ xhat,
                                                double *__restrict__ part) {
  __shared__ double red[4][WB];
  const int j = threadIdx.x % S, rl = threadIdx.x / S, RPB = WB / S;
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
  for (int i = blockIdx.x * RPB + rl; i < nR; i += gridDim.x * RPB) {
    const double x = xhat[(int64_t)i * S + j];
    const bool live = out.len[R[i]] > 0;
    a += x;
    c += fabs(x);
    if (live) {
      b += x;
      d += fabs(x);
    }
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  red[3][threadIdx.x] = d;
  __syncthreads();
  if (threadIdx.x < S) {
    for (int k = 0; k < 4; ++k) {
      double t = 0.0;
      for (int q = 0; q < RPB; ++q) t += red[k][q * S + threadIdx.x];
      part[(int64_t)blockIdx.x * 4 * S + k * S + threadIdx.x] = t;
    }
  }
}

// beta[j] from the partials and sum(q) = qn[S + j]; fa[j] = f(|xhat_j|),
// which the gradient through the correction needs.  One workgroup per
// column; fixed order (thread t takes partials t, t + WB, ..., then the
// thread sums in thread order).
__global__ __launch_bounds__(WB) void k_ws_beta(const double *__restrict__ part, int nb, int S, double c1,
                                                const double *__restrict__ qn, double *__restrict__ beta,
                                                double *__restrict__ fabs_out) {
  __shared__ double red[4][WB];
  const int j = blockIdx.x;
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
  for (int k = threadIdx.x; k < nb; k += WB) {
    const double *p = part + (int64_t)k * 4 * S;
    a += p[j];
    b += p[S + j];
    c += p[2 * S + j];
    d += p[3 * S + j];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  red[3][threadIdx.x] = d;
  __syncthreads();
  if (threadIdx.x == 0) {
    a = b = c = d = 0.0;
    for (int q = 0; q < WB; ++q) {
      a += red[0][q];
      b += red[1][q];
      c += red[2][q];
      d += red[3][q];
    }
    const double fx = a - c1 * b, fa = c - c1 * d;
    beta[j] = fa > 0.0 ? (fx - qn[S + j]) / fa : 0.0;
    fabs_out[j] = fa;
  }
}

// xhat' = xhat - beta |xhat|, scattered into the dense vector w (rows R)
__global__ void k_ws_adjust_scatter(const int32_t *__restrict__ R, int32_t nR, int S, const double *__restrict__ beta,
                                    double *__restrict__ xhat, double *__restrict__ w) {
  const int64_t rows = (int64_t)nR * S;
  for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < rows;
       row += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(row % S);
    const double x = xhat[row];
    const double y = x - beta[j] * fabs(x);
    xhat[row] = y;
    w[col_index(R[row / S], S, j)] = y;
  }
}

__global__ void k_ws_unscatter(const int32_t *__restrict__ R, int32_t nR, int S, double *__restrict__ w) {
  const int64_t rows = (int64_t)nR * S;
  for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < rows;
       row += (int64_t)gridDim.x * blockDim.x)
    w[col_index(R[row / S], S, (int)(row % S))] = 0.0;
}

// rho = q + g over every node, where g = (1-c) B~^T xhat - xhat (in pbuf):
// rho replaces g in pbuf and its sign goes to sg (one byte per entry, what
// the gradient gathers); partials of ||rho_j||_1 (entries j) and of the sum
// of xhat_j (entries S + j)
__global__ __launch_bounds__(WB) void k_ws_rho(int32_t n, int S, const double *__restrict__ ybuf,
                                               double *__restrict__ pbuf, const double *__restrict__ w,
                                               int8_t *__restrict__ sg, double *__restrict__ part) {
  __shared__ double rn[WB], xs[WB];
  const int j = threadIdx.x % S, rl = threadIdx.x / S, RPB = WB / S;
  double a = 0.0, b = 0.0;
  for (int v = blockIdx.x * RPB + rl; v < n; v += gridDim.x * RPB) {
    const int64_t kk = col_index(v, S, j);
    const double rho = ybuf[kk] + pbuf[kk];
    pbuf[kk] = rho;
    sg[kk] = (int8_t)(rho > 0.0 ? 1 : (rho < 0.0 ? -1 : 0));
    a += fabs(rho);
    b += w[kk];
  }
  rn[threadIdx.x] = a;
  xs[threadIdx.x] = b;
  __syncthreads();
  if (threadIdx.x < S) {
    double t = 0.0, u = 0.0;
    for (int q = 0; q < RPB; ++q) t += rn[q * S + threadIdx.x], u += xs[q * S + threadIdx.x];
    part[(int64_t)blockIdx.x * 2 * S + threadIdx.x] = t;
    part[(int64_t)blockIdx.x * 2 * S + S + threadIdx.x] = u;
  }
}

// Accepted columns: the offset seed becomes rho and the scores take xhat;
// nodes where an accepted rho is non-zero are stamped so that the first
// propagation slot reads them (stamps are never removed here).  pbuf (rho)
// is cleared everywhere.
__global__ void k_ws_apply(int32_t n, int S, uint64_t accept, double *__restrict__ ybuf, double *__restrict__ pbuf,
                           double *__restrict__ r, const double *__restrict__ w, int32_t *__restrict__ stamp,
                           const Ctl *__restrict__ ctl) {
  const int32_t st = ctl->stamp;
  const int64_t total = (int64_t)n * S;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e % S);
    const double rho = pbuf[e];
    pbuf[e] = 0.0;
    if (!((accept >> j) & 1ull)) continue;
    ybuf[e] = rho;
    r[e] += w[e];
    if (rho != 0.0) stamp[e / S] = st;  // every writer stores the same value
  }
}

__global__ void k_ws_sigma(Ctl *ctl, int S, uint64_t accept, const double *__restrict__ xsum) {
  const int j = threadIdx.x;
  if (j < S && ((accept >> j) & 1ull)) ctl->sigma[j] += xsum[j];
}

// ------------------------------------------------------------ sparse residual
// For a region whose out-rows are a small part of the graph, rho is formed
// from the region alone: pbuf = (1-c) B~^T xhat' by a push over the region's
// out-rows (FP64 atomics into pbuf, which is zero at rest), and rho = q -
// xhat' + pbuf on U = region + its out-neighbours, the only nodes where it
// can be non-zero.  Out-neighbours outside the region are marked in hop1
// with WS_BOUNDARY until the apply pass.
#define WS_BOUNDARY (1 << 30)

template <int S>
__global__ void k_ws_push(const int32_t *__restrict__ R, DevGraphView out, const int32_t *__restrict__ item_off,
                          const int32_t *__restrict__ item_row, const int32_t *__restrict__ nitems_p,
                          const double *__restrict__ xhat, double c1, double *__restrict__ pbuf,
                          int32_t *__restrict__ hop1) {
  constexpr int PER = RWR_WAVE / S;
  const int lane = threadIdx.x % RWR_WAVE;
  const int j = lane % S, p = lane / S;
  const int32_t total = *nitems_p;
  for (int32_t it = (blockIdx.x * blockDim.x + threadIdx.x) / RWR_WAVE; it < total;
       it += gridDim.x * blockDim.x / RWR_WAVE) {
    const int32_t i = item_row[it], k = it - item_off[i];
    const int u = R[i];
    const int o = out.off[u], d = out.len[u];
    const double val = d ? c1 * xhat[(int64_t)i * S + j] / (double)d : 0.0;
    if (__ballot(val != 0.0) == 0ull) continue;
    const int e1 = min(d, (k + 1) * GRAD_CHUNK);
    for (int e = k * GRAD_CHUNK + p; e < e1; e += PER) {
      const int v = out.adj[o + e];
      if (val != 0.0) atomic_add_f64(&pbuf[col_index(v, S, j)], val);
      if (j == 0 && hop1[v] == 0) hop1[v] = WS_BOUNDARY;  // every writer stores the same value
    }
  }
}

// rho on U (see above), in place of the push sums in pbuf, and its signs in
// sg; partials as k_ws_rho
__global__ __launch_bounds__(WB) void k_ws_rho_sparse(int32_t n, int S, const int32_t *__restrict__ hop1,
                                                      const double *__restrict__ ybuf, double *__restrict__ pbuf,
                                                      const double *__restrict__ w, int8_t *__restrict__ sg,
                                                      double *__restrict__ part) {
  __shared__ double rn[WB], xs[WB];
  const int j = threadIdx.x % S, rl = threadIdx.x / S, RPB = WB / S;
  double a = 0.0, b = 0.0;
  for (int v = blockIdx.x * RPB + rl; v < n; v += gridDim.x * RPB) {
    if (hop1[v] == 0) continue;
    const int64_t kk = col_index(v, S, j);
    const double xw = w[kk];
    const double rho = ybuf[kk] + pbuf[kk] - xw;
    pbuf[kk] = rho;
    sg[kk] = (int8_t)(rho > 0.0 ? 1 : (rho < 0.0 ? -1 : 0));
    a += fabs(rho);
    b += xw;
  }
  rn[threadIdx.x] = a;
  xs[threadIdx.x] = b;
  __syncthreads();
  if (threadIdx.x < S) {
    double t = 0.0, u = 0.0;
    for (int q = 0; q < RPB; ++q) t += rn[q * S + threadIdx.x], u += xs[q * S + threadIdx.x];
    part[(int64_t)blockIdx.x * 2 * S + threadIdx.x] = t;
    part[(int64_t)blockIdx.x * 2 * S + S + threadIdx.x] = u;
  }
}

// accepted columns on U: the seed becomes rho, the scores take xhat'; pbuf
// (rho) back to zero on U
__global__ void k_ws_apply_sparse(int32_t n, int S, uint64_t accept, const int32_t *__restrict__ hop1,
                                  double *__restrict__ ybuf, double *__restrict__ pbuf, double *__restrict__ r,
                                  const double *__restrict__ w, int32_t *__restrict__ stamp,
                                  const Ctl *__restrict__ ctl) {
  const int32_t st = ctl->stamp;
  const int64_t total = (int64_t)n * S;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e % S);
    if (hop1[e / S] == 0) continue;
    const double rho = pbuf[e];
    pbuf[e] = 0.0;
    if (!((accept >> j) & 1ull)) continue;
    ybuf[e] = rho;
    r[e] += w[e];
    if (rho != 0.0) stamp[e / S] = st;  // every writer stores the same value
  }
}

__global__ void k_ws_unmark_boundary(int32_t n, int32_t *__restrict__ hop1) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    if (hop1[v] == WS_BOUNDARY) hop1[v] = 0;
}


// ------------------------------------------------------------ training
// Gradient of the training loss L = sum_j ||rho_j||_1 / sum_j ||q_j||_1 over
// the active columns (the columns with the largest residuals set the
// iteration count, and eps is absolute) with respect to the network output o
// (xhat = ||q|| o, corrected to xhat' = xhat - beta |xhat|, rho = q - (I - P)
// xhat', P = (1-c) B~^T).  With the correction held fixed:
//   d(u, j) = ||q_j|| (-(I - P)^T sign(rho_j))(u) / Q
//           = ||q_j|| (-sign(rho(u, j)) + (1-c)/d_out(u) sum over u -> v of sign(rho(v, j))) / Q,
//   Q = sum over active columns of ||q_j||_1,
// and through the correction exactly (beta depends on xhat):
//   dL/do(v, j) = (1 - beta_j s(v, j)) (d(v, j) - w_v ||q_j|| K_j / f_j),
//   K_j = sum_u d(u, j) |o(u, j)|,  f_j = f(|xhat_j|),  s = sign(o),
//   w_v = 1 for a dead end, c otherwise (the column sums of I - P).
// For the exact offset result, ||rho||_1 is the L1 distance between xhat and
// r_offset measured through I - P.  Out-rows are cut into items of
// GRAD_CHUNK edges (one wavefront each); every sum runs in a fixed order
// (item partials, then each row's items in order, then per-workgroup column
// partials and their sum), so the gradient does not depend on timing.
__device__ __forceinline__ double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

__global__ void k_ws_grad_items(const int32_t *__restrict__ R, int32_t nR, DevGraphView out,
                                int32_t *__restrict__ items) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= nR; i += gridDim.x * blockDim.x)
    items[i] = i < nR ? (out.len[R[i]] + GRAD_CHUNK - 1) / GRAD_CHUNK : 0;
}

// gpart[it * S + j] = sum of sign(rho(v, j)) over the out-edges u -> v of
// item it (sg: the signs, one byte each; the sums are integers, exact in
// any order)
template <int S>
__global__ void k_ws_grad_sum(const int32_t *__restrict__ R, int32_t nR, DevGraphView out,
                              const int32_t *__restrict__ item_off, const int32_t *__restrict__ item_row,
                              const int8_t *__restrict__ sg, double *__restrict__ gpart) {
  constexpr int PER = RWR_WAVE / S;
  const int lane = threadIdx.x % RWR_WAVE;
  const int j = lane % S, p = lane / S;
  const int32_t total = item_off[nR];
  for (int32_t it = (blockIdx.x * blockDim.x + threadIdx.x) / RWR_WAVE; it < total;
       it += gridDim.x * blockDim.x / RWR_WAVE) {
    const int32_t i = item_row[it], k = it - item_off[i];
    const int u = R[i];
    const int o = out.off[u], d = out.len[u];
    const int e1 = min(d, (k + 1) * GRAD_CHUNK);
    int t = 0;
    for (int e = k * GRAD_CHUNK + p; e < e1; e += PER) t += sg[col_index(out.adj[o + e], S, j)];
    for (int off = S; off < RWR_WAVE; off <<= 1) t += __shfl_xor(t, off, RWR_WAVE);
    if (p == 0) gpart[(int64_t)it * S + j] = (double)t;
  }
}

// d(u, j) with the correction held fixed (into dout), and per-workgroup
// partials of K_j = sum d |o| (entries blockIdx * S + j).  The grid stride
// is a multiple of S, so each thread keeps one column.
__global__ __launch_bounds__(WB) void k_ws_grad_fixed(const int32_t *__restrict__ R, int32_t nR, int S,
                                                      DevGraphView out, double c1, const double *__restrict__ rho,
                                                      const double *__restrict__ gpart,
                                                      const int32_t *__restrict__ item_off,
                                                      const int32_t *__restrict__ active,
                                                      const double *__restrict__ qn, double inv_q,
                                                      const float *__restrict__ o, float *__restrict__ dout,
                                                      double *__restrict__ kpart) {
  __shared__ double red[WB];
  const int64_t rows = (int64_t)nR * S;
  const int j = threadIdx.x % S;
  double kk = 0.0;
  for (int64_t row = blockIdx.x * (int64_t)WB + threadIdx.x; row < rows; row += (int64_t)gridDim.x * WB) {
    const int i = (int)(row / S);
    const int u = R[i];
    const int d = out.len[u];
    double t = 0.0;
    for (int32_t it = item_off[i]; it < item_off[i + 1]; ++it) t += gpart[(int64_t)it * S + j];
    const double g =
        active[j] ? (-sgn(rho[col_index(u, S, j)]) + (d ? c1 * t / (double)d : 0.0)) * qn[j] * inv_q : 0.0;
    dout[row] = (float)g;
    kk += (double)(float)g * fabs((double)o[row]);
  }
  red[threadIdx.x] = kk;
  __syncthreads();
  if (threadIdx.x < S) {
    double a = 0.0;
    for (int q = threadIdx.x; q < WB; q += S) a += red[q];
    kpart[(int64_t)blockIdx.x * S + threadIdx.x] = a;
  }
}

// corr[j] = ||q_j|| K_j / f_j, K_j from its partials (one workgroup per column,
// fixed order as in k_ws_sum_parts)
__global__ __launch_bounds__(WB) void k_ws_corr(const double *__restrict__ kpart, int nb, int S,
                                                const double *__restrict__ qn, const double *__restrict__ fa,
                                                double *__restrict__ corr) {
  __shared__ double red[WB];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += WB) s += kpart[(int64_t)b * S + j];
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double K = 0.0;
    for (int q = 0; q < WB; ++q) K += red[q];
    corr[j] = fa[j] > 0.0 ? qn[j] * K / fa[j] : 0.0;
  }
}

// dL/do through the correction: dout = (1 - beta s)(d - w ||q|| K / f)
__global__ void k_ws_grad_corr(const int32_t *__restrict__ R, int32_t nR, int S, DevGraphView out, double c1,
                               const double *__restrict__ corr, const double *__restrict__ beta,
                               const double *__restrict__ fa, const float *__restrict__ o,
                               float *__restrict__ dout) {
  const int64_t rows = (int64_t)nR * S;
  for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < rows;
       row += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(row % S);
    if (fa[j] <= 0.0) continue;
    const double w = out.len[R[row / S]] > 0 ? 1.0 - c1 : 1.0;
    const double s = sgn((double)o[row]);
    dout[row] = (float)((1.0 - beta[j] * s) * ((double)dout[row] - w * corr[j]));
  }
}

// ------------------------------------------------------------ host launchers
static int wgrid(int64_t work, int cap = 4096) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((work + WB - 1) / WB, cap));
}

size_t ws_select_temp_bytes(int32_t n) {
  size_t bytes = 0;
  (void)hipcub::DeviceSelect::Flagged(nullptr, bytes, hipcub::CountingInputIterator<int32_t>(0), (const int32_t *)nullptr,
                                      (int32_t *)nullptr, (int32_t *)nullptr, n);
  return bytes;
}

hipError_t ws_select(const int32_t *flags, int32_t n, int32_t *out, int32_t *count, void *temp, size_t temp_bytes,
                     hipStream_t s) {
  return hipcub::DeviceSelect::Flagged(temp, temp_bytes, hipcub::CountingInputIterator<int32_t>(0), flags, out, count,
                                       n, s);
}


int64_t ws_max_items(int32_t max_nodes, int64_t m) { return (int64_t)max_nodes + m / WS_ROW_CHUNK + 2; }

static hipError_t row_items(const ListRef &L, int32_t cap, const DevGraphView &gv, int32_t *tmp, int32_t *rit,
                            int32_t *irow, void *temp, size_t temp_bytes, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_row_chunks, dim3(wgrid((int64_t)cap + 1)), dim3(WB), 0, s, L, cap, gv, tmp);
  hipError_t e = hipcub::DeviceScan::ExclusiveSum(temp, temp_bytes, tmp, rit, cap + 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ws_item_rows, dim3(wgrid(cap)), dim3(WB), 0, s, L, rit, irow);
  return hipSuccess;
}

hipError_t ws_region(const int32_t *stamp, int32_t st, int32_t n, int32_t hops, int32_t max_nodes,
                     const DevGraphView &out, int32_t *hop1, int32_t *flags, int32_t *wlist, int32_t *kcnt,
                     int32_t *R, int32_t *lv, const WsItems &it, void *sel_temp, size_t sel_bytes, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_lv_init, dim3(1), dim3(64), 0, s, lv, 2 + WS_MAX_HOPS + 1);
  for (int h = 0; h <= hops; ++h) {
    if (h > 0) {
      const ListRef L{R, lv, h - 1};
      hipError_t e = row_items(L, max_nodes, out, it.tmp, it.rit, it.irow, it.scan_temp, it.scan_bytes, s);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_ws_expand, dim3(1024), dim3(WB), 0, s, L, it.rit, it.irow, out, h, hop1);
    }
    hipLaunchKernelGGL(k_ws_level_flags, dim3(wgrid(n)), dim3(WB), 0, s, stamp, st, n, h, hop1, flags);
    hipError_t e = ws_select(flags, n, wlist, kcnt, sel_temp, sel_bytes, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ws_append, dim3(wgrid(max_nodes)), dim3(WB), 0, s, wlist, kcnt, R, lv, max_nodes, hop1);
    hipLaunchKernelGGL(k_ws_append_fin, dim3(1), dim3(1), 0, s, kcnt, lv, h, max_nodes);
  }
  return hipSuccess;
}

hipError_t ws_local_rows(const int32_t *R, const int32_t *lv, int32_t nR, const DevGraphView &gv,
                         const int32_t *loc1, const WsItems &it, int32_t *cnt, int32_t *off, hipStream_t s) {
  const ListRef L{R, lv, -1};
  hipError_t e = row_items(L, nR, gv, it.tmp, it.rit, it.irow, it.scan_temp, it.scan_bytes, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ws_count_items, dim3(1024), dim3(WB), 0, s, L, it.rit, it.irow, it.max_items, gv, loc1,
                     it.icnt);
  size_t bytes = it.scan_bytes;
  e = hipcub::DeviceScan::ExclusiveSum(it.scan_temp, bytes, it.icnt, it.ioff, it.max_items + 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ws_row_off, dim3(wgrid((int64_t)nR + 1)), dim3(WB), 0, s, it.rit, it.ioff, nR, off, cnt);
  return hipSuccess;
}

void ws_local_fill(const int32_t *R, const int32_t *lv, const DevGraphView &gv, const int32_t *loc1,
                   const WsItems &it, int32_t *adj, hipStream_t s) {
  const ListRef L{R, lv, -1};
  hipLaunchKernelGGL(k_ws_fill_items, dim3(1024), dim3(WB), 0, s, L, it.rit, it.irow, gv, loc1, it.ioff, adj);
}

size_t ws_scan_temp_bytes(int32_t n) {
  size_t bytes = 0;
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, (const int32_t *)nullptr, (int32_t *)nullptr, n + 1);
  return bytes;
}


__global__ void k_ws_chunks(const int32_t *__restrict__ cnt, int32_t nR, int32_t chunk, int32_t *__restrict__ items) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= nR; i += gridDim.x * blockDim.x)
    items[i] = i < nR ? (cnt[i] + chunk - 1) / chunk : 0;
}

hipError_t ws_chunk_items(const int32_t *cnt, int32_t nR, int32_t chunk, int32_t *tmp, int32_t *items, void *temp,
                          size_t temp_bytes, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_chunks, dim3(wgrid((int64_t)nR + 1)), dim3(WB), 0, s, cnt, nR, chunk, tmp);
  return hipcub::DeviceScan::ExclusiveSum(temp, temp_bytes, tmp, items, nR + 1, s);
}


void ws_loc(const int32_t *R, int32_t nR, const DevGraphView &out, int32_t *loc1, float *dinv, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_loc, dim3(wgrid(nR)), dim3(WB), 0, s, R, nR, out, loc1, dinv);
}

void ws_clear(const int32_t *R, int32_t nR, int32_t *hop1, int32_t *loc1, hipStream_t s) {
  if (nR <= 0) return;
  hipLaunchKernelGGL(k_ws_clear, dim3(wgrid(nR)), dim3(WB), 0, s, R, nR, hop1, loc1);
}

void ws_qnorm(const int32_t *R, int32_t n0, int S, const double *ybuf, double *part, double *qn, hipStream_t s) {
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)n0 * S + WB - 1) / WB, 1024));
  hipLaunchKernelGGL(k_ws_qnorm, dim3(nb), dim3(WB), 0, s, R, n0, S, ybuf, part);
  hipLaunchKernelGGL(k_ws_sum_parts, dim3(2 * S), dim3(WB), 0, s, part, nb, 2 * S, qn);
}

void ws_features(const int32_t *R, int32_t nR, int S, const int32_t *hop1, const DevGraphView &in,
                 const DevGraphView &out, const double *ybuf, const double *r, const Ctl *ctl, const int32_t *seeds,
                 const double *qn, int32_t n_total, float *F, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_features, dim3(wgrid((int64_t)nR * S)), dim3(WB), 0, s, R, nR, S, hop1, in, out, ybuf, r,
                     ctl, seeds, qn, n_total, F);
}

void ws_predict(const int32_t *R, int32_t nR, int S, const DevGraphView &out, const float *o, const double *qn,
                double c1, double *xhat, double *w, double *part, double *beta, double *fa, hipStream_t s) {
  const int g = wgrid((int64_t)nR * S);
  hipLaunchKernelGGL(k_ws_predict, dim3(g), dim3(WB), 0, s, nR, S, o, qn, xhat);
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)nR * S + WB - 1) / WB, 512));
  hipLaunchKernelGGL(k_ws_mass, dim3(nb), dim3(WB), 0, s, R, nR, S, out, xhat, part);
  hipLaunchKernelGGL(k_ws_beta, dim3(S), dim3(WB), 0, s, part, nb, S, c1, qn, beta, fa);
  hipLaunchKernelGGL(k_ws_adjust_scatter, dim3(g), dim3(WB), 0, s, R, nR, S, beta, xhat, w);
}

void ws_unscatter(const int32_t *R, int32_t nR, int S, double *w, hipStream_t s) {
  if (nR <= 0) return;
  hipLaunchKernelGGL(k_ws_unscatter, dim3(wgrid((int64_t)nR * S)), dim3(WB), 0, s, R, nR, S, w);
}

void ws_rho(int32_t n, int S, const double *ybuf, double *pbuf, const double *w, int8_t *sg, double *part,
            double *sums, hipStream_t s) {
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)n * S + WB - 1) / WB, 1024));
  hipLaunchKernelGGL(k_ws_rho, dim3(nb), dim3(WB), 0, s, n, S, ybuf, pbuf, w, sg, part);
  hipLaunchKernelGGL(k_ws_sum_parts, dim3(2 * S), dim3(WB), 0, s, part, nb, 2 * S, sums);
}

void ws_apply(int32_t n, int S, uint64_t accept, double *ybuf, double *pbuf, double *r, const double *w,
              int32_t *stamp, Ctl *ctl, const double *xsum, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_apply, dim3(wgrid((int64_t)n * S)), dim3(WB), 0, s, n, S, accept, ybuf, pbuf, r, w, stamp,
                     ctl);
  if (accept) hipLaunchKernelGGL(k_ws_sigma, dim3(1), dim3(64), 0, s, ctl, S, accept, xsum);
}

hipError_t ws_resid_grad(const int32_t *R, int32_t nR, int S, const DevGraphView &out, double c1, const double *rho,
                         const int8_t *sg, double *gpart, int32_t *items, int32_t *item_off, int32_t *item_row,
                         void *temp,
                         size_t temp_bytes, const int32_t *active, double q_active, const float *o, const double *qn,
                         const double *beta, const double *fa, double *kpart, double *corr, float *dout,
                         hipStream_t s) {
  (void)items;
  (void)temp;
  (void)temp_bytes;
  switch (S) {
#define WS_GRAD(SS)                                                                                              \
  case SS:                                                                                                       \
    hipLaunchKernelGGL(k_ws_grad_sum<SS>, dim3(1024), dim3(WB), 0, s, R, nR, out, item_off, item_row, sg, gpart); \
    break;
    WS_GRAD(1)
    WS_GRAD(2)
    WS_GRAD(4)
    WS_GRAD(8)
    WS_GRAD(16)
    WS_GRAD(32)
    WS_GRAD(64)
#undef WS_GRAD
    default:
      break;
  }
  const double inv = q_active > 0.0 ? 1.0 / q_active : 0.0;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)nR * S + WB - 1) / WB, WS_KPART_BLOCKS));
  hipLaunchKernelGGL(k_ws_grad_fixed, dim3(nb), dim3(WB), 0, s, R, nR, S, out, c1, rho, gpart, item_off, active, qn,
                     inv, o, dout, kpart);
  hipLaunchKernelGGL(k_ws_corr, dim3(S), dim3(WB), 0, s, kpart, nb, S, qn, fa, corr);
  hipLaunchKernelGGL(k_ws_grad_corr, dim3(wgrid((int64_t)nR * S)), dim3(WB), 0, s, R, nR, S, out, c1, corr, beta, fa,
                     o, dout);
  return hipSuccess;
}

hipError_t ws_out_items(const int32_t *R, int32_t nR, const DevGraphView &out, int32_t *items, int32_t *item_off,
                        int32_t *item_row, void *temp, size_t temp_bytes, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_grad_items, dim3(wgrid((int64_t)nR + 1)), dim3(WB), 0, s, R, nR, out, items);
  hipError_t e = hipcub::DeviceScan::ExclusiveSum(temp, temp_bytes, items, item_off, nR + 1, s);
  if (e != hipSuccess) return e;
  gnn::region_item_rows(item_off, nR, item_row, s);
  return hipSuccess;
}

void ws_rho_push(const int32_t *R, int32_t nR, int S, const DevGraphView &out, const int32_t *item_off,
                 const int32_t *item_row, const double *xhat, double c1, double *pbuf, int32_t *hop1, int32_t n,
                 const double *ybuf, const double *w, int8_t *sg, double *part, double *sums, hipStream_t s) {
  switch (S) {
#define WS_PUSH(SS)                                                                                              \
  case SS:                                                                                                       \
    hipLaunchKernelGGL(k_ws_push<SS>, dim3(2048), dim3(WB), 0, s, R, out, item_off, item_row, item_off + nR, xhat, \
                       c1, pbuf, hop1);                                                                          \
    break;
    WS_PUSH(1)
    WS_PUSH(2)
    WS_PUSH(4)
    WS_PUSH(8)
    WS_PUSH(16)
    WS_PUSH(32)
    WS_PUSH(64)
#undef WS_PUSH
    default:
      break;
  }
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)n * S + WB - 1) / WB, 1024));
  hipLaunchKernelGGL(k_ws_rho_sparse, dim3(nb), dim3(WB), 0, s, n, S, hop1, ybuf, pbuf, w, sg, part);
  hipLaunchKernelGGL(k_ws_sum_parts, dim3(2 * S), dim3(WB), 0, s, part, nb, 2 * S, sums);
}

void ws_apply_sparse(int32_t n, int S, uint64_t accept, const int32_t *hop1, double *ybuf, double *pbuf, double *r,
                     const double *w, int32_t *stamp, Ctl *ctl, const double *xsum, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_apply_sparse, dim3(wgrid((int64_t)n * S)), dim3(WB), 0, s, n, S, accept, hop1, ybuf, pbuf, r,
                     w, stamp, ctl);
  if (accept) hipLaunchKernelGGL(k_ws_sigma, dim3(1), dim3(64), 0, s, ctl, S, accept, xsum);
}

void ws_unmark_boundary(int32_t n, int32_t *hop1, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_unmark_boundary, dim3(wgrid(n)), dim3(WB), 0, s, n, hop1);
}
