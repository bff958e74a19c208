// Shared definitions of the HIP dynamic-RWR library (device + host).
//
// Data layout in HBM (one context, S = padded seed-column count, n_cap = node
// capacity):
//   graph, per orientation (out = rows of A~ / CSR, in = columns / CSC):
//     off[n_cap], len[n_cap], cap[n_cap] int32 -- row v occupies
//     adj[off[v] .. off[v]+len[v]) of an int32 array with per-row slack
//     (cap[v] >= len[v]) followed by a relocation arena; out.len[] is d_out.
//   scores r[n_cap*S] FP64, node-major (column j of node v at v*S + j), kept
//     un-normalised; sigma[j] = sum_v r[v,j] is tracked so that the scores
//     are r / sigma (Theorem 4's rescaling).
//   x[2][n_cap*S] in the propagation type (FP32 or FP64): the pre-scaled
//     vectors x^(i)[v] / d_out(v) of two consecutive iterations.
//   ybuf[n_cap*S] FP64: scatter target of the offset seed and of push
//     iterations; all zero between uses.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#define RWR_MAX_COLS 64
#define RWR_WAVE 64

// propagation phase of the current iteration slot
enum : int32_t { MODE_SPARSE = 0, MODE_DENSE = 1, MODE_DONE = 2 };

// error word values (same numbers as rwr_status)
enum : int32_t {
  ERR_OK = 0,
  ERR_EINVAL = -1,
  ERR_ENOMEM = -2,
  ERR_EEXIST = -4,
  ERR_ENOENT = -5,
  ERR_ENOCONV = -6,
  ERR_ENUMERIC = -7,
};

// Device control block: one per context, in device memory.  Written by the
// kernels' last-arriving workgroups, read by the host after a sync.
struct Ctl {
  int32_t err;          // first batch error (0 = none)
  int32_t prop_err;     // propagation error (ENOCONV / ENUMERIC)
  int32_t mode;         // MODE_* of the next iteration slot
  int32_t iter;         // iterations completed (x^(iter) is the newest)
  int32_t stamp;        // frontier stamp of the frontier being built
  int32_t max_iters;
  int32_t n_active;     // columns still propagating
  int32_t ended_dense;  // some dense sweep ran during this propagation
  int32_t lockstep;     // columns retire together, when the last of them passes the stop test
  int32_t fcount[2];    // frontier sizes (frontier of x^(i) is list i % 2)
  int32_t nT[2];        // touched rows per orientation (0 = out/CSR, 1 = in/CSC)
  uint32_t done_blocks; // last-arriver counter of the current kernel
  int32_t dense_iters;
  int32_t heavy_stale;  // rows that became heavy since the last schedule
  int32_t hist_base;    // first history row of this run (update runs 0, refinements after them)
  int64_t fedges;       // out-edges of the frontier being built
  uint64_t hpack;       // long push rows of this slot: count << 32 | chunks
  int64_t visited;      // edges read by propagation in this run
  int64_t demand[2];    // arena slots needed by relocated rows of this batch
  uint64_t tail[2];     // first free slot of each orientation's arena
  int64_t dense_thresh; // switch to dense once fedges exceeds this
  int64_t dense_nodes;  // ... or once the frontier holds more nodes than this
  int64_t node_dels;    // stored adjacency entries removed by this batch's node deletions
  int64_t seed_recs[32]; // old degrees summed over the touched rows (out orientation), in 32 parts
  int32_t nbig_v;       // rows above BIG_ROW left to the workgroup check
  int32_t nbig_a;       // rows above BIG_ROW left to the workgroup apply
  double eps;           // stop tolerance of this run
  int32_t active[RWR_MAX_COLS];
  double sigma[RWR_MAX_COLS];     // running sum of r per column
  double last_norm[RWR_MAX_COLS]; // ||x^(iter)||_1 of each column when it stopped
  double red_norm[RWR_MAX_COLS];  // scratch: ||.||_1 of the current kernel
  double red_sum[RWR_MAX_COLS];   // scratch: signed sum of the current kernel
  double norm0[RWR_MAX_COLS];     // ||x^(0)||_1 of this run
  double norm1[RWR_MAX_COLS];     // ||x^(1)||_1 of this run
  double sum_norm[RWR_MAX_COLS];  // sum over the run's iterations of ||x^(i)||_1
  int32_t last_it[RWR_MAX_COLS];  // iteration of last_norm
  double dr_l1[RWR_MAX_COLS];     // ||D r_old||_1 of the batch (D: row L1 norms of B~ - A~)
  int32_t inj[RWR_MAX_COLS];      // the column's pending carried vector joined this run
  uint64_t dr_fix[RWR_MAX_COLS];  // dr_l1 in fixed point (2^-52 units), summed in deterministic mode
};
// the host copies the block whole: host and device compilations must agree
// on its layout
static_assert(sizeof(Ctl) == 5800 && offsetof(Ctl, seed_recs) == 152 && offsetof(Ctl, nbig_a) == 412 &&
                  offsetof(Ctl, dr_fix) == 5288,
              "control block layout");

// history of per-iteration norms: hist[i * S + j] = ||x^(i)[:, j]||_1

#ifdef __HIPCC__

template <typename T>
__device__ __forceinline__ T wave_xor_sum(T v, int lane_mask_start, int width) {
  for (int off = lane_mask_start; off < width; off <<= 1) v += __shfl_xor(v, off, RWR_WAVE);
  return v;
}

__device__ __forceinline__ void atomic_add_f64(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_f32(float *p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ double atomic_add_f64_ret(double *p, double v) { return unsafeAtomicAdd(p, v); }

template <typename T>
__device__ __forceinline__ void atomic_add_any(T *p, T v);
template <>
__device__ __forceinline__ void atomic_add_any<double>(double *p, double v) {
  atomic_add_f64(p, v);
}
template <>
__device__ __forceinline__ void atomic_add_any<float>(float *p, float v) {
  atomic_add_f32(p, v);
}

__device__ __forceinline__ void set_error(Ctl *ctl, int32_t code) { atomicCAS(&ctl->err, 0, code); }

__device__ __forceinline__ int64_t col_index(int64_t v, int S, int j) { return v * (int64_t)S + j; }

#endif
