// Cumulative propagation of Section 2.2 / Algorithm 1 on the device:
//   x^(i) = (1-c) B~^T x^(i-1),  r += x^(i),  stop when ||x^(i)||_1 <= eps.
//
// Vectors are kept pre-scaled: the stored x-buffers hold xh(v) = x(v)/d_out(v)
// (0 for dead ends), so that (B~^T x)(v) = sum over in-neighbours u of xh(u)
// and a gather reads one value per edge.  Two phases, chosen per iteration:
//   sparse: push over the out-rows of the frontier (nodes with x != 0) with
//           FP64 atomics into ybuf, then an epilogue over the stamped nodes;
//   dense : pull over the in-rows of every node.  In-rows longer than the
//           heavy limit are cut into chunks (one wavefront each for one
//           seed column, one workgroup each for several).
// Every epilogue is fused: accumulate into r (FP64), L1 norm and signed sum
// per seed column, and the next pre-scaled vector.
//
// No workgroup waits for another inside a kernel.  Each workgroup writes its
// partial sums (and each heavy-row chunk its partial row sum) with plain
// stores; the heavy rows are finished by a small follow-up kernel or, when
// there are few, by the decision kernel: a single workgroup (k_decide) that
// adds all partials in a fixed order (deterministic), records ||x^(i)||_1,
// retires converged columns and picks the phase of the next iteration.
// Every kernel of an iteration slot first checks that phase and the parity
// of the iteration count, so the host can enqueue slots without waiting;
// slots after convergence, or of the phase not in effect, exit at once.
// Grids are sized to the resident capacity of the chip and loop over their
// work.
#include <math.h>

#include <type_traits>

#include "rwr_common.h"
#include "rwr_kernels.h"

#define BLOCK 256
#define NWAVES (BLOCK / RWR_WAVE)
#define DECIDE_BLOCK 1024

enum { KIND_SPARSE = 0, KIND_DENSE = 1, KIND_REFINE = 2, KIND_RESID = 3, KIND_SIGMA = 4 };

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (RWR_WAVE - lane));
}

// A kernel of iteration slot k runs only while the run is in its phase and
// at an iteration of k's parity: slots of both phases may then be enqueued
// for the same k (exactly one of them runs; the kernels use k only through
// its parity, so a slot enqueued for k runs correctly as any iteration of
// that parity).
__device__ __forceinline__ bool slot_live(const Ctl *ctl, int mode, int k) {
  return ctl->mode == mode && ((ctl->iter ^ k) & 1) == 0;
}

// ------------------------------------------------------------------ partials
// Partial-sum entry e: S columns x {norm, sum} at part[e * stride], two
// counters at part_i[e * 16].  Entries are padded to at least 128 bytes.
template <int S>
__device__ __forceinline__ int64_t entry_stride() {
  return 2 * S < 16 ? 16 : 2 * S;
}

struct BlockRed {
  double wn[NWAVES][RWR_MAX_COLS];
  double ws[NWAVES][RWR_MAX_COLS];
  int64_t wi[NWAVES][2];
};

// Sum the workgroup's per-thread values (nrm/sm of column lane % S, counters
// ia/ib) and store them as entry `e`.
template <int S>
__device__ void block_publish(double nrm, double sm, int64_t ia, int64_t ib, double *part, int64_t *part_i, int e,
                              BlockRed &sh) {
  const int lane = threadIdx.x % RWR_WAVE, w = threadIdx.x / RWR_WAVE;
  nrm = wave_xor_sum(nrm, S, RWR_WAVE);
  sm = wave_xor_sum(sm, S, RWR_WAVE);
  ia = wave_xor_sum(ia, 1, RWR_WAVE);
  ib = wave_xor_sum(ib, 1, RWR_WAVE);
  if (lane < S) {
    sh.wn[w][lane] = nrm;
    sh.ws[w][lane] = sm;
  }
  if (lane == 0) {
    sh.wi[w][0] = ia;
    sh.wi[w][1] = ib;
  }
  __syncthreads();
  if (threadIdx.x < S) {
    double a = 0.0, b = 0.0;
    for (int ww = 0; ww < NWAVES; ++ww) a += sh.wn[ww][threadIdx.x], b += sh.ws[ww][threadIdx.x];
    part[e * entry_stride<S>() + 2 * threadIdx.x] = a;
    part[e * entry_stride<S>() + 2 * threadIdx.x + 1] = b;
  }
  if (threadIdx.x == 0) {
    int64_t a = 0, b = 0;
    for (int ww = 0; ww < NWAVES; ++ww) a += sh.wi[ww][0], b += sh.wi[ww][1];
    part_i[(int64_t)e * 16] = a;
    part_i[(int64_t)e * 16 + 1] = b;
  }
}

// ------------------------------------------------------------------ decide
struct DecideShared {
  double wn[DECIDE_BLOCK / RWR_WAVE][RWR_MAX_COLS];
  double ws[DECIDE_BLOCK / RWR_WAVE][RWR_MAX_COLS];
  int64_t wi[DECIDE_BLOCK / RWR_WAVE][2];
  double s_norm[RWR_MAX_COLS];
  double s_sum[RWR_MAX_COLS];
  int64_t s_i[2];
  int s_active;  // columns still above eps
  int s_nact;    // columns active in this iteration
  int s_bad;  // a column's norm or sum is not finite
  int s_last;    // this workgroup arrived last
};

// workgroups of the decision kernel: each reduces a slice of the entries,
// the last to arrive adds their totals in workgroup order and decides
#define DECIDE_GRID 16

template <typename XT, int S, int KIND>
__device__ __forceinline__ void pull_epilogue(const SlotArgs &a, XT *__restrict__ xnext, int v, int j, double y,
                                              bool act, double &nrm, double &sm);

// Totals of entries 0..count-1, then the decision of the iteration (kind
// SPARSE/DENSE/REFINE), or the residual / column-sum results.  With `fold`
// (after a dense or residual sweep with few heavy rows) the heavy rows are
// finished here first: chunk sums added in order, row epilogue.  Every sum
// runs in a fixed order: strided per thread, then a shuffle tree in each
// wave, then the waves in index order, then (several workgroups) the
// workgroups' totals in workgroup order, added by the workgroup that arrives
// last (it publishes through entries count .. count + gridDim.x - 1, which
// the partial buffers hold beyond every sweep's entries).
template <typename XT, int S>
__global__ __launch_bounds__(DECIDE_BLOCK) void k_decide(SlotArgs a, int kind, int count, int new_list, int fold) {
  __shared__ DecideShared sh;
  constexpr int NW = DECIDE_BLOCK / RWR_WAVE;
  Ctl *ctl = a.ctl;
  constexpr int TPC = DECIDE_BLOCK / S;
  const int t = threadIdx.x, j = t % S;
  const int nb = gridDim.x, TPCG = TPC * nb;
  const int q = blockIdx.x * TPC + t / S;  // this thread's place among the column's threads of all workgroups
  const int lane = t % RWR_WAVE, w = t / RWR_WAVE;
  // The control values this kernel reads are loaded up front, together with
  // the partials below, so that their latencies overlap (the slot test would
  // otherwise hold every later load back).  Only this kernel writes them.
  const int mode0 = ctl->mode, it = ctl->iter;
  const bool actj = ctl->active[j] != 0;
  const double eps0 = ctl->eps;
  const int hb = ctl->hist_base;
  const int lock = ctl->lockstep;
  double sig0 = 0.0, sumn0 = 0.0;
  if (t < S) {
    sig0 = ctl->sigma[t];
    sumn0 = ctl->sum_norm[t];
  }
  int perr0 = 0, maxit = 0, dit = 0, stp = 0;
  int64_t fed = 0, dth = 0, dno = 0, vis = 0;
  if (t == 0) {
    perr0 = ctl->prop_err;
    maxit = ctl->max_iters;
    dit = ctl->dense_iters;
    stp = ctl->stamp;
    fed = ctl->fedges;
    dth = ctl->dense_thresh;
    dno = ctl->dense_nodes;
    vis = ctl->visited;
  }
  // heavy rows to finish here (at most two per thread, see fold_max): their
  // row data is loaded first, so that it arrives with the partials
  const int nh = fold ? a.heavy.n_rows : 0;
  int hf[2] = {0, 0}, hc[2] = {0, 0}, hv[2] = {0, 0};
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int h = q + u * TPCG;
    if (h < nh) {
      hf[u] = a.heavy.first[h];
      hc[u] = a.heavy.nchunks[h];
      hv[u] = a.heavy.rows[h];
    }
  }
  // eight partials per step in flight, into eight sums added in a fixed order
  double A, B;
  {
    constexpr int R = 8;
    double av[R], bv[R];
#pragma unroll
    for (int u = 0; u < R; ++u) av[u] = bv[u] = 0.0;
    const double *__restrict__ pp = a.part + 2 * j;
    const int64_t ES = entry_stride<S>();
    int e = q;
    for (; e + (R - 1) * TPCG < count; e += R * TPCG) {
#pragma unroll
      for (int u = 0; u < R; ++u) {
        av[u] += pp[(int64_t)(e + u * TPCG) * ES];
        bv[u] += pp[(int64_t)(e + u * TPCG) * ES + 1];
      }
    }
    for (; e < count; e += TPCG) {
      av[0] += pp[(int64_t)e * ES];
      bv[0] += pp[(int64_t)e * ES + 1];
    }
    A = ((av[0] + av[1]) + (av[2] + av[3])) + ((av[4] + av[5]) + (av[6] + av[7]));
    B = ((bv[0] + bv[1]) + (bv[2] + bv[3])) + ((bv[4] + bv[5]) + (bv[6] + bv[7]));
  }
  // a slot enqueued past the end of the run, or of the other phase
  const bool live_par = ((it ^ new_list) & 1) == 0;
  if (kind == KIND_SPARSE && !(mode0 == MODE_SPARSE && live_par)) return;
  if (kind == KIND_DENSE && !(mode0 == MODE_DENSE && live_par)) return;
  if (nh > 0) {
    const double c1 = 1.0 - a.c;
    const bool act = actj;
    XT *__restrict__ xnext = (XT *)a.x[new_list];
    double hn = 0.0, hs = 0.0;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (q + u * TPCG >= nh) break;
      double y = 0.0;
      for (int qq = 0; qq < hc[u]; ++qq) y += a.heavy.part[(int64_t)(hf[u] + qq) * S + j];
      if (kind == KIND_RESID)
        pull_epilogue<double, S, KIND_RESID>(a, nullptr, hv[u], j, c1 * y, act, hn, hs);
      else
        pull_epilogue<XT, S, KIND_DENSE>(a, xnext, hv[u], j, c1 * y, act, hn, hs);
    }
    A += hn;
    B += hs;
  }
  // frontier counters: only a sparse slot publishes them
  int64_t ia = 0, ib = 0;
  if (kind == KIND_SPARSE) {
    for (int e = blockIdx.x * DECIDE_BLOCK + t; e < count; e += nb * DECIDE_BLOCK) {
      ia += a.part_i[(int64_t)e * 16];
      ib += a.part_i[(int64_t)e * 16 + 1];
    }
  }
  A = wave_xor_sum(A, S, RWR_WAVE);
  B = wave_xor_sum(B, S, RWR_WAVE);
  ia = wave_xor_sum(ia, 1, RWR_WAVE);
  ib = wave_xor_sum(ib, 1, RWR_WAVE);
  if (lane < S) {
    sh.wn[w][lane] = A;
    sh.ws[w][lane] = B;
  }
  if (lane == 0) {
    sh.wi[w][0] = ia;
    sh.wi[w][1] = ib;
  }
  if (t == 0) {
    sh.s_active = 0;
    sh.s_nact = 0;
    sh.s_bad = 0;
  }
  __syncthreads();
  if (t < S) {
    double X = 0.0, Y = 0.0;
    for (int ww = 0; ww < NW; ++ww) X += sh.wn[ww][t], Y += sh.ws[ww][t];
    sh.s_norm[t] = X;
    sh.s_sum[t] = Y;
  }
  if (t == 0) {
    int64_t X = 0, Y = 0;
    for (int ww = 0; ww < NW; ++ww) X += sh.wi[ww][0], Y += sh.wi[ww][1];
    sh.s_i[0] = X;
    sh.s_i[1] = Y;
  }
  __syncthreads();
  if (nb > 1) {
    const int64_t ES = entry_stride<S>();
    const int64_t se = (int64_t)count + blockIdx.x;
    if (t < S) {
      a.part[se * ES + 2 * t] = sh.s_norm[t];
      a.part[se * ES + 2 * t + 1] = sh.s_sum[t];
    }
    if (t == 0) {
      a.part_i[se * 16] = sh.s_i[0];
      a.part_i[se * 16 + 1] = sh.s_i[1];
    }
    // release this workgroup's totals, then count the arrival
    __threadfence();
    __syncthreads();
    if (t == 0) sh.s_last = atomicAdd(&ctl->done_blocks, 1u) == (unsigned)(nb - 1);
    __syncthreads();
    if (!sh.s_last) return;
    // acquire the other workgroups' totals
    __threadfence();
    if (t < S) {
      double X = 0.0, Y = 0.0;
      for (int bb = 0; bb < nb; ++bb) {
        X += a.part[((int64_t)count + bb) * ES + 2 * t];
        Y += a.part[((int64_t)count + bb) * ES + 2 * t + 1];
      }
      sh.s_norm[t] = X;
      sh.s_sum[t] = Y;
    }
    if (t == 0) {
      ctl->done_blocks = 0;
      int64_t X = 0, Y = 0;
      for (int bb = 0; bb < nb; ++bb) {
        X += a.part_i[((int64_t)count + bb) * 16];
        Y += a.part_i[((int64_t)count + bb) * 16 + 1];
      }
      sh.s_i[0] = X;
      sh.s_i[1] = Y;
    }
    __syncthreads();
  }
  if (kind == KIND_RESID || kind == KIND_SIGMA) {
    if (t < S) {
      ctl->red_norm[t] = sh.s_norm[t];
      ctl->red_sum[t] = sh.s_sum[t];
      ctl->sigma[t] = sh.s_sum[t];
    }
    return;
  }
  if (t < S) {
    const double nr = sh.s_norm[t];
    const double su = sh.s_sum[t];
    a.hist[(int64_t)(hb + it) * S + t] = actj ? nr : 0.0;
    if (actj) {
      ctl->sigma[t] = sig0 + su;
      ctl->last_norm[t] = nr;
      ctl->last_it[t] = it;
      ctl->sum_norm[t] = sumn0 + nr;
      if (it == 0) ctl->norm0[t] = nr;
      if (it == 1) ctl->norm1[t] = nr;
      if (!isfinite(nr) || !isfinite(su)) {
        ctl->prop_err = ERR_ENUMERIC;
        sh.s_bad = 1;
      }
      const bool conv = it >= 1 && nr <= eps0;
      if (!conv) atomicAdd(&sh.s_active, 1);
      if (conv && !lock) ctl->active[t] = 0;
      atomicAdd(&sh.s_nact, 1);
    }
  }
  __syncthreads();
  // lockstep: the columns retire together once none is left above eps
  if (lock && t < S && actj && sh.s_active == 0) ctl->active[t] = 0;
  if (t == 0) {
    const int na = lock ? (sh.s_active > 0 ? sh.s_nact : 0) : sh.s_active;
    ctl->n_active = na;
    ctl->iter = it + 1;
    // the push of a sparse slot read the out-rows of the previous frontier
    if (kind == KIND_SPARSE) ctl->visited = vis + fed;
    if (kind == KIND_DENSE) ctl->dense_iters = dit + 1;
    if (kind == KIND_DENSE || kind == KIND_REFINE) ctl->ended_dense = 1;
    int mode = mode0;
    if (perr0 != 0 || sh.s_bad || na == 0) {
      mode = MODE_DONE;
    } else if (it >= maxit) {
      mode = MODE_DONE;
      ctl->prop_err = ERR_ENOCONV;
    } else if (kind == KIND_REFINE) {
      mode = MODE_DENSE;
    } else if (kind == KIND_SPARSE && (sh.s_i[0] > dth || sh.s_i[1] > dno)) {
      mode = MODE_DENSE;
    }
    ctl->fedges = kind == KIND_SPARSE ? sh.s_i[0] : 0;
    if (kind == KIND_SPARSE) ctl->fcount[new_list] = (int32_t)sh.s_i[1];
    ctl->stamp = stp + 1;
    ctl->hpack = 0;
    ctl->mode = mode;
  }
}

// ------------------------------------------------------------------ sparse
#define PUSH_LIGHT_MAX 128
#define PUSH_CHUNK 2048

// Sparse push, light part: G lanes per frontier node (frontier stamp = slot
// stamp - 1) with at most PUSH_LIGHT_MAX out-edges.  Every edge adds xh(u)
// into ybuf[v] (non-returning FP64 atomics) and stamps v (plain store; the
// epilogue scans the stamps).  A longer row gets a slot in the long-row list
// and a range of chunk numbers from one 64-bit atomic (slot in the high half,
// chunk base in the low half), so the chunk bases increase with the slot.
// Each wavefront tests 64 consecutive nodes at once (one coalesced load of
// their frontier stamps) and hands the frontier nodes among them to its
// groups of G lanes, one node per group at a time.
template <typename XT, int S, int G>
__global__ __launch_bounds__(BLOCK) void k_push(SlotArgs a, int k) {
  Ctl *ctl = a.ctl;
  if (!slot_live(ctl, MODE_SPARSE, k)) return;
  const int cur = (k - 1) & 1;
  const XT *__restrict__ xcur = (const XT *)a.x[cur];
  const int32_t st = ctl->stamp;
  constexpr int P = G / S;
  constexpr int GPW = RWR_WAVE / G;  // groups per wavefront
  const int lane = threadIdx.x % RWR_WAVE, gl = lane % G, j = gl % S, p = gl / S, grp = lane / G;
  const int nwv = gridDim.x * (BLOCK / RWR_WAVE);
  for (int base = (blockIdx.x * (BLOCK / RWR_WAVE) + threadIdx.x / RWR_WAVE) * RWR_WAVE; base < a.n;
       base += nwv * RWR_WAVE) {
    const int ul = base + lane;
    // frontier of x^(k-1) among the 64 nodes (the mask is the same in every lane)
    unsigned long long m = __ballot(ul < a.n && a.fstamp[ul] == st - 1);
    while (m) {
      // group grp takes the grp-th lowest frontier node left in m
      unsigned long long mm = m;
      for (int q = 0; q < grp; ++q) mm &= mm - 1;
#pragma unroll
      for (int q = 0; q < GPW; ++q) m &= m - 1;
      if (!mm) continue;
      const int u = base + __builtin_ctzll(mm);
      const int d = a.out.len[u];
      if (d > PUSH_LIGHT_MAX) {
        if (gl == 0) {
          const unsigned long long nch = (unsigned long long)((d + PUSH_CHUNK - 1) / PUSH_CHUNK);
          const unsigned long long old = atomicAdd((unsigned long long *)&ctl->hpack, (1ull << 32) | nch);
          const int slot = (int)(old >> 32);
          a.hfront[slot] = u;
          a.hbase[slot] = (int32_t)(old & 0xffffffffull);
        }
        continue;
      }
      const XT xv = xcur[col_index(u, S, j)];
      const int o = a.out.off[u];
      for (int e = p; e < d; e += P) {
        const int v = a.out.adj[o + e];
        if (xv != (XT)0) atomic_add_f64(&a.ybuf[col_index(v, S, j)], (double)xv);
        if (j == 0) a.stamp[v] = st;
      }
    }
  }
}

#define HBASE_LDS 2048

// Sparse push, long rows: chunk c (of all listed rows) goes to workgroup
// c mod grid; its row is found by binary search over the chunk bases.
template <typename XT, int S>
__global__ __launch_bounds__(BLOCK) void k_push_heavy(SlotArgs a, int k) {
  __shared__ int32_t s_base[HBASE_LDS];
  Ctl *ctl = a.ctl;
  if (!slot_live(ctl, MODE_SPARSE, k)) return;
  const unsigned long long pk = ctl->hpack;
  const int nh = (int)(pk >> 32);
  const int total = (int)(pk & 0xffffffffull);
  if (nh == 0) return;
  const int cur = (k - 1) & 1;
  const XT *__restrict__ xcur = (const XT *)a.x[cur];
  const int32_t st = ctl->stamp;
  constexpr int PP = RWR_WAVE / S;
  const int lane = threadIdx.x % RWR_WAVE, w = threadIdx.x / RWR_WAVE;
  const int j = lane % S, pp = lane / S;
  const bool in_lds = nh <= HBASE_LDS;
  if (in_lds) {
    for (int i = threadIdx.x; i < nh; i += BLOCK) s_base[i] = a.hbase[i];
    __syncthreads();
  }
  for (int ch = blockIdx.x; ch < total; ch += gridDim.x) {
    int lo = 0, hi = nh - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      const int bm = in_lds ? s_base[mid] : a.hbase[mid];
      if (bm <= ch)
        lo = mid;
      else
        hi = mid - 1;
    }
    const int base = in_lds ? s_base[lo] : a.hbase[lo];
    const int u = a.hfront[lo];
    const int d = a.out.len[u], o = a.out.off[u];
    const int e0 = (ch - base) * PUSH_CHUNK, e1 = min(d, e0 + PUSH_CHUNK);
    const XT xv = xcur[col_index(u, S, j)];
    for (int e = e0 + w * PP + pp; e < e1; e += NWAVES * PP) {
      const int v = a.out.adj[o + e];
      if (xv != (XT)0) atomic_add_f64(&a.ybuf[col_index(v, S, j)], (double)xv);
      if (j == 0) a.stamp[v] = st;
    }
  }
}

// Sparse epilogue over all nodes: a node stamped in this slot (by the push,
// the offset seed or the seed vector) holds y = ybuf; r += scale*y, the next
// pre-scaled vector is written, ybuf is cleared, and the node's frontier stamp
// is set.  The previous vector is cleared where the previous frontier stamp
// is found.  Publishes norms, signed sums, frontier out-edges and size.
template <typename XT, int S>
__global__ __launch_bounds__(BLOCK) void k_epi(SlotArgs a, int k, double scale, int first) {
  __shared__ BlockRed sh;
  Ctl *ctl = a.ctl;
  if (!slot_live(ctl, MODE_SPARSE, k)) return;
  const int nw = k & 1, old = nw ^ 1;
  XT *__restrict__ xnew = (XT *)a.x[nw];
  XT *__restrict__ xold = (XT *)a.x[old];
  const int32_t st = ctl->stamp;
  // each wavefront tests the stamps of 64 consecutive nodes with one load per
  // array, then its groups of S lanes (one lane per column) take the marked
  // nodes, P at a time
  constexpr int P = RWR_WAVE / S;
  const int lane = threadIdx.x % RWR_WAVE, j = lane % S, g = lane / S;
  const bool act = ctl->active[j] != 0;
  double nrm = 0.0, sm = 0.0;
  int64_t fe = 0, fn = 0;
  auto node = [&](int v, bool clear, bool work) {
    const int64_t kk = col_index(v, S, j);
    if (clear) xold[kk] = (XT)0;
    if (!work) return;
    const double y = a.ybuf[kk] * scale;
    a.ybuf[kk] = 0.0;
    const int d = a.out.len[v];
    if (act) {
      a.r[kk] += y;
      nrm += fabs(y);
      sm += y;
      xnew[kk] = d ? (XT)(y / (double)d) : (XT)0;
    } else {
      xnew[kk] = (XT)0;
    }
    if (j == 0) {
      a.fstamp[v] = st;
      fe += d;
      fn += 1;
    }
  };
  const int nwv = gridDim.x * (BLOCK / RWR_WAVE);
  for (int base = (blockIdx.x * (BLOCK / RWR_WAVE) + threadIdx.x / RWR_WAVE) * RWR_WAVE; base < a.n;
       base += nwv * RWR_WAVE) {
    const int ul = base + lane;
    const bool in = ul < a.n;
    const int32_t fs = in ? a.fstamp[ul] : 0, ts = in ? a.stamp[ul] : 0;
    const unsigned long long mc = __ballot(in && !first && fs == st - 1);  // the previous frontier
    const unsigned long long mw = __ballot(in && ts == st);                 // this slot's nodes
    if constexpr (P <= 8) {
      // few nodes per step: group g takes the g-th lowest marked node left
      unsigned long long m = mc | mw;
      while (m) {
        unsigned long long mm = m;
        for (int q = 0; q < g; ++q) mm &= mm - 1;
#pragma unroll
        for (int q = 0; q < P; ++q) m &= m - 1;
        if (!mm) continue;
        const int bit = __builtin_ctzll(mm);
        node(base + bit, (mc >> bit) & 1ull, (mw >> bit) & 1ull);
      }
    } else {
      // many: group g takes positions g, g + P, ...
#pragma unroll
      for (int c0 = 0; c0 < RWR_WAVE; c0 += P) {
        const int bit = c0 + g;
        const bool cl = (mc >> bit) & 1ull, wk = (mw >> bit) & 1ull;
        if (cl || wk) node(base + bit, cl, wk);
      }
    }
  }
  block_publish<S>(nrm, sm, fe, fn, a.part, a.part_i, blockIdx.x, sh);
}

// ------------------------------------------------------------------ dense
// gather of one in-neighbour: pre-scaled vector, or r/d_out for the residual
template <typename XT, int S, int KIND>
struct Gather {
  __device__ __forceinline__ static double get(const SlotArgs &a, const XT *__restrict__ x, int u, int j) {
    if constexpr (KIND == KIND_RESID) {
      return a.xres[col_index(u, S, j)];
    } else {
      return (double)x[col_index(u, S, j)];
    }
  }
};

// epilogue of one row: propagation (r += y, next pre-scaled vector) or the
// residual g = y - r (zero at the column's seed; the sum collects r)
template <typename XT, int S, int KIND>
__device__ __forceinline__ void pull_epilogue(const SlotArgs &a, XT *__restrict__ xnext, int v, int j, double y,
                                              bool act, double &nrm, double &sm) {
  const int64_t kk = col_index(v, S, j);
  if constexpr (KIND == KIND_RESID) {
    const double rv = a.r[kk];
    double g = y - rv;
    if (j >= a.n_seeds || (a.zero_seed_rows && a.seeds[j] == v)) g = 0.0;
    a.gbuf[kk] = g;
    nrm += fabs(g);
    sm += rv;
  } else {
    const int d = a.out.len[v];
    if (act) {
      a.r[kk] += y;
      nrm += fabs(y);
      sm += y;
      xnext[kk] = d ? (XT)(y / (double)d) : (XT)0;
    } else {
      xnext[kk] = (XT)0;
    }
  }
}

// One chunk of a heavy in-row, processed by the whole workgroup; its sum per
// column goes to heavy.part[item * S + j].  Each thread keeps four
// independent gathers in flight.
template <typename XT, int S, int KIND>
__device__ __forceinline__ void heavy_item(const SlotArgs &a, int item, const XT *__restrict__ xcur,
                                           double (*hred)[RWR_MAX_COLS]) {
  constexpr int PP = RWR_WAVE / S;
  constexpr int STRIDE = NWAVES * PP;
  const int lane = threadIdx.x % RWR_WAVE, w = threadIdx.x / RWR_WAVE;
  const int jj = lane % S, pp = lane / S;
  const int h = a.heavy.item_row[item], ck = a.heavy.item_chunk[item];
  const int v = a.heavy.rows[h];
  const int nch = a.heavy.nchunks[h];
  const int o = a.in.off[v], d = a.in.len[v];
  const int e0 = ck * a.heavy.chunk;
  const int e1 = (ck == nch - 1) ? d : min(d, e0 + a.heavy.chunk);
  const int32_t *__restrict__ adj = a.in.adj + o;
  double acc = 0.0;
  int e = e0 + w * PP + pp;
  auto get = [&](int u) -> double { return Gather<XT, S, KIND>::get(a, xcur, u, jj); };
  for (; e + 3 * STRIDE < e1; e += 4 * STRIDE) {
    const int u0 = adj[e], u1 = adj[e + STRIDE], u2 = adj[e + 2 * STRIDE], u3 = adj[e + 3 * STRIDE];
    const double g0 = get(u0);
    const double g1 = get(u1);
    const double g2 = get(u2);
    const double g3 = get(u3);
    acc += (g0 + g1) + (g2 + g3);
  }
  for (; e < e1; e += STRIDE) acc += get(adj[e]);
  acc = wave_xor_sum(acc, S, RWR_WAVE);
  if (lane < S) hred[w][lane] = acc;
  __syncthreads();
  if (threadIdx.x < S) {
    double s = 0.0;
    for (int ww = 0; ww < NWAVES; ++ww) s += hred[ww][threadIdx.x];
    a.heavy.part[(int64_t)item * S + threadIdx.x] = s;
  }
  __syncthreads();
}

// Dense sweep for S >= 2 columns: heavy-row chunks first, then light rows,
// G lanes per row (lane = column x edge slot), every workgroup looping.
template <typename XT, int S, int G, int KIND>
__global__ __launch_bounds__(BLOCK) void k_pull(SlotArgs a, int k) {
  __shared__ BlockRed sh;
  __shared__ double hred[NWAVES][RWR_MAX_COLS];
  Ctl *ctl = a.ctl;
  if (KIND == KIND_DENSE && !slot_live(ctl, MODE_DENSE, k)) return;
  const XT *__restrict__ xcur = (const XT *)a.x[(k - 1) & 1];
  XT *__restrict__ xnext = (XT *)a.x[k & 1];
  const double c1 = 1.0 - a.c;
  const int lane = threadIdx.x % RWR_WAVE;
  double nrm = 0.0, sm = 0.0;
  for (int item = blockIdx.x; item < a.heavy.n_items; item += gridDim.x) heavy_item<XT, S, KIND>(a, item, xcur, hred);
  constexpr int P = G / S;
  const int gl = lane % G, j = gl % S, p = gl / S;
  constexpr int GPB = BLOCK / G;
  const bool act = ctl->active[j] != 0;
  const int ngroups = gridDim.x * GPB;
  for (int v = blockIdx.x * GPB + threadIdx.x / G; v < a.n; v += ngroups) {
    if (a.in.heavy[v]) continue;
    const int o = a.in.off[v], d = a.in.len[v];
    double acc = 0.0;
    int e = p;
    for (; e + 3 * P < d; e += 4 * P) {
      const int u0 = a.in.adj[o + e], u1 = a.in.adj[o + e + P], u2 = a.in.adj[o + e + 2 * P],
                u3 = a.in.adj[o + e + 3 * P];
      const double g0 = Gather<XT, S, KIND>::get(a, xcur, u0, j);
      const double g1 = Gather<XT, S, KIND>::get(a, xcur, u1, j);
      const double g2 = Gather<XT, S, KIND>::get(a, xcur, u2, j);
      const double g3 = Gather<XT, S, KIND>::get(a, xcur, u3, j);
      acc += (g0 + g1) + (g2 + g3);
    }
    for (; e < d; e += P) acc += Gather<XT, S, KIND>::get(a, xcur, a.in.adj[o + e], j);
    for (int off = S; off < G; off <<= 1) acc += __shfl_xor(acc, off, RWR_WAVE);
    if (p == 0) pull_epilogue<XT, S, KIND>(a, xnext, v, j, c1 * acc, act, nrm, sm);
  }
  block_publish<S>(nrm, sm, 0, 0, a.part, a.part_i, blockIdx.x, sh);
}

// ------------------------------------------------ dense, S >= 4 columns
// Each lane moves 16 bytes of a gathered row: V consecutive columns (V = 4
// for FP32 vectors, 2 for FP64 vectors and for the residual's FP64 scores).
// L = S / V lanes cover one edge's row; a group of G lanes works on one
// in-row with P = G / L edge slots, each slot keeping four gathers in
// flight.  Same sums and epilogue as k_pull, in the same fixed order per
// column.
// Streamed operands (adjacency, scores, the next vector) are touched once
// per sweep: load and store them non-temporally so that the caches keep the
// gathered rows of the current vector.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int32_t nt_load(const int32_t *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ nt_d2 nt_load2(const double *p) {
  return __builtin_nontemporal_load(reinterpret_cast<const nt_d2 *>(p));
}
__device__ __forceinline__ void nt_store2(double *p, double a, double b) {
  nt_d2 v = {a, b};
  __builtin_nontemporal_store(v, reinterpret_cast<nt_d2 *>(p));
}
__device__ __forceinline__ void nt_store4(float *p, float a, float b, float c, float d) {
  nt_f4 v = {a, b, c, d};
  __builtin_nontemporal_store(v, reinterpret_cast<nt_f4 *>(p));
}

template <typename XT, int KIND>
struct VecGather {
  using GT = typename std::conditional<KIND == KIND_RESID, double, XT>::type;
  static constexpr int V = 16 / (int)sizeof(GT);
  using VT = typename std::conditional<sizeof(GT) == 4, float4, double2>::type;
};

// One 16-byte gather, kept in its storage type while it is in flight (the
// FP64 widening happens when it is added, so four gathers in flight hold 16
// registers, not 32).
template <typename XT, int S, int KIND>
__device__ __forceinline__ typename VecGather<XT, KIND>::VT gather_vec(const SlotArgs &a, const XT *__restrict__ x,
                                                                       int u, int j0) {
  using VT = typename VecGather<XT, KIND>::VT;
  if constexpr (KIND == KIND_RESID) {
    return *reinterpret_cast<const VT *>(a.xres + col_index(u, S, j0));
  } else {
    return *reinterpret_cast<const VT *>(x + col_index(u, S, j0));
  }
}

template <typename VT>
__device__ __forceinline__ VT vzero() {
  VT z;
  if constexpr (sizeof(z.x) == 4) {
    z = VT{0.f, 0.f, 0.f, 0.f};
  } else {
    z = VT{0.0, 0.0};
  }
  return z;
}

// acc[q] += (g0 + g1) + (g2 + g3) per column, in FP64
template <int V, typename VT>
__device__ __forceinline__ void vacc4(double (&acc)[V], const VT (&g)[4]) {
  acc[0] += ((double)g[0].x + (double)g[1].x) + ((double)g[2].x + (double)g[3].x);
  acc[1] += ((double)g[0].y + (double)g[1].y) + ((double)g[2].y + (double)g[3].y);
  if constexpr (V == 4) {
    acc[2] += ((double)g[0].z + (double)g[1].z) + ((double)g[2].z + (double)g[3].z);
    acc[3] += ((double)g[0].w + (double)g[1].w) + ((double)g[2].w + (double)g[3].w);
  }
}

// the row's scores, loaded when the row starts so that the load overlaps the
// gathers
template <int S, int V>
__device__ __forceinline__ void load_scores_vec(const SlotArgs &a, int v, int j0, double (&rv)[V]) {
  const int64_t kk = col_index(v, S, j0);
#pragma unroll
  for (int q = 0; q < V; q += 2) {
    const nt_d2 t = nt_load2(a.r + kk + q);
    rv[q] = t.x;
    rv[q + 1] = t.y;
  }
}

template <typename XT, int S, int KIND, int V>
__device__ __forceinline__ void pull_epilogue_vec(const SlotArgs &a, XT *__restrict__ xnext, int v, int j0,
                                                  const double (&y)[V], double (&rv)[V], const bool (&act)[V],
                                                  double (&nrm)[V], double (&sm)[V]) {
  const int64_t kk = col_index(v, S, j0);
  if constexpr (KIND == KIND_RESID) {
    double g[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
      g[q] = y[q] - rv[q];
      if (j0 + q >= a.n_seeds || (a.zero_seed_rows && a.seeds[j0 + q] == v)) g[q] = 0.0;
      nrm[q] += fabs(g[q]);
      sm[q] += rv[q];
    }
#pragma unroll
    for (int q = 0; q < V; q += 2) nt_store2(a.gbuf + kk + q, g[q], g[q + 1]);
  } else {
    const int d = a.out.len[v];
    XT xo[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
      if (act[q]) {
        rv[q] += y[q];
        nrm[q] += fabs(y[q]);
        sm[q] += y[q];
        xo[q] = d ? (XT)(y[q] / (double)d) : (XT)0;
      } else {
        xo[q] = (XT)0;
      }
    }
#pragma unroll
    for (int q = 0; q < V; q += 2) nt_store2(a.r + kk + q, rv[q], rv[q + 1]);
    if constexpr (V == 4) {
      nt_store4(xnext + kk, xo[0], xo[1], xo[2], xo[3]);
    } else {
      nt_store2(xnext + kk, xo[0], xo[1]);
    }
  }
}

// block_publish for lanes holding V columns each (lane l of a group of L
// holds columns l*V .. l*V+V-1)
template <int S, int V>
__device__ void block_publish_vec(double (&nrm)[V], double (&sm)[V], double *part, int64_t *part_i, int e,
                                  BlockRed &sh) {
  constexpr int L = S / V;
  const int lane = threadIdx.x % RWR_WAVE, w = threadIdx.x / RWR_WAVE;
#pragma unroll
  for (int q = 0; q < V; ++q) {
    nrm[q] = wave_xor_sum(nrm[q], L, RWR_WAVE);
    sm[q] = wave_xor_sum(sm[q], L, RWR_WAVE);
  }
  if (lane < L) {
#pragma unroll
    for (int q = 0; q < V; ++q) {
      sh.wn[w][lane * V + q] = nrm[q];
      sh.ws[w][lane * V + q] = sm[q];
    }
  }
  __syncthreads();
  if (threadIdx.x < S) {
    double x = 0.0, y = 0.0;
    for (int ww = 0; ww < NWAVES; ++ww) x += sh.wn[ww][threadIdx.x], y += sh.ws[ww][threadIdx.x];
    part[e * entry_stride<S>() + 2 * threadIdx.x] = x;
    part[e * entry_stride<S>() + 2 * threadIdx.x + 1] = y;
  }
  if (threadIdx.x == 0) {
    part_i[(int64_t)e * 16] = 0;
    part_i[(int64_t)e * 16 + 1] = 0;
  }
}

// One chunk of a heavy in-row for S >= 4: the workgroup's BLOCK / L edge
// slots each move 16 bytes per lane, four gathers in flight per slot; slot
// sums are added in a fixed order (shuffle tree in each wave, then the
// waves in index order).
template <typename XT, int S, int KIND>
__device__ __forceinline__ void heavy_item_vec(const SlotArgs &a, int item, const XT *__restrict__ xcur,
                                               double (*hred)[RWR_MAX_COLS]) {
  constexpr int V = VecGather<XT, KIND>::V;
  using VT = typename VecGather<XT, KIND>::VT;
  constexpr int L = S / V;
  constexpr int SLOTS = BLOCK / L;
  const int lane = threadIdx.x % RWR_WAVE, w = threadIdx.x / RWR_WAVE;
  const int slot = threadIdx.x / L, j0 = (threadIdx.x % L) * V;
  const int h = a.heavy.item_row[item], ck = a.heavy.item_chunk[item];
  const int v = a.heavy.rows[h];
  const int nch = a.heavy.nchunks[h];
  const int o = a.in.off[v], d = a.in.len[v];
  const int e0 = ck * a.heavy.chunk;
  const int e1 = (ck == nch - 1) ? d : min(d, e0 + a.heavy.chunk);
  const int32_t *__restrict__ adj = a.in.adj + o;
  double acc[V];
#pragma unroll
  for (int q = 0; q < V; ++q) acc[q] = 0.0;
  for (int e = e0 + slot; e < e1; e += 4 * SLOTS) {
    int uu[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) uu[t] = e + t * SLOTS < e1 ? nt_load(adj + e + t * SLOTS) : -1;
    VT g[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) g[t] = uu[t] >= 0 ? gather_vec<XT, S, KIND>(a, xcur, uu[t], j0) : vzero<VT>();
    vacc4<V>(acc, g);
  }
#pragma unroll
  for (int q = 0; q < V; ++q) acc[q] = wave_xor_sum(acc[q], L, RWR_WAVE);
  if (lane < L) {
#pragma unroll
    for (int q = 0; q < V; ++q) hred[w][j0 + q] = acc[q];
  }
  __syncthreads();
  if (threadIdx.x < S) {
    double t = 0.0;
    for (int ww = 0; ww < NWAVES; ++ww) t += hred[ww][threadIdx.x];
    a.heavy.part[(int64_t)item * S + threadIdx.x] = t;
  }
  __syncthreads();
}

template <typename XT, int S, int G, int KIND>
__global__ __launch_bounds__(BLOCK) void k_pull_v(SlotArgs a, int k) {
  constexpr int V = VecGather<XT, KIND>::V;
  using VT = typename VecGather<XT, KIND>::VT;
  constexpr int L = S / V;
  constexpr int P = G / L;
  static_assert(L >= 1 && G % L == 0 && G <= RWR_WAVE && P >= 1, "lane layout");
  __shared__ BlockRed sh;
  __shared__ double hred[NWAVES][RWR_MAX_COLS];
  Ctl *ctl = a.ctl;
  if (KIND == KIND_DENSE && !slot_live(ctl, MODE_DENSE, k)) return;
  const XT *__restrict__ xcur = (const XT *)a.x[(k - 1) & 1];
  XT *__restrict__ xnext = (XT *)a.x[k & 1];
  const double c1 = 1.0 - a.c;
  const int lane = threadIdx.x % RWR_WAVE;
  for (int item = blockIdx.x; item < a.heavy.n_items; item += gridDim.x)
    heavy_item_vec<XT, S, KIND>(a, item, xcur, hred);
  const int gl = lane % G, p = gl / L, j0 = (gl % L) * V;
  constexpr int GPB = BLOCK / G;
  bool act[V];
  double nrm[V], sm[V];
#pragma unroll
  for (int q = 0; q < V; ++q) {
    act[q] = ctl->active[j0 + q] != 0;
    nrm[q] = 0.0;
    sm[q] = 0.0;
  }
  const int ngroups = gridDim.x * GPB;
  for (int i = blockIdx.x * GPB + threadIdx.x / G; i < a.n_order; i += ngroups) {
    const int v = a.row_order[i];
    if (v >= a.n || a.in.heavy[v]) continue;
    const int o = a.in.off[v], d = a.in.len[v];
    const int32_t *__restrict__ adj = a.in.adj + o;
    double acc[V];
#pragma unroll
    for (int q = 0; q < V; ++q) acc[q] = 0.0;
    for (int e = p; e < d; e += 4 * P) {
      int uu[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) uu[t] = e + t * P < d ? nt_load(adj + e + t * P) : -1;
      VT g[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) g[t] = uu[t] >= 0 ? gather_vec<XT, S, KIND>(a, xcur, uu[t], j0) : vzero<VT>();
      vacc4<V>(acc, g);
    }
#pragma unroll
    for (int off = L; off < G; off <<= 1) {
#pragma unroll
      for (int q = 0; q < V; ++q) acc[q] += __shfl_xor(acc[q], off, RWR_WAVE);
    }
    if (p == 0) {
      double y[V], rv[V];
      load_scores_vec<S, V>(a, v, j0, rv);
#pragma unroll
      for (int q = 0; q < V; ++q) y[q] = c1 * acc[q];
      pull_epilogue_vec<XT, S, KIND, V>(a, xnext, v, j0, y, rv, act, nrm, sm);
    }
  }
  block_publish_vec<S, V>(nrm, sm, a.part, a.part_i, blockIdx.x, sh);
}

#define WV_PER_LANE 8                       // consecutive in-edges per lane in a round
#define WV_ROUND (WV_PER_LANE * RWR_WAVE)   // in-edges per round of a wave item
static_assert(WV_ROUND == WV_EDGES && WV_ROWS == RWR_WAVE, "wave item shape");

// Order LDS accesses between the lanes of one wavefront (LDS requests of a
// wavefront complete in issue order; the fences keep the compiler from
// moving accesses across this point).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS of one wavefront's light item: the row of each entry of the round,
// off - pref per row, and the finished row sums
struct alignas(16) WaveBuf {
  int16_t rmap[WV_ROUND];
  int32_t base[WV_ROWS];
  double rsum[WV_ROWS];
};

// Per-lane row data of one wave item (lane i holds row r0 + i)
struct WvRows {
  int r0, nr;    // first row, number of rows (uniform)
  int d, off;    // light in-degree (0 for a heavy row or no row), in-row offset
  int dout;      // out-degree
  bool light;    // the lane holds a row that is not heavy
  double rv;     // r of the row
};

template <int KIND>
__device__ __forceinline__ WvRows wv_rows(const SlotArgs &a, int b, int lane) {
  WvRows m;
  m.r0 = a.mp_rows[b];
  m.nr = max(0, min(a.mp_rows[b + 1], a.n) - m.r0);
  m.d = 0;
  m.off = 0;
  m.dout = 0;
  m.light = false;
  m.rv = 0.0;
  if (lane < m.nr) {
    const int v = m.r0 + lane;
    m.light = a.in.heavy[v] == 0;
    m.off = a.in.off[v];
    const int d = a.in.len[v];
    m.d = m.light ? d : 0;
    if constexpr (KIND != KIND_RESID) m.dout = a.out.len[v];
    m.rv = a.r[v];
  }
  return m;
}

// Dense sweep for one seed column at wavefront granularity: every wavefront
// takes its own work items, with no workgroup barrier between items, so the
// load chains (row data -> in-row indices -> gathers) of all resident
// wavefronts overlap.  Items, in index order:
//   heavy chunks: a range of at most heavy.chunk in-edges of one heavy row;
//     lanes take consecutive edges, WV_PER_LANE loads in flight each; the
//     chunk sum (fixed shuffle tree) goes to heavy.part[item];
//   light items: rows mp_rows[b] .. mp_rows[b+1] (at most WV_ROWS rows and
//     about WV_ROUND light in-edges), merge-path style.  The rows' in-edges
//     are numbered consecutively; in each round lane t takes WV_PER_LANE
//     consecutive entries.  The row of every entry comes from a row map
//     (each row marks its first entry in LDS, then a running maximum over
//     the lane's entries and across the wave), so all index loads and
//     gathers of a lane are independent.  Sums by row: runs inside the lane,
//     then a segmented scan of the lanes' last runs across the wave; the
//     lane holding a row's last entry stores the row total.  A row that
//     continues into the next round carries its partial sum.  The row data
//     of the wavefront's next item is loaded while the current one runs.
// Every sum runs in a fixed order (deterministic).  Nodes are numbered by
// descending out-degree, so the leading entries of the gathered vector are
// the most gathered ones: the workgroup copies the first CACHE entries into
// LDS once and reads them there (4096 FP32 entries serve about a third of
// the gathers of an R-MAT graph of a million nodes; 6144 are kept, which
// still allows five workgroups per CU).
template <typename XT, int KIND, int NWV, int CACHE>
__global__ __launch_bounds__(NWV * RWR_WAVE) void k_pull_wv(SlotArgs a, int k) {
  constexpr int BLOCKW = NWV * RWR_WAVE;
  using PT = typename std::conditional<sizeof(XT) == 4 && KIND == KIND_DENSE, float, double>::type;
  struct Red {
    double n[NWV], s[NWV];
  };
  __shared__ union {
    Red red;
    WaveBuf wb[NWV];
  } U;
  __shared__ XT xc[CACHE > 0 ? CACHE : 1];
  Ctl *ctl = a.ctl;
  if (KIND == KIND_DENSE && !slot_live(ctl, MODE_DENSE, k)) return;
  const XT *__restrict__ xcur = (const XT *)a.x[(k - 1) & 1];
  const int ncache = CACHE > 0 ? min(CACHE, a.n) : 0;
  if constexpr (CACHE > 0) {
    const XT *src = KIND == KIND_RESID ? (const XT *)a.xres : xcur;
    for (int i = threadIdx.x; i < ncache; i += BLOCKW) xc[i] = src[i];
    __syncthreads();
  }
  XT *__restrict__ xnext = (XT *)a.x[k & 1];
  const double c1 = 1.0 - a.c;
  const bool act = ctl->active[0] != 0;
  const int lane = threadIdx.x % RWR_WAVE, w = threadIdx.x / RWR_WAVE;
  auto get = [&](int u) -> PT {
    if (CACHE > 0 && u < ncache) return (PT)xc[u];
    return (PT)Gather<XT, 1, KIND>::get(a, xcur, u, 0);
  };
  double nrm = 0.0, sm = 0.0;
  const int nwaves = gridDim.x * NWV;
  const int nh = a.heavy.n_items;
  int it = blockIdx.x * NWV + w;
  // heavy-row chunks
  for (; it < nh; it += nwaves) {
    const int h = a.heavy.item_row[it], ck = a.heavy.item_chunk[it];
    const int v = a.heavy.rows[h], nch = a.heavy.nchunks[h];
    const int o = a.in.off[v], d = a.in.len[v];
    const int e0 = ck * a.heavy.chunk;
    const int e1 = (ck == nch - 1) ? d : min(d, e0 + a.heavy.chunk);
    const int32_t *__restrict__ adj = a.in.adj + o;
    double acc = 0.0;
    for (int e = e0 + lane; e < e1; e += WV_ROUND) {
      int uq[WV_PER_LANE];
#pragma unroll
      for (int q = 0; q < WV_PER_LANE; ++q) uq[q] = e + q * RWR_WAVE < e1 ? nt_load(adj + e + q * RWR_WAVE) : -1;
      PT gq[WV_PER_LANE];
#pragma unroll
      for (int q = 0; q < WV_PER_LANE; ++q) gq[q] = uq[q] < 0 ? (PT)0 : get(uq[q]);
      double s4[WV_PER_LANE / 2];
#pragma unroll
      for (int q = 0; q < WV_PER_LANE / 2; ++q) s4[q] = (double)gq[2 * q] + (double)gq[2 * q + 1];
#pragma unroll
      for (int q = 0; q < WV_PER_LANE / 4; ++q) acc += s4[2 * q] + s4[2 * q + 1];
    }
    acc = wave_xor_sum(acc, 1, RWR_WAVE);
    if (lane == 0) a.heavy.part[it] = acc;
  }
  // light items
  WaveBuf &B = U.wb[w];
  int b = it - nh;
  WvRows cur{};
  if (b < a.n_mp) cur = wv_rows<KIND>(a, b, lane);
  while (b < a.n_mp) {
    const int bn = b + nwaves;
    // exclusive scan of the row lengths: row t owns entries pref_t .. incl_t - 1
    int incl = cur.d;
    for (int s2 = 1; s2 < RWR_WAVE; s2 <<= 1) {
      const int y = __shfl_up(incl, s2, RWR_WAVE);
      if (lane >= s2) incl += y;
    }
    const int my_pref = incl - cur.d;
    const int total = __shfl(incl, RWR_WAVE - 1, RWR_WAVE);
    B.base[lane] = cur.off - my_pref;
    B.rsum[lane] = 0.0;
    WvRows nxt{};
    if (bn < a.n_mp) nxt = wv_rows<KIND>(a, bn, lane);
    int carry_row = -1;  // row of the previous round's last entry
    double carry = 0.0;  // its partial sum up to there
    for (int base0 = 0; base0 < total; base0 += WV_ROUND) {
      // row of every entry of the round: each row marks its first entry,
      // then a running maximum (lane-local over 8 entries, then the wave)
      int4 *rm4 = reinterpret_cast<int4 *>(B.rmap);
      rm4[lane] = make_int4(-1, -1, -1, -1);
      wave_lds_sync();
      if (cur.d > 0 && my_pref >= base0 && my_pref < base0 + WV_ROUND) B.rmap[my_pref - base0] = (int16_t)lane;
      wave_lds_sync();
      const int4 mk = rm4[lane];
      int r[WV_PER_LANE];
      r[0] = (int16_t)(mk.x & 0xffff);
      r[1] = (int16_t)(mk.x >> 16);
      r[2] = (int16_t)(mk.y & 0xffff);
      r[3] = (int16_t)(mk.y >> 16);
      r[4] = (int16_t)(mk.z & 0xffff);
      r[5] = (int16_t)(mk.z >> 16);
      r[6] = (int16_t)(mk.w & 0xffff);
      r[7] = (int16_t)(mk.w >> 16);
      if (lane == 0) r[0] = max(r[0], carry_row);  // the round may start inside a row
#pragma unroll
      for (int q = 1; q < WV_PER_LANE; ++q) r[q] = max(r[q], r[q - 1]);
      int mx = r[WV_PER_LANE - 1];
      for (int s2 = 1; s2 < RWR_WAVE; s2 <<= 1) {
        const int y = __shfl_up(mx, s2, RWR_WAVE);
        if (lane >= s2) mx = max(mx, y);
      }
      int before = __shfl_up(mx, 1, RWR_WAVE);
      if (lane == 0) before = -1;
      const int i0 = base0 + WV_PER_LANE * lane;
#pragma unroll
      for (int q = 0; q < WV_PER_LANE; ++q) r[q] = i0 + q < total ? max(r[q], before) : WV_ROWS;
      int uq[WV_PER_LANE];
#pragma unroll
      for (int q = 0; q < WV_PER_LANE; ++q) uq[q] = r[q] < WV_ROWS ? a.in.adj[B.base[r[q]] + i0 + q] : -1;
      PT gq[WV_PER_LANE];
#pragma unroll
      for (int q = 0; q < WV_PER_LANE; ++q) gq[q] = uq[q] < 0 ? (PT)0 : get(uq[q]);
      // sums by row: runs inside the lane, then a segmented scan of the
      // lanes' last runs across the wave (fixed order: left to right)
      double sq[WV_PER_LANE];
      sq[0] = (lane == 0 && r[0] == carry_row) ? carry + (double)gq[0] : (double)gq[0];
#pragma unroll
      for (int q = 1; q < WV_PER_LANE; ++q) sq[q] = r[q] == r[q - 1] ? sq[q - 1] + (double)gq[q] : (double)gq[q];
      const int last_prev = __shfl_up(r[WV_PER_LANE - 1], 1, RWR_WAVE);
      const bool cont = lane > 0 && last_prev == r[0];  // the first run continues the previous lane's last
      double v = sq[WV_PER_LANE - 1];
      int f = (!cont || r[0] != r[WV_PER_LANE - 1]) ? 1 : 0;
      for (int s2 = 1; s2 < RWR_WAVE; s2 <<= 1) {
        const double vu = __shfl_up(v, s2, RWR_WAVE);
        const int fu = __shfl_up(f, s2, RWR_WAVE);
        if (lane >= s2) {
          if (!f) v = vu + v;
          f |= fu;
        }
      }
      const double v_prev = __shfl_up(v, 1, RWR_WAVE);
      const double cin = cont ? v_prev : 0.0;
      // a run ends where the row's last entry is; its total goes to rsum
      const int end_last = __shfl(incl, r[WV_PER_LANE - 1] & (RWR_WAVE - 1), RWR_WAVE);
#pragma unroll
      for (int q = 0; q < WV_PER_LANE; ++q) {
        const bool ends = q < WV_PER_LANE - 1 ? r[q + 1] != r[q] : i0 + q + 1 == end_last;
        if (r[q] < WV_ROWS && ends) B.rsum[r[q]] = r[q] == r[0] ? cin + sq[q] : sq[q];
      }
      carry_row = __shfl(r[WV_PER_LANE - 1], RWR_WAVE - 1, RWR_WAVE);
      carry = __shfl(v, RWR_WAVE - 1, RWR_WAVE);
      wave_lds_sync();
    }
    const double acc = B.rsum[lane];
    if (cur.light) {
      const int v = cur.r0 + lane;
      const double y = c1 * acc;
      if constexpr (KIND == KIND_RESID) {
        double g = y - cur.rv;
        if (a.n_seeds < 1 || (a.zero_seed_rows && a.seeds[0] == v)) g = 0.0;
        a.gbuf[v] = g;
        nrm += fabs(g);
        sm += cur.rv;
      } else {
        if (act) {
          a.r[v] = cur.rv + y;
          nrm += fabs(y);
          sm += y;
          xnext[v] = cur.dout ? (XT)(y / (double)cur.dout) : (XT)0;
        } else {
          xnext[v] = (XT)0;
        }
      }
    }
    cur = nxt;
    b = bn;
  }
  // partial sums of the workgroup: shuffle tree per wave, waves in order
  nrm = wave_xor_sum(nrm, 1, RWR_WAVE);
  sm = wave_xor_sum(sm, 1, RWR_WAVE);
  __syncthreads();
  if (lane == 0) {
    U.red.n[w] = nrm;
    U.red.s[w] = sm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tn = 0.0, ts = 0.0;
    for (int ww = 0; ww < NWV; ++ww) tn += U.red.n[ww], ts += U.red.s[ww];
    a.part[blockIdx.x * entry_stride<1>()] = tn;
    a.part[blockIdx.x * entry_stride<1>() + 1] = ts;
    a.part_i[(int64_t)blockIdx.x * 16] = 0;
    a.part_i[(int64_t)blockIdx.x * 16 + 1] = 0;
  }
}

// Heavy rows after a dense sweep: the chunk sums of row h (items first[h] ..
// first[h]+nchunks[h]-1) are added in order and the row's epilogue runs.
// Publishes its norms as entries entry_base + blockIdx.x.
template <typename XT, int S, int KIND>
__global__ __launch_bounds__(BLOCK) void k_heavy_epi(SlotArgs a, int k, int entry_base) {
  __shared__ BlockRed sh;
  Ctl *ctl = a.ctl;
  if (KIND == KIND_DENSE && !slot_live(ctl, MODE_DENSE, k)) return;
  XT *__restrict__ xnext = (XT *)a.x[k & 1];
  const double c1 = 1.0 - a.c;
  const int j = threadIdx.x % S;
  constexpr int NPB = BLOCK / S;
  const bool act = ctl->active[j] != 0;
  double nrm = 0.0, sm = 0.0;
  for (int h = blockIdx.x * NPB + threadIdx.x / S; h < a.heavy.n_rows; h += gridDim.x * NPB) {
    const int f = a.heavy.first[h], nch = a.heavy.nchunks[h];
    double s = 0.0;
    for (int q = 0; q < nch; ++q) s += a.heavy.part[(int64_t)(f + q) * S + j];
    pull_epilogue<XT, S, KIND>(a, xnext, a.heavy.rows[h], j, c1 * s, act, nrm, sm);
  }
  block_publish<S>(nrm, sm, 0, 0, a.part, a.part_i, entry_base + blockIdx.x, sh);
}

// V values of T in one aligned access
template <typename T, int V>
struct alignas(sizeof(T) * V) VecT {
  T v[V];
};

// Carried vectors (one column per seed, FP64 in gbuf).  A pending vector p is
// part of r, and r - p has residual p in the graph before the batch (Section
// 3.1's expansion).  Two kinds: the last iterate x^(k) of a run that ended in
// the dense phase, left in x[last] pre-scaled by 1/d_out (it was added to r,
// and r - x^(k) has residual x^(k)); and the FP64 residual g of an earlier
// check, added to r when it is kept.
//
// Before an update: gbuf = d_out * x[last] for the columns in tail_mask (with
// the degrees before the batch), the pending vector for the columns in
// keep_mask, 0 elsewhere; both x buffers are cleared for the run.  Each
// thread takes V consecutive columns (16-byte accesses of x where S allows);
// S is a compile-time power of two, so the node and column of an element
// are a shift and a mask
template <typename XT, int S>
__global__ __launch_bounds__(BLOCK) void k_carry_prepare(SlotArgs a, int last, uint64_t tail_mask,
                                                         uint64_t keep_mask) {
  constexpr int V = S >= 4 && sizeof(XT) == 4 ? 4 : (S >= 2 ? 2 : 1);
  using XV = VecT<XT, V>;
  using DV = VecT<double, V>;
  XT *__restrict__ x0 = (XT *)a.x[0];
  XT *__restrict__ x1 = (XT *)a.x[1];
  const XT *__restrict__ xl = (last == 1) ? x1 : x0;
  const int64_t groups = (int64_t)a.n * (S / V);
  XV zx;
#pragma unroll
  for (int q = 0; q < V; ++q) zx.v[q] = (XT)0;
  for (int64_t t = blockIdx.x * (int64_t)BLOCK + threadIdx.x; t < groups; t += (int64_t)gridDim.x * BLOCK) {
    const int64_t i = t * V;
    const int v = (int)(i / S), j0 = (int)(i % S);
    const uint64_t tails = last >= 0 ? (tail_mask >> j0) & ((1ull << V) - 1) : 0ull;
    const uint64_t keeps = (keep_mask >> j0) & ((1ull << V) - 1);
    DV p;
    XV xv = zx;
    DV g;
#pragma unroll
    for (int q = 0; q < V; ++q) g.v[q] = 0.0;
    if (tails) xv = *reinterpret_cast<const XV *>(xl + i);
    if (keeps & ~tails) g = *reinterpret_cast<const DV *>(a.gbuf + i);
    const int d = tails ? a.out.len[v] : 0;
#pragma unroll
    for (int q = 0; q < V; ++q) {
      if ((tails >> q) & 1ull)
        p.v[q] = d ? (double)xv.v[q] * (double)d : 0.0;
      else if ((keeps >> q) & 1ull)
        p.v[q] = g.v[q];
      else
        p.v[q] = 0.0;
    }
    *reinterpret_cast<DV *>(a.gbuf + i) = p;
    *reinterpret_cast<XV *>(x0 + i) = zx;
    *reinterpret_cast<XV *>(x1 + i) = zx;
  }
}

// The pending vectors join the run at its first dense sweep (slot k): they are
// added to that sweep's input, x^(k-1) += p (pre-scaled by the new 1/d_out),
// so that every later iterate carries their propagation.  r already holds p.
// Columns that stopped before the dense phase keep theirs pending; ctl->inj
// records which columns took it.  A column that takes its vector leaves the
// pending set, and readers of gbuf skip such columns, so gbuf is only read.
template <typename XT, int S>
__global__ __launch_bounds__(BLOCK) void k_inject(SlotArgs a, int k, uint64_t mask) {
  Ctl *ctl = a.ctl;
  if (!slot_live(ctl, MODE_DENSE, k)) return;
  // V consecutive columns per thread, as in k_carry_prepare
  constexpr int V = S >= 4 && sizeof(XT) == 4 ? 4 : (S >= 2 ? 2 : 1);
  using XV = VecT<XT, V>;
  using DV = VecT<double, V>;
  XT *__restrict__ xin = (XT *)a.x[(k - 1) & 1];
  uint64_t take = 0;  // pending columns still propagating
  for (int j = 0; j < S; ++j)
    if (((mask >> j) & 1ull) && ctl->active[j] != 0) take |= 1ull << j;
  if (blockIdx.x == 0 && threadIdx.x < S) ctl->inj[threadIdx.x] = (int32_t)((take >> threadIdx.x) & 1ull);
  if (!take) return;
  const int64_t groups = (int64_t)a.n * (S / V);
  for (int64_t t = blockIdx.x * (int64_t)BLOCK + threadIdx.x; t < groups; t += (int64_t)gridDim.x * BLOCK) {
    const int64_t i = t * V;
    const int v = (int)(i / S), j0 = (int)(i % S);
    const uint64_t tk = (take >> j0) & ((1ull << V) - 1);
    if (!tk) continue;
    const int d = a.out.len[v];
    if (!d) continue;
    const DV g = *reinterpret_cast<const DV *>(a.gbuf + i);
    XV xv = *reinterpret_cast<const XV *>(xin + i);
#pragma unroll
    for (int q = 0; q < V; ++q)
      if (((tk >> q) & 1ull) && g.v[q] != 0.0) xv.v[q] = (XT)((double)xv.v[q] + g.v[q] / (double)d);
    *reinterpret_cast<XV *>(xin + i) = xv;
  }
}

// r += g for a residual that is kept as a pending vector (then sigma is
// recomputed exactly)
template <int S>
__global__ __launch_bounds__(BLOCK) void k_add_resid(SlotArgs a) {
  const int64_t total = (int64_t)a.n * S;
  for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < total; i += (int64_t)gridDim.x * BLOCK)
    if ((int)(i % S) < a.n_seeds) a.r[i] += a.gbuf[i];
}

// Restart term of seed vectors after a residual sweep: g += c q on every
// node, then the workgroup's partial sums of ||g||_1 and of r (they replace
// the sweep's own partials).  The seed-vector columns have no seed rows, so
// the sweep left g = P r - r everywhere.
template <int S>
__global__ __launch_bounds__(BLOCK) void k_resid_q(SlotArgs a) {
  __shared__ BlockRed sh;
  const int j = threadIdx.x % S;
  constexpr int NPB = BLOCK / S;
  double nrm = 0.0, sm = 0.0;
  for (int v = blockIdx.x * NPB + threadIdx.x / S; v < a.n; v += gridDim.x * NPB) {
    const int64_t kk = col_index(v, S, j);
    const double g = j < a.n_seeds ? a.gbuf[kk] + a.c * a.qvec[kk] : 0.0;
    a.gbuf[kk] = g;
    nrm += fabs(g);
    sm += a.r[kk];
  }
  block_publish<S>(nrm, sm, 0, 0, a.part, a.part_i, blockIdx.x, sh);
}

// input of the residual sweep: xres = r / d_out (0 for a node without
// out-edges), so that its gathers read one value per in-edge
template <int S>
__global__ __launch_bounds__(BLOCK) void k_prescale(SlotArgs a) {
  const int64_t total = (int64_t)a.n * S;
  for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < total; i += (int64_t)gridDim.x * BLOCK) {
    const int d = a.out.len[i / S];
    a.xres[i] = d ? a.r[i] / (double)d : 0.0;
  }
}

// ------------------------------------------------------------------ others
// x^(0) = residual g for the active columns: r += g, pre-scaled into x[0]
template <typename XT, int S>
__global__ __launch_bounds__(BLOCK) void k_refine_init(SlotArgs a) {
  __shared__ BlockRed sh;
  Ctl *ctl = a.ctl;
  XT *__restrict__ x0 = (XT *)a.x[0];
  const int j = threadIdx.x % S;
  constexpr int NPB = BLOCK / S;
  const bool act = ctl->active[j] != 0;
  double nrm = 0.0, sm = 0.0;
  for (int v = blockIdx.x * NPB + threadIdx.x / S; v < a.n; v += gridDim.x * NPB) {
    const int64_t kk = col_index(v, S, j);
    const int d = a.out.len[v];
    if (act) {
      const double g = a.gbuf[kk];
      a.r[kk] += g;
      nrm += fabs(g);
      sm += g;
      x0[kk] = d ? (XT)(g / (double)d) : (XT)0;
    } else {
      x0[kk] = (XT)0;
    }
  }
  block_publish<S>(nrm, sm, 0, 0, a.part, a.part_i, blockIdx.x, sh);
}

// exact column sums of r
template <int S>
__global__ __launch_bounds__(BLOCK) void k_sigma(SlotArgs a) {
  __shared__ BlockRed sh;
  const int j = threadIdx.x % S;
  constexpr int NPB = BLOCK / S;
  double sm = 0.0;
  for (int v = blockIdx.x * NPB + threadIdx.x / S; v < a.n; v += gridDim.x * NPB) sm += a.r[col_index(v, S, j)];
  block_publish<S>(0.0, sm, 0, 0, a.part, a.part_i, blockIdx.x, sh);
}

// x^(0) = c e_s per column (Section 2.2): seed the scatter buffer, stamp
template <int S>
__global__ void k_seed_init(SlotArgs a) {
  const int j = threadIdx.x;
  Ctl *ctl = a.ctl;
  const int32_t st = ctl->stamp;
  if (j < a.n_seeds) {
    const int v = a.seeds[j];
    a.ybuf[col_index(v, S, j)] = a.c;
    a.stamp[v] = st;
  }
}

// leave both x-buffers zero for the next propagation
template <typename XT, int S>
__global__ __launch_bounds__(BLOCK) void k_finish(SlotArgs a) {
  Ctl *ctl = a.ctl;
  if (ctl->ended_dense) {
    const int64_t total = (int64_t)a.n * S;
    XT *x0 = (XT *)a.x[0];
    XT *x1 = (XT *)a.x[1];
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < total; i += (int64_t)gridDim.x * BLOCK) {
      x0[i] = (XT)0;
      x1[i] = (XT)0;
    }
  } else {
    // the last epilogue stamped its frontier with ctl->stamp - 1
    const int last = max(ctl->iter - 1, 0) & 1;
    XT *x = (XT *)a.x[last];
    const int32_t fst = ctl->stamp - 1;
    const int j = threadIdx.x % S;
    constexpr int NPB = BLOCK / S;
    for (int v = blockIdx.x * NPB + threadIdx.x / S; v < a.n; v += gridDim.x * NPB)
      if (a.fstamp[v] == fst) x[col_index(v, S, j)] = (XT)0;
  }
}

__global__ void k_reset_run(Ctl *ctl, int32_t S, uint64_t active_mask, double eps, int32_t max_iters,
                            int64_t dense_thresh, int64_t dense_nodes, int32_t hist_base, int32_t lockstep) {
  const int t = threadIdx.x;
  if (t < RWR_MAX_COLS) {
    const int a = (t < S) && ((active_mask >> t) & 1ull);
    ctl->active[t] = a;
    ctl->last_norm[t] = 0.0;
    ctl->norm0[t] = 0.0;
    ctl->norm1[t] = 0.0;
    ctl->sum_norm[t] = 0.0;
    ctl->last_it[t] = 0;
    ctl->inj[t] = 0;
  }
  if (t == 0) {
    ctl->prop_err = 0;
    ctl->mode = MODE_SPARSE;
    ctl->iter = 0;
    ctl->max_iters = max_iters;
    ctl->n_active = __popcll(active_mask);
    ctl->ended_dense = 0;
    ctl->fcount[0] = 0;
    ctl->fcount[1] = 0;
    ctl->done_blocks = 0;
    ctl->dense_iters = 0;
    ctl->fedges = 0;
    ctl->visited = 0;
    ctl->dense_thresh = dense_thresh;
    ctl->dense_nodes = dense_nodes;
    ctl->eps = eps;
    ctl->hpack = 0;
    ctl->hist_base = hist_base;
    ctl->lockstep = lockstep;
  }
}

// scores in external id order: out[v] = r[perm[v], j] / sigma_j
__global__ void k_scores(const double *__restrict__ r, const Ctl *ctl, const int32_t *__restrict__ perm, int S, int j,
                         int32_t n, double *__restrict__ out) {
  const double inv = 1.0 / ctl->sigma[j];
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    out[v] = r[(int64_t)perm[v] * S + j] * inv;
}

// ------------------------------------------------------------------ launchers
template <int S>
static constexpr int push_lanes() {
  return S >= 16 ? 64 : 16;
}

void launch_reset_run(Ctl *ctl, int32_t S, uint64_t mask, double eps, int32_t max_iters, int64_t dense_thresh,
                      int64_t dense_nodes, hipStream_t st, int32_t hist_base, int32_t lockstep) {
  hipLaunchKernelGGL(k_reset_run, dim3(1), dim3(64), 0, st, ctl, S, mask, eps, max_iters, dense_thresh, dense_nodes,
                     hist_base, lockstep);
}

#define RWR_DISPATCH_S(S, CALL)  \
  switch (S) {                   \
    case 1: {                    \
      constexpr int SS = 1;      \
      CALL;                      \
    } break;                     \
    case 2: {                    \
      constexpr int SS = 2;      \
      CALL;                      \
    } break;                     \
    case 4: {                    \
      constexpr int SS = 4;      \
      CALL;                      \
    } break;                     \
    case 8: {                    \
      constexpr int SS = 8;      \
      CALL;                      \
    } break;                     \
    case 16: {                   \
      constexpr int SS = 16;     \
      CALL;                      \
    } break;                     \
    case 32: {                   \
      constexpr int SS = 32;     \
      CALL;                      \
    } break;                     \
    default: {                   \
      constexpr int SS = 64;     \
      CALL;                      \
    } break;                     \
  }

template <int S, typename XT = float>
static void decide_impl(const SlotArgs &a, int kind, int count, int new_list, hipStream_t st, int fold = 0) {
  // several workgroups once the entries are large (many columns): one
  // workgroup streams them at a fraction of the chip's rate, while the
  // arrival count and fences cost a few microseconds
  const int64_t bytes = (int64_t)count * std::max(16, 2 * S) * 8;
  const int nb = bytes >= (2 << 20) ? std::max(1, std::min(DECIDE_GRID, count / 128)) : 1;
  hipLaunchKernelGGL((k_decide<XT, S>), dim3(nb), dim3(DECIDE_BLOCK), 0, st, a, kind, count, new_list, fold);
}

void launch_seed_init(const SlotArgs &a, int S, hipStream_t st) {
  RWR_DISPATCH_S(S, hipLaunchKernelGGL(k_seed_init<SS>, dim3(1), dim3(64), 0, st, a));
}

// x^(0) = c q for seed vectors (Section 2.2 with a general restart vector)
template <int S>
__global__ __launch_bounds__(BLOCK) void k_seed_init_q(SlotArgs a) {
  const int32_t st = a.ctl->stamp;
  const int64_t total = (int64_t)a.n * S;
  for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < total; i += (int64_t)gridDim.x * BLOCK) {
    const double y = a.c * a.qvec[i];
    if (y != 0.0) {
      a.ybuf[i] = y;
      a.stamp[i / S] = st;
    }
  }
}

void launch_seed_init_q(const SlotArgs &a, int S, hipStream_t st) {
  RWR_DISPATCH_S(S, hipLaunchKernelGGL(k_seed_init_q<SS>, dim3(a.grid_light), dim3(BLOCK), 0, st, a));
}

void launch_inject(const SlotArgs &a, int S, bool fp64, int k, uint64_t mask, hipStream_t st) {
  if (fp64) {
    RWR_DISPATCH_S(S, hipLaunchKernelGGL((k_inject<double, SS>), dim3(a.grid_light), dim3(BLOCK), 0, st, a, k, mask));
  } else {
    RWR_DISPATCH_S(S, hipLaunchKernelGGL((k_inject<float, SS>), dim3(a.grid_light), dim3(BLOCK), 0, st, a, k, mask));
  }
}

void launch_add_resid(const SlotArgs &a, int S, hipStream_t st) {
  RWR_DISPATCH_S(S, hipLaunchKernelGGL(k_add_resid<SS>, dim3(a.grid_light), dim3(BLOCK), 0, st, a));
}

template <typename XT, int S>
static void slot0_impl(const SlotArgs &a, hipStream_t st) {
  hipLaunchKernelGGL((k_epi<XT, S>), dim3(a.grid_light), dim3(BLOCK), 0, st, a, 0, 1.0, 1);
  decide_impl<S>(a, KIND_SPARSE, a.grid_light, 0, st);
}

void launch_slot0_epilogue(const SlotArgs &a, int S, bool fp64, hipStream_t st) {
  if (fp64) {
    RWR_DISPATCH_S(S, (slot0_impl<double, SS>(a, st)));
  } else {
    RWR_DISPATCH_S(S, (slot0_impl<float, SS>(a, st)));
  }
}

void launch_carry_prepare(const SlotArgs &a, int S, bool fp64, int last, uint64_t tail_mask, uint64_t keep_mask,
                          hipStream_t st) {
  if (fp64) {
    RWR_DISPATCH_S(S, hipLaunchKernelGGL((k_carry_prepare<double, SS>), dim3(a.grid_light), dim3(BLOCK), 0, st, a,
                                         last, tail_mask, keep_mask));
  } else {
    RWR_DISPATCH_S(S, hipLaunchKernelGGL((k_carry_prepare<float, SS>), dim3(a.grid_light), dim3(BLOCK), 0, st, a,
                                         last, tail_mask, keep_mask));
  }
}

// dense sweep (or residual) + heavy rows + decision; the heavy-row kernel
// publishes after the sweep's entries
template <typename XT, int S, int KIND>
static void pull_impl(const SlotArgs &a, int k, hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                      bool decide = true) {
  int grid;
  if constexpr (KIND == KIND_RESID)
    hipLaunchKernelGGL(k_prescale<S>, dim3(a.grid_light), dim3(BLOCK), 0, st, a);
  if (ev0) (void)hipEventRecord(ev0, st);
  if constexpr (S == 1) {
    // cached leading entries: 16 KB of the FP32 vector, or of r / d_out
    constexpr int CW = (KIND == KIND_DENSE && sizeof(XT) == 4) ? 6144 : KIND == KIND_RESID ? 2048 : 0;
    grid = std::max(1, std::min((a.heavy.n_items + a.n_mp + NWAVES - 1) / NWAVES, a.grid_pull));
    hipLaunchKernelGGL((k_pull_wv<XT, KIND, NWAVES, CW>), dim3(grid), dim3(BLOCK), 0, st, a, k);
  } else if constexpr (S == 2) {
    grid = a.grid_pull;
    hipLaunchKernelGGL((k_pull<XT, S, 16, KIND>), dim3(grid), dim3(BLOCK), 0, st, a, k);
  } else {
    grid = a.grid_pull;
    // lanes per in-row: 16, 32 or 64, at least one edge's row
    constexpr int L = S / VecGather<XT, KIND>::V;
    const int g = std::max(a.pull_lanes, L);
    if (g <= 16 && L <= 16) {
      hipLaunchKernelGGL((k_pull_v<XT, S, (L <= 16 ? 16 : L), KIND>), dim3(grid), dim3(BLOCK), 0, st, a, k);
    } else if (g <= 32 && L <= 32) {
      hipLaunchKernelGGL((k_pull_v<XT, S, (L <= 32 ? 32 : L), KIND>), dim3(grid), dim3(BLOCK), 0, st, a, k);
    } else {
      hipLaunchKernelGGL((k_pull_v<XT, S, 64, KIND>), dim3(grid), dim3(BLOCK), 0, st, a, k);
    }
  }
  if (ev1) (void)hipEventRecord(ev1, st);
  if constexpr (KIND == KIND_RESID) {
    if (decide && a.qvec) {
      // seed vectors: heavy rows, then the restart term c q with the
      // residual's partial sums, then the decision over those partials
      if (a.heavy.n_rows > 0) {
        const int hg = std::max(1, std::min((a.heavy.n_rows * S + BLOCK - 1) / BLOCK, 256));
        hipLaunchKernelGGL((k_heavy_epi<XT, S, KIND>), dim3(hg), dim3(BLOCK), 0, st, a, k, grid);
      }
      hipLaunchKernelGGL(k_resid_q<S>, dim3(a.grid_light), dim3(BLOCK), 0, st, a);
      decide_impl<S, XT>(a, KIND, a.grid_light, k & 1, st, 0);
      return;
    }
  }
  // few heavy rows: the decision kernel finishes them (one launch less)
  const bool fold = decide && (int64_t)a.heavy.n_rows * S <= std::min(a.fold_max, 2 * DECIDE_BLOCK);
  int hgrid = 0;
  if (a.heavy.n_rows > 0 && !fold) {
    hgrid = std::max(1, std::min((a.heavy.n_rows * S + BLOCK - 1) / BLOCK, HEAVY_EPI_MAX_GRID));
    hipLaunchKernelGGL((k_heavy_epi<XT, S, KIND>), dim3(hgrid), dim3(BLOCK), 0, st, a, k, grid);
  }
  if (decide) decide_impl<S, XT>(a, KIND, grid + hgrid, k & 1, st, fold ? 1 : 0);
}

template <typename XT, int S>
static void sparse_slot_impl(const SlotArgs &a, int k, hipStream_t st) {
  hipLaunchKernelGGL((k_push<XT, S, push_lanes<S>()>), dim3(a.grid_sparse), dim3(BLOCK), 0, st, a, k);
  hipLaunchKernelGGL((k_push_heavy<XT, S>), dim3(a.grid_sparse), dim3(BLOCK), 0, st, a, k);
  hipLaunchKernelGGL((k_epi<XT, S>), dim3(a.grid_light), dim3(BLOCK), 0, st, a, k, 1.0 - a.c, 0);
  decide_impl<S>(a, KIND_SPARSE, a.grid_light, k & 1, st);
}

void launch_sparse_slot(const SlotArgs &a, int S, bool fp64, int k, hipStream_t st) {
  if (fp64) {
    RWR_DISPATCH_S(S, (sparse_slot_impl<double, SS>(a, k, st)));
  } else {
    RWR_DISPATCH_S(S, (sparse_slot_impl<float, SS>(a, k, st)));
  }
}

void launch_dense_slot(const SlotArgs &a, int S, bool fp64, int k, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (fp64) {
    RWR_DISPATCH_S(S, (pull_impl<double, SS, KIND_DENSE>(a, k, st, ev0, ev1)));
  } else {
    RWR_DISPATCH_S(S, (pull_impl<float, SS, KIND_DENSE>(a, k, st, ev0, ev1)));
  }
}

template <typename XT, int S>
static void finish_impl(const SlotArgs &a, hipStream_t st) {
  hipLaunchKernelGGL((k_finish<XT, S>), dim3(a.grid_light), dim3(BLOCK), 0, st, a);
}

void launch_finish(const SlotArgs &a, int S, bool fp64, hipStream_t st) {
  if (fp64) {
    RWR_DISPATCH_S(S, (finish_impl<double, SS>(a, st)));
  } else {
    RWR_DISPATCH_S(S, (finish_impl<float, SS>(a, st)));
  }
}

void launch_residual(const SlotArgs &a, int S, hipStream_t st) {
  RWR_DISPATCH_S(S, (pull_impl<double, SS, KIND_RESID>(a, 1, st)));
}

void launch_apply_p(const SlotArgs &a, int S, hipStream_t st) {
  RWR_DISPATCH_S(S, (pull_impl<double, SS, KIND_RESID>(a, 1, st, nullptr, nullptr, false)));
}

template <typename XT, int S>
static void refine_impl(const SlotArgs &a, hipStream_t st) {
  hipLaunchKernelGGL((k_refine_init<XT, S>), dim3(a.grid_light), dim3(BLOCK), 0, st, a);
  decide_impl<S>(a, KIND_REFINE, a.grid_light, 0, st);
}

void launch_refine_init(const SlotArgs &a, int S, bool fp64, hipStream_t st) {
  if (fp64) {
    RWR_DISPATCH_S(S, (refine_impl<double, SS>(a, st)));
  } else {
    RWR_DISPATCH_S(S, (refine_impl<float, SS>(a, st)));
  }
}

template <int S>
static void sigma_impl(const SlotArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_sigma<S>, dim3(a.grid_light), dim3(BLOCK), 0, st, a);
  decide_impl<S>(a, KIND_SIGMA, a.grid_light, 0, st);
}

void launch_sigma_exact(const SlotArgs &a, int S, hipStream_t st) { RWR_DISPATCH_S(S, (sigma_impl<SS>(a, st))); }

__global__ void k_set_scores(const double *__restrict__ in, const int32_t *__restrict__ perm, int S, int j, int32_t n,
                             double *__restrict__ r) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    r[(int64_t)perm[v] * S + j] = in[v];
}

void launch_set_scores(const double *in, const int32_t *perm, int S, int j, int32_t n, double *r, hipStream_t st) {
  const int grid = std::max(1, std::min((n + 255) / 256, 2048));
  hipLaunchKernelGGL(k_set_scores, dim3(grid), dim3(256), 0, st, in, perm, S, j, n, r);
}

void launch_scores(const double *r, const Ctl *ctl, const int32_t *perm, int S, int j, int32_t n, double *out,
                   hipStream_t st) {
  const int grid = std::max(1, std::min((n + 255) / 256, 2048));
  hipLaunchKernelGGL(k_scores, dim3(grid), dim3(256), 0, st, r, ctl, perm, S, j, n, out);
}
