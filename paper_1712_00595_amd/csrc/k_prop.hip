// Cumulative propagation of Section 2.2 / Algorithm 1 on the device:
//   x^(i) = (1-c) B~^T x^(i-1),  r += x^(i),  stop when ||x^(i)||_1 <= eps.
//
// Vectors are kept pre-scaled: the stored x-buffers hold xh(v) = x(v)/d_out(v)
// (0 for dead ends), so that (B~^T x)(v) = sum over in-neighbours u of xh(u)
// and a gather reads one value per edge.  Two phases, chosen per iteration:
//   sparse: push over the out-rows of the frontier (nodes with x != 0),
//           FP64 atomics into ybuf, then an epilogue over the new frontier;
//   dense : pull over the in-rows of every node, one group of lanes per row
//           (rows above the light limit are split into chunks, one workgroup
//           each, combined by the last arriving chunk).
// Every epilogue is fused: accumulate into r (FP64), L1 norm and signed sum
// per seed column, and the next pre-scaled vector.  The last workgroup of each
// iteration reduces the per-workgroup partials in a fixed order (two levels,
// deterministic) and decides the phase of the next iteration, so the host can
// enqueue many iteration slots without waiting; slots after convergence exit
// at once.
//
// Cross-workgroup handoff inside a kernel uses no memory fences: on this part
// an agent-scope fence writes back the (per-XCD) L2, which is far too costly
// per workgroup.  A workgroup publishes its partial sums with returning
// agent-scope atomics, waits for their results, and only then bumps the
// arrival counter; the last arriver reads the partials with agent-scope
// atomic loads.  Plain stores are read only by later kernels.
#include <math.h>

#include "rwr_common.h"
#include "rwr_kernels.h"

#define BLOCK 256
#define NWAVES (BLOCK / RWR_WAVE)
#define GROUP_BLOCKS 32

enum { KIND_SPARSE = 0, KIND_DENSE = 1, KIND_REFINE = 2, KIND_RESID = 3, KIND_SIGMA = 4 };

template <typename T>
__device__ __forceinline__ T load_agent(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ T xchg_agent(T *p, T v) {
  return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// forces the wait for a returning atomic before the next statement
template <typename T>
__device__ __forceinline__ void consume(T v) {
  asm volatile("" : : "v"(v));
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (RWR_WAVE - lane));
}

// Append `v` (for lanes with pred) to list/counter with one atomic per wave.
__device__ __forceinline__ void wave_append(bool pred, int32_t v, int32_t *list, int32_t *counter) {
  const uint64_t act = __ballot(1);
  const uint64_t m = __ballot(pred);
  if (m == 0ull) return;
  const int leader = __ffsll((unsigned long long)act) - 1;
  int base = 0;
  if (__lane_id() == leader) base = atomicAdd(counter, (int)__popcll(m));
  base = __shfl(base, leader, RWR_WAVE);
  if (pred) list[base + __popcll(m & lanemask_lt())] = v;
}

// ------------------------------------------------------------------ reduction
// Per-thread inputs: nrm/sm belong to column lane % S; ia/ib are counters.
// Two-level deterministic reduction over the grid.  Returns true in the one
// workgroup that arrives last; it then holds the totals in s_norm/s_sum/s_i.
struct RedShared {
  double wn[NWAVES][RWR_MAX_COLS];
  double ws[NWAVES][RWR_MAX_COLS];
  int64_t wi[NWAVES][2];
  double fn[BLOCK];
  double fs[BLOCK];
  int64_t fi[BLOCK][2];
  double s_norm[RWR_MAX_COLS];
  double s_sum[RWR_MAX_COLS];
  int64_t s_i[2];
  int last_group;
  int last;
};

template <int S>
__device__ void reduce_level(const double *__restrict__ src, const int64_t *__restrict__ src_i, int first, int count,
                             RedShared &sh) {
  // sums entries first..first+count-1 of src (layout [entry][S][2]) in order
  constexpr int TPC = BLOCK / S;
  const int t = threadIdx.x, j = t % S, q = t / S;
  double a = 0.0, b = 0.0;
  for (int e = first + q; e < first + count; e += TPC) {
    a += load_agent(&src[((int64_t)e * S + j) * 2]);
    b += load_agent(&src[((int64_t)e * S + j) * 2 + 1]);
  }
  sh.fn[t] = a;
  sh.fs[t] = b;
  int64_t ia = 0, ib = 0;
  for (int e = first + t; e < first + count; e += BLOCK) {
    ia += load_agent(&src_i[(int64_t)e * 2]);
    ib += load_agent(&src_i[(int64_t)e * 2 + 1]);
  }
  sh.fi[t][0] = ia;
  sh.fi[t][1] = ib;
  __syncthreads();
  if (t < S) {
    double A = 0.0, B = 0.0;
    for (int qq = 0; qq < TPC; ++qq) {
      A += sh.fn[qq * S + t];
      B += sh.fs[qq * S + t];
    }
    sh.s_norm[t] = A;
    sh.s_sum[t] = B;
  }
  if (t == 0) {
    int64_t A = 0, B = 0;
    for (int qq = 0; qq < BLOCK; ++qq) A += sh.fi[qq][0], B += sh.fi[qq][1];
    sh.s_i[0] = A;
    sh.s_i[1] = B;
  }
  __syncthreads();
}

template <int S>
__device__ bool grid_reduce(double nrm, double sm, int64_t ia, int64_t ib, double *part, int64_t *part_i,
                            int32_t *gcnt, Ctl *ctl, RedShared &sh) {
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
  // level 0 partial of this workgroup
  double *p0 = part;
  int64_t *p0i = part_i;
  const int nblk = gridDim.x;
  const int ngroups = (nblk + GROUP_BLOCKS - 1) / GROUP_BLOCKS;
  double *p1 = part + (size_t)nblk * S * 2;
  int64_t *p1i = part_i + (size_t)nblk * 2;
  if (threadIdx.x < S) {
    double a = 0.0, b = 0.0;
    for (int ww = 0; ww < NWAVES; ++ww) a += sh.wn[ww][threadIdx.x], b += sh.ws[ww][threadIdx.x];
    consume(xchg_agent(&p0[((int64_t)blockIdx.x * S + threadIdx.x) * 2], a));
    consume(xchg_agent(&p0[((int64_t)blockIdx.x * S + threadIdx.x) * 2 + 1], b));
  }
  if (threadIdx.x == 0) {
    int64_t a = 0, b = 0;
    for (int ww = 0; ww < NWAVES; ++ww) a += sh.wi[ww][0], b += sh.wi[ww][1];
    consume(xchg_agent(&p0i[blockIdx.x * 2], a));
    consume(xchg_agent(&p0i[blockIdx.x * 2 + 1], b));
  }
  __syncthreads();
  const int g = blockIdx.x / GROUP_BLOCKS;
  const int gfirst = g * GROUP_BLOCKS;
  const int gsize = min(GROUP_BLOCKS, nblk - gfirst);
  if (threadIdx.x == 0) sh.last_group = atomicAdd(&gcnt[g], 1) == gsize - 1;
  __syncthreads();
  if (!sh.last_group) return false;
  reduce_level<S>(p0, p0i, gfirst, gsize, sh);
  if (threadIdx.x < S) {
    consume(xchg_agent(&p1[((int64_t)g * S + threadIdx.x) * 2], sh.s_norm[threadIdx.x]));
    consume(xchg_agent(&p1[((int64_t)g * S + threadIdx.x) * 2 + 1], sh.s_sum[threadIdx.x]));
  }
  if (threadIdx.x == 0) {
    consume(xchg_agent(&p1i[g * 2], sh.s_i[0]));
    consume(xchg_agent(&p1i[g * 2 + 1], sh.s_i[1]));
    gcnt[g] = 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) sh.last = atomicAdd(&ctl->done_blocks, 1u) == (unsigned)(ngroups - 1);
  __syncthreads();
  if (!sh.last) return false;
  reduce_level<S>(p1, p1i, 0, ngroups, sh);
  return true;
}

// Run by the whole last workgroup.  Records ||x^(it)||_1, updates the running
// sums, retires converged columns (after at least one iteration) and picks the
// phase of the next slot.
template <int S>
__device__ void decide(Ctl *ctl, double *hist, RedShared &sh, int kind, int new_list) {
  __shared__ int s_active;
  const int t = threadIdx.x;
  if (t == 0) s_active = 0;
  __syncthreads();
  const int it = ctl->iter;
  if (t < S) {
    const double nr = sh.s_norm[t];
    const double su = sh.s_sum[t];
    const bool act = ctl->active[t] != 0;
    hist[(int64_t)it * S + t] = act ? nr : 0.0;
    if (act) {
      ctl->sigma[t] += su;
      ctl->last_norm[t] = nr;
      if (!isfinite(nr) || !isfinite(su)) ctl->prop_err = ERR_ENUMERIC;
      if (it >= 1 && nr <= ctl->eps)
        ctl->active[t] = 0;
      else
        atomicAdd(&s_active, 1);
    }
  }
  __syncthreads();
  if (t == 0) {
    const int na = s_active;
    ctl->n_active = na;
    ctl->iter = it + 1;
    if (kind == KIND_SPARSE) ctl->visited += sh.s_i[1];
    if (kind == KIND_DENSE) ctl->dense_iters += 1;
    if (kind == KIND_DENSE || kind == KIND_REFINE) ctl->ended_dense = 1;
    int mode = ctl->mode;
    if (ctl->prop_err != 0 || na == 0) {
      mode = MODE_DONE;
    } else if (it >= ctl->max_iters) {
      mode = MODE_DONE;
      ctl->prop_err = ERR_ENOCONV;
    } else if (kind == KIND_REFINE) {
      mode = MODE_DENSE;
    } else if (kind == KIND_SPARSE &&
               (sh.s_i[0] > ctl->dense_thresh || (int64_t)ctl->fcount[new_list] > ctl->dense_nodes)) {
      mode = MODE_DENSE;
    }
    ctl->fedges = sh.s_i[0];
    if (kind == KIND_SPARSE || kind == KIND_REFINE) ctl->fcount[new_list ^ 1] = 0;
    ctl->stamp = ctl->stamp + 1;
    ctl->hfcount = 0;
    ctl->mode = mode;
    ctl->done_blocks = 0;
  }
}

// ------------------------------------------------------------------ kernels
#define PUSH_LIGHT_MAX 128
#define PUSH_CHUNK 2048

// Sparse push, light part: G lanes per frontier node with at most
// PUSH_LIGHT_MAX out-edges; longer rows are listed for k_push_heavy.  Every
// edge adds xh(u) into ybuf[v] (non-returning FP64 atomics) and stamps v as
// a member of the next frontier (plain store; the epilogue scans the stamps).
template <typename XT, int S, int G>
__global__ __launch_bounds__(BLOCK) void k_push(SlotArgs a, int k) {
  Ctl *ctl = a.ctl;
  if (ctl->mode != MODE_SPARSE) return;
  const int cur = (k - 1) & 1;
  const XT *__restrict__ xcur = (const XT *)a.x[cur];
  const int32_t *__restrict__ fcur = a.front[cur];
  const int nf = ctl->fcount[cur];
  const int32_t st = ctl->stamp;
  constexpr int P = G / S;
  const int lane = threadIdx.x % RWR_WAVE, gl = lane % G, j = gl % S, p = gl / S;
  constexpr int GPB = BLOCK / G;
  const int ngroups = gridDim.x * GPB;
  int64_t vis = 0;
  for (int i = blockIdx.x * GPB + threadIdx.x / G; i < nf; i += ngroups) {
    const int u = fcur[i];
    const int d = a.out.len[u];
    if (d > PUSH_LIGHT_MAX) {
      wave_append(gl == 0, u, a.hfront, &ctl->hfcount);
      continue;
    }
    const XT xv = xcur[col_index(u, S, j)];
    const int o = a.out.off[u];
    if (gl == 0) vis += d;
    for (int e = p; e < d; e += P) {
      const int v = a.out.adj[o + e];
      if (xv != (XT)0) atomic_add_f64(&a.ybuf[col_index(v, S, j)], (double)xv);
      if (j == 0) a.stamp[v] = st;
    }
  }
  vis = wave_xor_sum(vis, 1, RWR_WAVE);
  if (lane == 0 && vis) atomicAdd((unsigned long long *)&ctl->visited, (unsigned long long)vis);
}

// Sparse push, long rows: every row listed by k_push is cut into chunks of
// PUSH_CHUNK edges, numbered consecutively over the list; workgroup b takes
// the chunks whose number is b modulo the grid size.
template <typename XT, int S>
__global__ __launch_bounds__(BLOCK) void k_push_heavy(SlotArgs a, int k) {
  Ctl *ctl = a.ctl;
  if (ctl->mode != MODE_SPARSE) return;
  const int nh = ctl->hfcount;
  if (nh == 0) return;
  const int cur = (k - 1) & 1;
  const XT *__restrict__ xcur = (const XT *)a.x[cur];
  const int32_t st = ctl->stamp;
  constexpr int PP = RWR_WAVE / S;
  const int lane = threadIdx.x % RWR_WAVE, w = threadIdx.x / RWR_WAVE;
  const int j = lane % S, pp = lane / S;
  const int G = gridDim.x;
  int64_t base = 0, vis = 0;
  for (int h = 0; h < nh; ++h) {
    const int u = a.hfront[h];
    const int d = a.out.len[u], o = a.out.off[u];
    const int nch = (d + PUSH_CHUNK - 1) / PUSH_CHUNK;
    const XT xv = xcur[col_index(u, S, j)];
    int first = (int)(((int64_t)blockIdx.x - base % G + G) % G);
    for (int ck = first; ck < nch; ck += G) {
      const int e0 = ck * PUSH_CHUNK, e1 = min(d, e0 + PUSH_CHUNK);
      if (threadIdx.x == 0) vis += e1 - e0;
      for (int e = e0 + w * PP + pp; e < e1; e += NWAVES * PP) {
        const int v = a.out.adj[o + e];
        if (xv != (XT)0) atomic_add_f64(&a.ybuf[col_index(v, S, j)], (double)xv);
        if (j == 0) a.stamp[v] = st;
      }
    }
    base += nch;
  }
  if (threadIdx.x == 0 && vis) atomicAdd((unsigned long long *)&ctl->visited, (unsigned long long)vis);
}

// Sparse epilogue: every node stamped in this slot (by the push, the offset
// seed or the seed vector) holds y = ybuf in this slot; r += scale*y, the next
// pre-scaled vector is written, ybuf is cleared, and the node joins frontier
// list k % 2.  The previous vector is cleared on its frontier list.
template <typename XT, int S>
__global__ __launch_bounds__(BLOCK) void k_epi(SlotArgs a, int k, double scale, int first) {
  __shared__ RedShared sh;
  Ctl *ctl = a.ctl;
  if (ctl->mode != MODE_SPARSE) return;
  const int nw = k & 1, old = nw ^ 1;
  XT *__restrict__ xnew = (XT *)a.x[nw];
  XT *__restrict__ xold = (XT *)a.x[old];
  const int32_t *__restrict__ fold = a.front[old];
  const int no = first ? 0 : ctl->fcount[old];
  const int32_t st = ctl->stamp;
  const int j = threadIdx.x % S;
  constexpr int NPB = BLOCK / S;
  const bool act = ctl->active[j] != 0;
  double nrm = 0.0, sm = 0.0;
  int64_t fe = 0;
  for (int v = blockIdx.x * NPB + threadIdx.x / S; v < a.n; v += gridDim.x * NPB) {
    if (a.stamp[v] != st) continue;
    const int64_t kk = col_index(v, S, j);
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
    if (j == 0) fe += d;
    wave_append(j == 0, v, a.front[nw], &ctl->fcount[nw]);
  }
  for (int i = blockIdx.x * NPB + threadIdx.x / S; i < no; i += gridDim.x * NPB)
    xold[col_index(fold[i], S, j)] = (XT)0;
  if (grid_reduce<S>(nrm, sm, fe, 0, a.part, a.part_i, a.gcnt, ctl, sh)) decide<S>(ctl, a.hist, sh, KIND_SPARSE, nw);
}

// gather of one in-neighbour: pre-scaled vector, or r/d_out for the residual
template <typename XT, int S, int KIND>
struct Gather {
  __device__ __forceinline__ static double get(const SlotArgs &a, const XT *__restrict__ x, int u, int j) {
    if constexpr (KIND == KIND_RESID) {
      return a.r[col_index(u, S, j)] / (double)a.out.len[u];
    } else {
      return (double)x[col_index(u, S, j)];
    }
  }
};

template <typename XT, int S, int KIND>
__device__ __forceinline__ void pull_epilogue(const SlotArgs &a, XT *__restrict__ xnext, int v, int j, double y,
                                              bool act, double &nrm, double &sm) {
  const int64_t kk = col_index(v, S, j);
  if constexpr (KIND == KIND_RESID) {
    const double rv = a.r[kk];
    double g = y - rv;
    if (j >= a.n_seeds || a.seeds[j] == v) g = 0.0;
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

template <int S, int KIND>
__device__ __forceinline__ void pull_finish(const SlotArgs &a, int k, double nrm, double sm, RedShared &sh) {
  Ctl *ctl = a.ctl;
  if (grid_reduce<S>(nrm, sm, 0, 0, a.part, a.part_i, a.gcnt, ctl, sh)) {
    if constexpr (KIND == KIND_DENSE) {
      decide<S>(ctl, a.hist, sh, KIND_DENSE, k & 1);
    } else {
      if (threadIdx.x < S) {
        ctl->red_norm[threadIdx.x] = sh.s_norm[threadIdx.x];
        ctl->red_sum[threadIdx.x] = sh.s_sum[threadIdx.x];
        ctl->sigma[threadIdx.x] = sh.s_sum[threadIdx.x];
      }
      if (threadIdx.x == 0) ctl->done_blocks = 0;
    }
  }
}

// One chunk of a heavy in-row, processed by the whole workgroup; the last
// arriving chunk of the row runs the epilogue.  Each thread keeps four
// independent gathers in flight.
template <typename XT, int S, int KIND>
__device__ __forceinline__ void heavy_item(const SlotArgs &a, const XT *__restrict__ xcur, XT *__restrict__ xnext,
                                           double c1, double &nrm, double &sm, double (*hred)[RWR_MAX_COLS],
                                           int *hlast) {
  constexpr int PP = RWR_WAVE / S;
  constexpr int STRIDE = NWAVES * PP;
  const int lane = threadIdx.x % RWR_WAVE, w = threadIdx.x / RWR_WAVE;
  const int jj = lane % S, pp = lane / S;
  const int item = blockIdx.x;
  const int h = a.heavy.item_row[item], ck = a.heavy.item_chunk[item];
  const int v = a.heavy.rows[h];
  const int nch = a.heavy.nchunks[h];
  const int o = a.in.off[v], d = a.in.len[v];
  const int e0 = ck * a.heavy.chunk;
  const int e1 = (ck == nch - 1) ? d : min(d, e0 + a.heavy.chunk);
  const int32_t *__restrict__ adj = a.in.adj + o;
  double acc = 0.0;
  int e = e0 + w * PP + pp;
  for (; e + 3 * STRIDE < e1; e += 4 * STRIDE) {
    const int u0 = adj[e], u1 = adj[e + STRIDE], u2 = adj[e + 2 * STRIDE], u3 = adj[e + 3 * STRIDE];
    const double g0 = Gather<XT, S, KIND>::get(a, xcur, u0, jj);
    const double g1 = Gather<XT, S, KIND>::get(a, xcur, u1, jj);
    const double g2 = Gather<XT, S, KIND>::get(a, xcur, u2, jj);
    const double g3 = Gather<XT, S, KIND>::get(a, xcur, u3, jj);
    acc += (g0 + g1) + (g2 + g3);
  }
  for (; e < e1; e += STRIDE) acc += Gather<XT, S, KIND>::get(a, xcur, adj[e], jj);
  acc = wave_xor_sum(acc, S, RWR_WAVE);
  if (lane < S) hred[w][lane] = acc;
  __syncthreads();
  if (threadIdx.x < S) {
    double s = 0.0;
    for (int ww = 0; ww < NWAVES; ++ww) s += hred[ww][threadIdx.x];
    consume(atomic_add_f64_ret(&a.heavy.acc[(int64_t)h * S + threadIdx.x], s));
  }
  __syncthreads();
  if (threadIdx.x == 0) *hlast = atomicAdd(&a.heavy.cnt[h], 1) == nch - 1;
  __syncthreads();
  if (*hlast) {
    if (threadIdx.x < S) {
      const int t = threadIdx.x;
      const double tot = load_agent(&a.heavy.acc[(int64_t)h * S + t]);
      a.heavy.acc[(int64_t)h * S + t] = 0.0;
      const bool act = a.ctl->active[t] != 0;
      pull_epilogue<XT, S, KIND>(a, xnext, v, t, c1 * tot, act, nrm, sm);
    }
    if (threadIdx.x == 0) a.heavy.cnt[h] = 0;
  }
}

template <typename XT, int S, int G, int KIND>
__global__ __launch_bounds__(BLOCK) void k_pull(SlotArgs a, int k) {
  __shared__ RedShared sh;
  __shared__ double hred[NWAVES][RWR_MAX_COLS];
  __shared__ int hlast;
  Ctl *ctl = a.ctl;
  if (KIND == KIND_DENSE && ctl->mode != MODE_DENSE) return;
  const XT *__restrict__ xcur = (const XT *)a.x[(k - 1) & 1];
  XT *__restrict__ xnext = (XT *)a.x[k & 1];
  const double c1 = 1.0 - a.c;
  const int lane = threadIdx.x % RWR_WAVE;
  double nrm = 0.0, sm = 0.0;
  if ((int)blockIdx.x < a.heavy.n_items) {
    heavy_item<XT, S, KIND>(a, xcur, xnext, c1, nrm, sm, hred, &hlast);
  } else {
    // light rows: G lanes per row, P = G/S edges in flight per row
    constexpr int P = G / S;
    const int gl = lane % G, j = gl % S, p = gl / S;
    constexpr int GPB = BLOCK / G;
    const bool act = ctl->active[j] != 0;
    const int lb = blockIdx.x - a.heavy.n_items;
    const int nlb = gridDim.x - a.heavy.n_items;
    const int ngroups = nlb * GPB;
    for (int v = lb * GPB + threadIdx.x / G; v < a.n; v += ngroups) {
      if (a.in.heavy[v]) continue;
      const int o = a.in.off[v], d = a.in.len[v];
      double acc;
      if constexpr (KIND == KIND_RESID || sizeof(XT) == 8) {
        acc = 0.0;
        for (int e = p; e < d; e += P) acc += Gather<XT, S, KIND>::get(a, xcur, a.in.adj[o + e], j);
      } else {
        float f = 0.0f;
        for (int e = p; e < d; e += P) f += xcur[col_index(a.in.adj[o + e], S, j)];
        acc = (double)f;
      }
      for (int off = S; off < G; off <<= 1) acc += __shfl_xor(acc, off, RWR_WAVE);
      if (p == 0) pull_epilogue<XT, S, KIND>(a, xnext, v, j, c1 * acc, act, nrm, sm);
    }
  }
  pull_finish<S, KIND>(a, k, nrm, sm, sh);
}

#define MP_ROWS 256
#define MP_ROUND (4 * BLOCK)

// Dense sweep for one seed column, merge-path style.  Workgroup b owns the
// rows mp_rows[b] .. mp_rows[b+1] (at most MP_ROWS rows and about MP_EDGES
// light in-edges, heavy rows excluded).  The rows' in-edges are numbered
// consecutively; in each round every thread fetches four of them (four
// independent index loads and gathers), the products go to LDS, and each
// row's owner thread adds its segment in index order (deterministic).
template <typename XT, int KIND>
__global__ __launch_bounds__(BLOCK) void k_pull_mp(SlotArgs a, int k) {
  struct MpShared {
    int32_t pref[MP_ROWS + 1];
    int32_t off[MP_ROWS];
    int32_t wsum[NWAVES];
    double prod[MP_ROUND];
  };
  __shared__ union {
    RedShared red;
    MpShared mp;
  } U;
  __shared__ double hred[NWAVES][RWR_MAX_COLS];
  __shared__ int hlast;
  Ctl *ctl = a.ctl;
  if (KIND == KIND_DENSE && ctl->mode != MODE_DENSE) return;
  const XT *__restrict__ xcur = (const XT *)a.x[(k - 1) & 1];
  XT *__restrict__ xnext = (XT *)a.x[k & 1];
  const double c1 = 1.0 - a.c;
  double nrm = 0.0, sm = 0.0;
  if ((int)blockIdx.x < a.heavy.n_items) {
    heavy_item<XT, 1, KIND>(a, xcur, xnext, c1, nrm, sm, hred, &hlast);
  } else {
    MpShared &M = U.mp;
    const int b = blockIdx.x - a.heavy.n_items;
    const int r0 = a.mp_rows[b];
    const int r1 = min(a.mp_rows[b + 1], a.n);
    const int nr = max(0, r1 - r0);
    const int t = threadIdx.x;
    const int lane = t % RWR_WAVE, w = t / RWR_WAVE;
    int d = 0;
    bool heavy = false;
    if (t < nr) {
      const int v = r0 + t;
      heavy = a.in.heavy[v] != 0;
      d = heavy ? 0 : a.in.len[v];
      M.off[t] = a.in.off[v];
    }
    // exclusive scan of the row lengths
    int incl = d;
    for (int s2 = 1; s2 < RWR_WAVE; s2 <<= 1) {
      const int y = __shfl_up(incl, s2, RWR_WAVE);
      if (lane >= s2) incl += y;
    }
    if (lane == RWR_WAVE - 1) M.wsum[w] = incl;
    __syncthreads();
    int wb = 0;
    for (int ww = 0; ww < w; ++ww) wb += M.wsum[ww];
    M.pref[t] = wb + incl - d;
    if (t == BLOCK - 1) M.pref[BLOCK] = wb + incl;
    __syncthreads();
    const int total = M.pref[nr];
    double acc = 0.0;
    for (int base = 0; base < total; base += MP_ROUND) {
      int uq[4];
      bool okq[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = base + q * BLOCK + t;
        okq[q] = i < total;
        uq[q] = 0;
        if (okq[q]) {
          int lo = 0, hi = nr - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (M.pref[mid] <= i)
              lo = mid;
            else
              hi = mid - 1;
          }
          uq[q] = a.in.adj[M.off[lo] + (i - M.pref[lo])];
        }
      }
      double gq[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) gq[q] = okq[q] ? Gather<XT, 1, KIND>::get(a, xcur, uq[q], 0) : 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) M.prod[q * BLOCK + t] = gq[q];
      __syncthreads();
      if (t < nr) {
        const int lo = max(M.pref[t], base) - base;
        const int hi = min(M.pref[t + 1], base + MP_ROUND) - base;
        for (int kk = lo; kk < hi; ++kk) acc += M.prod[kk];
      }
      __syncthreads();
    }
    if (t < nr && !heavy) {
      const bool act = ctl->active[0] != 0;
      pull_epilogue<XT, 1, KIND>(a, xnext, r0 + t, 0, c1 * acc, act, nrm, sm);
    }
    __syncthreads();
  }
  pull_finish<1, KIND>(a, k, nrm, sm, U.red);
}

// x^(0) = residual g for the active columns: r += g, pre-scaled into x[0]
template <typename XT, int S>
__global__ __launch_bounds__(BLOCK) void k_refine_init(SlotArgs a) {
  __shared__ RedShared sh;
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
  if (grid_reduce<S>(nrm, sm, 0, 0, a.part, a.part_i, a.gcnt, ctl, sh)) decide<S>(ctl, a.hist, sh, KIND_REFINE, 0);
}

// exact column sums of r
template <int S>
__global__ __launch_bounds__(BLOCK) void k_sigma(SlotArgs a) {
  __shared__ RedShared sh;
  const int j = threadIdx.x % S;
  constexpr int NPB = BLOCK / S;
  double sm = 0.0;
  for (int v = blockIdx.x * NPB + threadIdx.x / S; v < a.n; v += gridDim.x * NPB) sm += a.r[col_index(v, S, j)];
  if (grid_reduce<S>(0.0, sm, 0, 0, a.part, a.part_i, a.gcnt, a.ctl, sh)) {
    if (threadIdx.x < S) a.ctl->sigma[threadIdx.x] = sh.s_sum[threadIdx.x];
    if (threadIdx.x == 0) a.ctl->done_blocks = 0;
  }
}

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
    const int last = max(ctl->iter - 1, 0) & 1;
    XT *x = (XT *)a.x[last];
    const int32_t *f = a.front[last];
    const int cnt = ctl->fcount[last];
    const int j = threadIdx.x % S;
    constexpr int NPB = BLOCK / S;
    for (int i = blockIdx.x * NPB + threadIdx.x / S; i < cnt; i += gridDim.x * NPB) x[col_index(f[i], S, j)] = (XT)0;
  }
}

__global__ void k_reset_run(Ctl *ctl, int32_t S, uint64_t active_mask, double eps, int32_t max_iters,
                            int64_t dense_thresh, int64_t dense_nodes) {
  const int t = threadIdx.x;
  if (t < RWR_MAX_COLS) {
    const int a = (t < S) && ((active_mask >> t) & 1ull);
    ctl->active[t] = a;
    ctl->last_norm[t] = 0.0;
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
    ctl->hfcount = 0;
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
                           int64_t dense_nodes, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_run, dim3(1), dim3(64), 0, st, ctl, S, mask, eps, max_iters, dense_thresh, dense_nodes);
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

void launch_seed_init(const SlotArgs &a, int S, hipStream_t st) {
  RWR_DISPATCH_S(S, hipLaunchKernelGGL(k_seed_init<SS>, dim3(1), dim3(64), 0, st, a));
}

template <typename XT, int S>
static void slot0_impl(const SlotArgs &a, hipStream_t st) {
  hipLaunchKernelGGL((k_epi<XT, S>), dim3(a.grid_light), dim3(BLOCK), 0, st, a, 0, 1.0, 1);
}

void launch_slot0_epilogue(const SlotArgs &a, int S, bool fp64, hipStream_t st) {
  if (fp64) {
    RWR_DISPATCH_S(S, (slot0_impl<double, SS>(a, st)));
  } else {
    RWR_DISPATCH_S(S, (slot0_impl<float, SS>(a, st)));
  }
}

template <typename XT, int S, int KIND>
static void pull_impl(const SlotArgs &a, int k, hipStream_t st) {
  if constexpr (S == 1) {
    const int grid = a.heavy.n_items + a.n_mp;
    hipLaunchKernelGGL((k_pull_mp<XT, KIND>), dim3(grid), dim3(BLOCK), 0, st, a, k);
  } else {
    const int grid = a.heavy.n_items + a.grid_light;
    constexpr int G = S >= 8 ? 64 : 8 * S;
    hipLaunchKernelGGL((k_pull<XT, S, G, KIND>), dim3(grid), dim3(BLOCK), 0, st, a, k);
  }
}

template <typename XT, int S>
static void sparse_slot_impl(const SlotArgs &a, int k, hipStream_t st) {
  hipLaunchKernelGGL((k_push<XT, S, push_lanes<S>()>), dim3(a.grid_sparse), dim3(BLOCK), 0, st, a, k);
  hipLaunchKernelGGL((k_push_heavy<XT, S>), dim3(a.grid_sparse), dim3(BLOCK), 0, st, a, k);
  hipLaunchKernelGGL((k_epi<XT, S>), dim3(a.grid_light), dim3(BLOCK), 0, st, a, k, 1.0 - a.c, 0);
}

void launch_sparse_slot(const SlotArgs &a, int S, bool fp64, int k, hipStream_t st) {
  if (fp64) {
    RWR_DISPATCH_S(S, (sparse_slot_impl<double, SS>(a, k, st)));
  } else {
    RWR_DISPATCH_S(S, (sparse_slot_impl<float, SS>(a, k, st)));
  }
}

void launch_dense_slot(const SlotArgs &a, int S, bool fp64, int k, hipStream_t st) {
  if (fp64) {
    RWR_DISPATCH_S(S, (pull_impl<double, SS, KIND_DENSE>(a, k, st)));
  } else {
    RWR_DISPATCH_S(S, (pull_impl<float, SS, KIND_DENSE>(a, k, st)));
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

template <typename XT, int S>
static void refine_impl(const SlotArgs &a, hipStream_t st) {
  hipLaunchKernelGGL((k_refine_init<XT, S>), dim3(a.grid_light), dim3(BLOCK), 0, st, a);
}

void launch_refine_init(const SlotArgs &a, int S, bool fp64, hipStream_t st) {
  if (fp64) {
    RWR_DISPATCH_S(S, (refine_impl<double, SS>(a, st)));
  } else {
    RWR_DISPATCH_S(S, (refine_impl<float, SS>(a, st)));
  }
}

void launch_sigma_exact(const SlotArgs &a, int S, hipStream_t st) {
  RWR_DISPATCH_S(S, hipLaunchKernelGGL(k_sigma<SS>, dim3(a.grid_light), dim3(BLOCK), 0, st, a));
}

void launch_scores(const double *r, const Ctl *ctl, const int32_t *perm, int S, int j, int32_t n, double *out,
                   hipStream_t st) {
  const int grid = std::max(1, std::min((n + 255) / 256, 2048));
  hipLaunchKernelGGL(k_scores, dim3(grid), dim3(256), 0, st, r, ctl, perm, S, j, n, out);
}
