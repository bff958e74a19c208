// Device-side application of one update batch to the slack CSR/CSC graph,
// and the offset seed of Section 3.1:
//   q_offset = (1-c) (B~^T - A~^T) r_old,
// which is non-zero only on the neighbours of the rows of A~ that the batch
// changes (the non-zero rows of Delta A, Section 3.3).  For a changed row u
// with old degree d_o and new degree d_n (1/0 read as 0, Section 3.4.2):
//   neighbour kept      : (1-c) r(u) (1/d_n - 1/d_o)
//   neighbour inserted  : (1-c) r(u) / d_n
//   neighbour deleted   : -(1-c) r(u) / d_o
//
// Batch entries are packed into 64-bit keys
//   key = (row << (B+1)) | (col << 1) | is_insert,   B = bits of the largest id,
// one key array per orientation (out: row = source; in: row = destination).
// Sorting a key array groups a row's entries, ordered by column, so each
// touched row owns one segment that a wavefront can binary-search.
#include <hipcub/hipcub.hpp>

#include "rwr_common.h"
#include "rwr_kernels.h"

static constexpr uint64_t KEY_PAD = ~0ull;

__device__ __forceinline__ int32_t key_row(uint64_t k, int b1) { return (int32_t)(k >> b1); }
__device__ __forceinline__ int32_t key_col(uint64_t k, int b1) {
  return (int32_t)((k >> 1) & ((1ull << (b1 - 1)) - 1));
}

// ---------------------------------------------------------------- keys
__global__ void k_make_keys(const int32_t *__restrict__ ins_s, const int32_t *__restrict__ ins_d, int64_t n_ins,
                            const int32_t *__restrict__ del_s, const int32_t *__restrict__ del_d, int64_t n_del,
                            int32_t n_nodes, int b1, int undirected, const int32_t *__restrict__ perm,
                            const int32_t *__restrict__ mark, uint64_t *__restrict__ k_out,
                            uint64_t *__restrict__ k_in, Ctl *ctl) {
  const int64_t total = n_ins + n_del;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const bool ins = i < n_ins;
    const int32_t ue = ins ? ins_s[i] : del_s[i - n_ins];
    const int32_t ve = ins ? ins_d[i] : del_d[i - n_ins];
    const uint64_t t = ins ? 1ull : 0ull;
    if (ue < 0 || ue >= n_nodes || ve < 0 || ve >= n_nodes) {
      set_error(ctl, ERR_EINVAL);
      if (undirected) {
        k_out[2 * i] = KEY_PAD;
        k_out[2 * i + 1] = KEY_PAD;
      } else {
        k_out[i] = KEY_PAD;
        k_in[i] = KEY_PAD;
      }
      continue;
    }
    const int32_t u = perm[ue], v = perm[ve];  // internal ids
    if (mark && (mark[u] | mark[v])) {
      // an edge entry naming a node that the same batch deletes
      set_error(ctl, ERR_EINVAL);
      if (undirected) {
        k_out[2 * i] = KEY_PAD;
        k_out[2 * i + 1] = KEY_PAD;
      } else {
        k_out[i] = KEY_PAD;
        k_in[i] = KEY_PAD;
      }
      continue;
    }
    if (undirected) {
      // a pair stands for both directed edges; a self-loop for one
      k_out[2 * i] = ((uint64_t)u << b1) | ((uint64_t)v << 1) | t;
      k_out[2 * i + 1] = (u == v) ? KEY_PAD : (((uint64_t)v << b1) | ((uint64_t)u << 1) | t);
    } else {
      k_out[i] = ((uint64_t)u << b1) | ((uint64_t)v << 1) | t;
      k_in[i] = ((uint64_t)v << b1) | ((uint64_t)u << 1) | t;
    }
  }
}

// ------------------------------------------------------- node deletions
// A deleted node loses every incident edge (its row and column of A become
// zero; Section 3.4.1).  The removed edges enter the batch as ordinary
// deletion keys, so validation, the offset seed and the structural update
// treat them like any other deletion.  k_node_mark marks each deleted node
// (internal id) and reports how many adjacency entries its keys are drawn
// from; the host turns the counts into key offsets.
__global__ void k_node_mark(const int32_t *__restrict__ del_nodes, int32_t n_del, const int32_t *__restrict__ perm,
                            DevGraphView out, DevGraphView in, int undirected, int rows_only,
                            int32_t *__restrict__ mark, int64_t *__restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_del) return;
  const int32_t u = perm[del_nodes[i]];
  mark[u] = 1;
  cnt[i] = (int64_t)out.len[u] + (undirected || rows_only ? 0 : in.len[u]);
}

// One block per deleted node u; its keys start at entry `first + off[i]`
// (pairs of entries in undirected mode).  Directed: every out-edge (u, v),
// and (unless rows_only: the row alone, Section 3.4.1 read literally) every
// in-edge (w, u) unless w is u (the self-loop came with the row) or w is
// itself deleted (that edge came with w's row).  Undirected: every pair
// {u, v} once, skipped at u when v is deleted and v < u.  Skipped entries
// are padding.  ctl->node_dels counts the stored entries removed.
__global__ void k_node_keys(const int32_t *__restrict__ del_nodes, const int64_t *__restrict__ off, int64_t first,
                            const int32_t *__restrict__ perm, DevGraphView out, DevGraphView in, int undirected,
                            int rows_only, const int32_t *__restrict__ mark, int b1, uint64_t *__restrict__ k_out,
                            uint64_t *__restrict__ k_in, Ctl *ctl) {
  __shared__ int64_t wsum[256 / RWR_WAVE];
  const int32_t u = perm[del_nodes[blockIdx.x]];
  const int64_t base = first + off[blockIdx.x];
  const int32_t lo = out.len[u];
  const int32_t li = undirected || rows_only ? 0 : in.len[u];
  const int32_t *ro = out.adj + out.off[u];
  const int32_t *ri = in.adj + in.off[u];
  int64_t removed = 0;
  for (int32_t j = threadIdx.x; j < lo + li; j += blockDim.x) {
    const int64_t e = base + j;
    if (undirected) {
      const int32_t v = ro[j];
      if (v == u) {
        k_out[2 * e] = ((uint64_t)u << b1) | ((uint64_t)u << 1);
        k_out[2 * e + 1] = KEY_PAD;
        removed += 1;
      } else if (mark[v] && v < u) {
        k_out[2 * e] = KEY_PAD;
        k_out[2 * e + 1] = KEY_PAD;
      } else {
        k_out[2 * e] = ((uint64_t)u << b1) | ((uint64_t)v << 1);
        k_out[2 * e + 1] = ((uint64_t)v << b1) | ((uint64_t)u << 1);
        removed += 2;
      }
    } else if (j < lo) {
      const int32_t v = ro[j];
      k_out[e] = ((uint64_t)u << b1) | ((uint64_t)v << 1);
      k_in[e] = ((uint64_t)v << b1) | ((uint64_t)u << 1);
      removed += 1;
    } else {
      const int32_t w = ri[j - lo];
      if (w == u || mark[w]) {
        k_out[e] = KEY_PAD;
        k_in[e] = KEY_PAD;
      } else {
        k_out[e] = ((uint64_t)w << b1) | ((uint64_t)u << 1);
        k_in[e] = ((uint64_t)u << b1) | ((uint64_t)w << 1);
        removed += 1;
      }
    }
  }
  removed = wave_xor_sum(removed, 1, RWR_WAVE);
  if (threadIdx.x % RWR_WAVE == 0) wsum[threadIdx.x / RWR_WAVE] = removed;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < (int)(blockDim.x / RWR_WAVE); ++w) t += wsum[w];
    if (t) atomicAdd((unsigned long long *)&ctl->node_dels, (unsigned long long)t);
  }
}

__global__ void k_node_unmark(const int32_t *__restrict__ del_nodes, int32_t n_del, const int32_t *__restrict__ perm,
                              int32_t *__restrict__ mark) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_del) mark[perm[del_nodes[i]]] = 0;
}

// ------------------------------------------------- small batches: one block
// Bitonic sort of up to SMALL_SORT_MAX keys in LDS, then duplicate check and
// segment extraction.  blockIdx.x selects the orientation.
__global__ __launch_bounds__(1024) void k_sort_segment_small(uint64_t *__restrict__ keys0, uint64_t *__restrict__ keys1,
                                                             int32_t n_keys, int b1, int32_t *__restrict__ seg0,
                                                             int32_t *__restrict__ row0, int32_t *__restrict__ seg1,
                                                             int32_t *__restrict__ row1, Ctl *ctl) {
  __shared__ uint64_t s[SMALL_SORT_MAX];
  __shared__ int32_t wsum[1024 / RWR_WAVE];
  uint64_t *keys = blockIdx.x == 0 ? keys0 : keys1;
  int32_t *seg = blockIdx.x == 0 ? seg0 : seg1;
  int32_t *row = blockIdx.x == 0 ? row0 : row1;
  int np = 2;
  while (np < n_keys) np <<= 1;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s[i] = i < n_keys ? keys[i] : KEY_PAD;
  __syncthreads();
  for (int k = 2; k <= np; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < np; i += blockDim.x) {
        const int p = i ^ j;
        if (p > i) {
          const uint64_t a = s[i], b = s[p];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            s[i] = b;
            s[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  // each thread owns a contiguous run of ITEMS positions
  constexpr int ITEMS = SMALL_SORT_MAX / 1024;
  const int base = threadIdx.x * ITEMS;
  int heads = 0;
  int32_t nvalid_local = -1;
  for (int q = 0; q < ITEMS; ++q) {
    const int i = base + q;
    if (i >= np) break;
    const uint64_t k = s[i];
    if (k == KEY_PAD) {
      if (nvalid_local < 0) nvalid_local = i;
      continue;
    }
    if (i > 0) {
      const uint64_t kp = s[i - 1];
      if ((k >> 1) == (kp >> 1) && blockIdx.x == 0) set_error(ctl, ERR_EINVAL);
      if (key_row(k, b1) != key_row(kp, b1)) ++heads;
    } else {
      ++heads;
    }
  }
  // block exclusive scan of `heads`
  const int lane = threadIdx.x % RWR_WAVE, wid = threadIdx.x / RWR_WAVE;
  int incl = heads;
  for (int off = 1; off < RWR_WAVE; off <<= 1) {
    const int t = __shfl_up(incl, off, RWR_WAVE);
    if (lane >= off) incl += t;
  }
  if (lane == RWR_WAVE - 1) wsum[wid] = incl;
  __syncthreads();
  int wbase = 0;
  for (int w = 0; w < wid; ++w) wbase += wsum[w];
  int pos = wbase + incl - heads;
  for (int q = 0; q < ITEMS; ++q) {
    const int i = base + q;
    if (i >= np) break;
    const uint64_t k = s[i];
    if (k == KEY_PAD) break;
    if (i == 0 || key_row(k, b1) != key_row(s[i - 1], b1)) {
      seg[pos] = i;
      row[pos] = key_row(k, b1);
      ++pos;
    }
  }
  for (int i = threadIdx.x; i < n_keys; i += blockDim.x) keys[i] = s[i];
  // first PAD position = number of valid keys; segment end sentinel
  __shared__ int32_t s_nvalid;
  if (threadIdx.x == 0) s_nvalid = np;
  __syncthreads();
  if (nvalid_local >= 0) atomicMin(&s_nvalid, nvalid_local);
  __syncthreads();
  if (threadIdx.x == 0) {
    int total = 0;
    for (int w = 0; w < (int)(blockDim.x / RWR_WAVE); ++w) total += wsum[w];
    seg[total] = s_nvalid < n_keys ? s_nvalid : n_keys;
    ctl->nT[blockIdx.x] = total;
  }
}

// ------------------------------------------------- large batches: device sort
__global__ void k_heads(const uint64_t *__restrict__ keys, int32_t n_keys, int b1, int32_t *__restrict__ flags,
                        Ctl *ctl, int check_dups) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_keys; i += gridDim.x * blockDim.x) {
    const uint64_t k = keys[i];
    int h = 0;
    if (k != KEY_PAD) {
      if (i == 0) {
        h = 1;
      } else {
        const uint64_t kp = keys[i - 1];
        if (check_dups && (k >> 1) == (kp >> 1)) set_error(ctl, ERR_EINVAL);
        h = key_row(k, b1) != key_row(kp, b1);
      }
    }
    flags[i] = h;
  }
}

__global__ void k_segments(const uint64_t *__restrict__ keys, int32_t n_keys, int b1,
                           const int32_t *__restrict__ flags, const int32_t *__restrict__ pos,
                           int32_t *__restrict__ seg, int32_t *__restrict__ row, Ctl *ctl, int orient) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_keys; i += gridDim.x * blockDim.x) {
    const uint64_t k = keys[i];
    if (k == KEY_PAD) continue;
    if (flags[i]) {
      seg[pos[i]] = i;
      row[pos[i]] = key_row(k, b1);
    }
    if (i == n_keys - 1 || keys[i + 1] == KEY_PAD) {
      const int32_t nT = pos[i] + flags[i];
      seg[nT] = i + 1;
      ctl->nT[orient] = nT;
    }
  }
}

// position of `col` in the sorted segment keys[b, e) of row `r`; -1 if absent
__device__ __forceinline__ int32_t seg_find(const uint64_t *__restrict__ keys, int32_t b, int32_t e, int32_t r,
                                            int32_t col, int b1) {
  const uint64_t target = ((uint64_t)r << b1) | ((uint64_t)col << 1);
  int32_t lo = b, hi = e;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (keys[mid] < target)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < e && (keys[lo] >> 1) == (target >> 1)) ? lo : -1;
}

__device__ __forceinline__ int32_t grown_cap(int32_t d) { return d + max(4, d >> 2); }

// ------------------------------------------------- validation and planning
// One wavefront per touched row.  For the out orientation (rows of A~) also
// checks the batch against the graph: an inserted edge must be absent
// (EEXIST), a deleted edge present (ENOENT).  Records old/new degree of each
// touched row and the arena demand of rows that outgrow their capacity.
// Both orientations in one launch (blockIdx.y selects one).
__global__ void k_validate_plan(OrientPair P, int b1, Ctl *ctl) {
  const OrientArgs &q = P.o[blockIdx.y];
  const uint64_t *__restrict__ keys = q.keys;
  const int32_t *__restrict__ seg = q.seg;
  const int32_t *__restrict__ row = q.row;
  const int32_t *__restrict__ off = q.g.off;
  const int32_t *__restrict__ len = q.g.len;
  const int32_t *__restrict__ cap = q.g.cap;
  const int32_t *__restrict__ adj = q.g.adj;
  int32_t *__restrict__ t_dold = q.t_dold;
  int32_t *__restrict__ t_dnew = q.t_dnew;
  const int orient = q.orient, check = q.check, heavy_limit = q.heavy_limit;
  const int lane = threadIdx.x % RWR_WAVE;
  const int32_t t = (blockIdx.x * blockDim.x + threadIdx.x) / RWR_WAVE;
  if (t >= ctl->nT[orient]) return;
  const int32_t u = row[t], b = seg[t], e = seg[t + 1];
  int n_ins = 0;
  for (int32_t i = b + lane; i < e; i += RWR_WAVE) n_ins += (int)(keys[i] & 1ull);
  n_ins = wave_xor_sum(n_ins, 1, RWR_WAVE);
  const int n_del = (e - b) - n_ins;
  const int32_t d_old = len[u];
  int found = 0;
  int exists = 0;
  if (check) {
    const int32_t o = off[u];
    for (int32_t i = lane; i < d_old; i += RWR_WAVE) {
      const int32_t v = adj[o + i];
      const int32_t p = seg_find(keys, b, e, u, v, b1);
      if (p >= 0) {
        if (keys[p] & 1ull)
          exists = 1;
        else
          ++found;
      }
    }
    found = wave_xor_sum(found, 1, RWR_WAVE);
    exists = wave_xor_sum(exists, 1, RWR_WAVE);
  }
  if (lane == 0) {
    if (check) {
      if (exists)
        set_error(ctl, ERR_EEXIST);
      else if (found != n_del)
        set_error(ctl, ERR_ENOENT);
    }
    const int32_t d_new = d_old - n_del + n_ins;
    t_dold[t] = d_old;
    t_dnew[t] = d_new;
    if (d_new > cap[u]) atomicAdd((unsigned long long *)&ctl->demand[orient], (unsigned long long)grown_cap(d_new));
    if (heavy_limit > 0 && d_old <= heavy_limit && d_new > heavy_limit) atomicAdd(&ctl->heavy_stale, 1);
  }
}

// ------------------------------------------------- offset seed
// Work items: touched row u of A~ (before the row is rewritten) cut into
// chunks of SEED_CHUNK old neighbours; item 0 of a row also takes the row's
// inserted neighbours.  k_seed_items counts the items of each touched row
// (0 past the touched rows); an exclusive prefix sum gives each row's first
// item, and the total is the entry at index max_rows.
#define SEED_CHUNK 1024

__global__ void k_seed_items(const int32_t *__restrict__ t_dold, const Ctl *__restrict__ ctl, int32_t max_rows,
                             int32_t *__restrict__ items) {
  const int32_t nT = ctl->err ? 0 : ctl->nT[0];
  for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t <= max_rows; t += gridDim.x * blockDim.x)
    items[t] = t < nT ? max(1, (t_dold[t] + SEED_CHUNK - 1) / SEED_CHUNK) : 0;
}

// Small batches (max_rows < SEED_SMALL): counts and the exclusive prefix sum
// in one workgroup of 1024 threads, four consecutive rows per thread (no
// library scan, one launch less).
#define SEED_SMALL 4096
__global__ __launch_bounds__(1024) void k_seed_items_small(const int32_t *__restrict__ t_dold,
                                                           const Ctl *__restrict__ ctl, int32_t max_rows,
                                                           int32_t *__restrict__ item_off) {
  __shared__ int32_t wsum[1024 / RWR_WAVE];
  const int32_t nT = ctl->err ? 0 : ctl->nT[0];
  const int t = threadIdx.x, lane = t % RWR_WAVE, w = t / RWR_WAVE;
  int32_t v[4];
  int32_t s = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int32_t i = 4 * t + q;
    v[q] = i < nT ? max(1, (t_dold[i] + SEED_CHUNK - 1) / SEED_CHUNK) : 0;
    s += v[q];
  }
  int32_t incl = s;
  for (int off = 1; off < RWR_WAVE; off <<= 1) {
    const int32_t y = __shfl_up(incl, off, RWR_WAVE);
    if (lane >= off) incl += y;
  }
  if (lane == RWR_WAVE - 1) wsum[w] = incl;
  __syncthreads();
  int32_t base = incl - s;
  for (int ww = 0; ww < w; ++ww) base += wsum[ww];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int32_t i = 4 * t + q;
    if (i <= max_rows) item_off[i] = base;
    base += v[q];
  }
}

// One wavefront per item, the waves looping over all items.  Lane layout:
// column j = lane % S, edge slot p = lane / S.  Contributions go to ybuf
// (FP64, atomically); receiving nodes are stamped.  With ybuf null only the
// stamps (the offset support) and the cost model's sums are produced.
template <int S>
__global__ void k_offset_seed(const uint64_t *__restrict__ keys, const int32_t *__restrict__ seg,
                              const int32_t *__restrict__ row, const int32_t *__restrict__ t_dold,
                              const int32_t *__restrict__ t_dnew, const int32_t *__restrict__ item_off,
                              const int32_t *__restrict__ off, const int32_t *__restrict__ adj,
                              const double *__restrict__ r, const double *__restrict__ rsub,
                              double *__restrict__ ybuf, int32_t *__restrict__ stamp, Ctl *ctl, int b1, double c1,
                              int32_t max_rows) {
  if (ctl->err) return;
  constexpr int P = RWR_WAVE / S;
  const int lane = threadIdx.x % RWR_WAVE;
  const int j = lane % S, p = lane / S;
  const int32_t nT = ctl->nT[0];
  const int32_t total = item_off[max_rows];
  const int32_t st = ctl->stamp;
  for (int32_t it = (blockIdx.x * blockDim.x + threadIdx.x) / RWR_WAVE; it < total;
       it += gridDim.x * blockDim.x / RWR_WAVE) {
    // the touched row of item `it`: last t with item_off[t] <= it
    int32_t lo = 0, hi = nT - 1;
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (item_off[mid] <= it) lo = mid;
      else hi = mid - 1;
    }
    const int32_t t = lo;
    const int32_t k = it - item_off[t];
    const int32_t u = row[t], b = seg[t], e = seg[t + 1];
    const int32_t d_old = t_dold[t], d_new = t_dnew[t];
    // the scores without a deferred last iterate (rsub) when one is carried
    const double ru = rsub ? r[col_index(u, S, j)] - rsub[col_index(u, S, j)] : r[col_index(u, S, j)];
    if (__ballot(ru != 0.0) == 0ull) continue;
    const double w_old = d_old ? c1 * ru / (double)d_old : 0.0;
    const double w_new = d_new ? c1 * ru / (double)d_new : 0.0;
    const int32_t o = off[u];
    const int32_t i1 = min(d_old, (k + 1) * SEED_CHUNK);
    for (int32_t i = k * SEED_CHUNK + p; i < i1; i += P) {
      const int32_t v = adj[o + i];
      const bool del = seg_find(keys, b, e, u, v, b1) >= 0;  // validated: a hit is a deletion
      const double contrib = del ? -w_old : (w_new - w_old);
      if (ybuf && contrib != 0.0) atomic_add_f64(&ybuf[col_index(v, S, j)], contrib);
      if (j == 0 && (del || d_new != d_old)) stamp[v] = st;
    }
    if (k != 0) continue;
    if (p == 0) {
      // cost model: D_uu |r_old(u)|, D_uu = sum_v |B~[u,v] - A~[u,v]| =
      // kept |1/d_new - 1/d_old| + inserted / d_new + deleted / d_old
      int32_t n_ins = 0;
      for (int32_t i = b; i < e; ++i) n_ins += (int32_t)(keys[i] & 1ull);
      const int32_t n_del = (e - b) - n_ins, kept = d_old - n_del;
      double du = 0.0;
      if (d_old > 0 && d_new > 0) du += kept * fabs(1.0 / d_new - 1.0 / d_old);
      if (d_new > 0) du += n_ins / (double)d_new;
      if (d_old > 0) du += n_del / (double)d_old;
      // without ybuf (deterministic mode) in fixed point: integer sums do not
      // depend on the order of the additions
      if (ybuf)
        atomic_add_f64(&ctl->dr_l1[j], du * fabs(ru));
      else
        atomicAdd((unsigned long long *)&ctl->dr_fix[j], (unsigned long long)llrint(du * fabs(ru) * 0x1p52));
    }
    for (int32_t i = b + p; i < e; i += P) {
      const uint64_t kk = keys[i];
      if (!(kk & 1ull)) continue;
      const int32_t v = key_col(kk, b1);
      if (ybuf && w_new != 0.0) atomic_add_f64(&ybuf[col_index(v, S, j)], w_new);
      if (j == 0) stamp[v] = st;
    }
  }
}

// ------------------------------------------- offset seed in a fixed order
// The offset seed without floating-point atomics, for runs that must not
// depend on timing.  After the structural apply, every node v that the
// support pass stamped gets q(v, j) with a plain store, summed in one fixed
// order: the in-row of v in the new graph (each in-neighbour u whose row the
// batch changed contributes (1-c) r(u) / d_new(u), minus (1-c) r(u) /
// d_old(u) unless the edge (u, v) is inserted), then the edges into v that
// the batch deletes (-(1-c) r(u) / d_old(u)), in key order; lane parts are
// added by a fixed shuffle tree.  tmark[u] = 1 + the index of u's segment
// among the changed rows (out orientation), imark[v] = 1 + the index of v's
// segment among the changed rows of the pull orientation, 0 elsewhere.
__global__ void k_mark_segments(const int32_t *__restrict__ row0, const int32_t *__restrict__ rowp, Ctl *ctl,
                                int po, int32_t *__restrict__ tmark, int32_t *__restrict__ imark, int32_t value) {
  if (ctl->err) return;
  const int32_t n0 = ctl->nT[0], np = ctl->nT[po];
  for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < max(n0, np); t += gridDim.x * blockDim.x) {
    if (t < n0) tmark[row0[t]] = value ? t + 1 : 0;
    if (t < np) imark[rowp[t]] = value ? t + 1 : 0;
  }
}

template <int S>
__global__ void k_offset_pull(const int32_t *__restrict__ stamp, const Ctl *ctl, int32_t n, DevGraphView in,
                              const int32_t *__restrict__ tmark, const int32_t *__restrict__ t_dold,
                              const int32_t *__restrict__ t_dnew, const int32_t *__restrict__ imark,
                              const uint64_t *__restrict__ ikeys, const int32_t *__restrict__ iseg, int b1,
                              const double *__restrict__ r, const double *__restrict__ rsub,
                              double *__restrict__ ybuf, double c1) {
  if (ctl->err) return;
  constexpr int P = RWR_WAVE / S;
  const int lane = threadIdx.x % RWR_WAVE;
  const int j = lane % S, p = lane / S;
  const int32_t st = ctl->stamp;
  auto score = [&](int u) -> double {
    const int64_t k = col_index(u, S, j);
    return rsub ? r[k] - rsub[k] : r[k];
  };
  const int nwv = gridDim.x * (blockDim.x / RWR_WAVE);
  for (int base = ((blockIdx.x * blockDim.x + threadIdx.x) / RWR_WAVE) * RWR_WAVE; base < n;
       base += nwv * RWR_WAVE) {
    // the stamped nodes among 64 consecutive ones, one at a time
    unsigned long long m = __ballot(base + lane < n && stamp[base + lane] == st);
    while (m) {
      const int v = base + __builtin_ctzll(m);
      m &= m - 1;
      const int32_t sv = imark[v];
      const int32_t b = sv ? iseg[sv - 1] : 0, e = sv ? iseg[sv] : 0;
      const int o = in.off[v], d = in.len[v];
      double q = 0.0;
      for (int i = p; i < d; i += P) {
        const int u = in.adj[o + i];
        const int32_t tu = tmark[u];
        if (!tu) continue;
        const double ru = score(u);
        const int d_old = t_dold[tu - 1], d_new = t_dnew[tu - 1];
        const double w_new = d_new ? c1 * ru / (double)d_new : 0.0;
        const double w_old = d_old ? c1 * ru / (double)d_old : 0.0;
        const int32_t hit = sv ? seg_find(ikeys, b, e, v, u, b1) : -1;
        q += (hit >= 0 && (ikeys[hit] & 1ull)) ? w_new : (w_new - w_old);
      }
      for (int32_t i = b + p; i < e; i += P) {
        const uint64_t kk = ikeys[i];
        if (kk & 1ull) continue;  // an insertion: counted in the in-row
        const int u = key_col(kk, b1);
        const int32_t tu = tmark[u];
        const int d_old = tu ? t_dold[tu - 1] : 0;
        if (d_old) q -= c1 * score(u) / (double)d_old;
      }
      for (int off = S; off < RWR_WAVE; off <<= 1) q += __shfl_xor(q, off, RWR_WAVE);
      if (p == 0) ybuf[col_index(v, S, j)] = q;
    }
  }
}

hipError_t launch_offset_pull(int S, const OrientPair &P, int po, const DevGraphView &in, const int32_t *stamp,
                              const Ctl *ctl, int32_t n, int32_t *tmark, int32_t *imark, int b1, const double *r,
                              const double *rsub, double *ybuf, double c1, int32_t max_rows, int grid,
                              hipStream_t st) {
  const int mg = std::max(1, std::min(1024, (max_rows + 255) / 256));
  hipLaunchKernelGGL(k_mark_segments, dim3(mg), dim3(256), 0, st, P.o[0].row, P.o[po].row, (Ctl *)ctl, po, tmark,
                     imark, 1);
#define RWR_PULL_CASE(SS)                                                                                        \
  case SS:                                                                                                       \
    hipLaunchKernelGGL(k_offset_pull<SS>, dim3(grid), dim3(256), 0, st, stamp, ctl, n, in, tmark, P.o[0].t_dold, \
                       P.o[0].t_dnew, imark, P.o[po].keys, P.o[po].seg, b1, r, rsub, ybuf, c1);                   \
    break;
  switch (S) {
    RWR_PULL_CASE(1)
    RWR_PULL_CASE(2)
    RWR_PULL_CASE(4)
    RWR_PULL_CASE(8)
    RWR_PULL_CASE(16)
    RWR_PULL_CASE(32)
    RWR_PULL_CASE(64)
  }
#undef RWR_PULL_CASE
  hipLaunchKernelGGL(k_mark_segments, dim3(mg), dim3(256), 0, st, P.o[0].row, P.o[po].row, (Ctl *)ctl, po, tmark,
                     imark, 0);
  return hipGetLastError();
}

// ------------------------------------------------- structural apply
// One wavefront per touched row: drop deleted entries (stable compaction in
// place, or into a fresh arena slot when the row outgrows its capacity), then
// append the inserted entries.
__global__ void k_apply(OrientPair P, int b1, Ctl *ctl) {
  const OrientArgs &q = P.o[blockIdx.y];
  const uint64_t *__restrict__ keys = q.keys;
  const int32_t *__restrict__ seg = q.seg;
  const int32_t *__restrict__ row = q.row;
  const int32_t *__restrict__ t_dold = q.t_dold;
  const int32_t *__restrict__ t_dnew = q.t_dnew;
  int32_t *__restrict__ off = q.g.off;
  int32_t *__restrict__ len = q.g.len;
  int32_t *__restrict__ cap = q.g.cap;
  int32_t *__restrict__ adj = q.g.adj;
  const int orient = q.orient;
  const int64_t e_cap = q.e_cap;
  if (ctl->err) return;
  const int lane = threadIdx.x % RWR_WAVE;
  const int32_t t = (blockIdx.x * blockDim.x + threadIdx.x) / RWR_WAVE;
  if (t >= ctl->nT[orient]) return;
  const int32_t u = row[t], b = seg[t], e = seg[t + 1];
  const int32_t d_old = t_dold[t], d_new = t_dnew[t];
  const int32_t o = off[u];
  int32_t base = o;
  int32_t ncap = cap[u];
  const bool move = d_new > ncap;
  if (move) {
    ncap = grown_cap(d_new);
    unsigned long long pos = 0;
    if (lane == 0) pos = atomicAdd((unsigned long long *)&ctl->tail[orient], (unsigned long long)ncap);
    pos = (unsigned long long)__shfl((long long)pos, 0, RWR_WAVE);
    if ((int64_t)pos + ncap > e_cap) {
      // the host sizes the arena from the validated demand; never write past it
      if (lane == 0) atomicCAS(&ctl->prop_err, 0, ERR_ENOMEM);
      return;
    }
    base = (int32_t)pos;
  }
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (RWR_WAVE - lane));
  int32_t w = 0;
  for (int32_t i0 = 0; i0 < d_old; i0 += RWR_WAVE) {
    const int32_t i = i0 + lane;
    int32_t v = -1;
    bool keep = false;
    if (i < d_old) {
      v = adj[o + i];
      keep = seg_find(keys, b, e, u, v, b1) < 0;
    }
    const uint64_t m = __ballot(keep);
    if (keep) adj[base + w + __popcll(m & lt_mask)] = v;
    w += __popcll(m);
  }
  for (int32_t i0 = b; i0 < e; i0 += RWR_WAVE) {
    const int32_t i = i0 + lane;
    const bool ins = i < e && (keys[i] & 1ull);
    const uint64_t m = __ballot(ins);
    if (ins) adj[base + w + __popcll(m & lt_mask)] = key_col(keys[i], b1);
    w += __popcll(m);
  }
  if (lane == 0) {
    len[u] = d_new;
    if (move) {
      off[u] = base;
      cap[u] = ncap;
    }
  }
}

__global__ void k_reset_batch(Ctl *ctl, int demand_only) {
  if (!demand_only) {
    ctl->err = 0;
    ctl->nT[0] = 0;
    ctl->nT[1] = 0;
  }
  ctl->demand[0] = 0;
  ctl->demand[1] = 0;
  ctl->heavy_stale = 0;
  if (!demand_only) {
    ctl->node_dels = 0;
    for (int j = 0; j < RWR_MAX_COLS; ++j) {
      ctl->dr_l1[j] = 0.0;
      ctl->dr_fix[j] = 0;
    }
  }
}

// ------------------------------------------------- host launchers
void launch_reset_batch(Ctl *ctl, int demand_only, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_batch, dim3(1), dim3(1), 0, st, ctl, demand_only);
}

void launch_make_keys(const int32_t *ins_s, const int32_t *ins_d, int64_t n_ins, const int32_t *del_s,
                      const int32_t *del_d, int64_t n_del, int32_t n_nodes, int b1, int undirected,
                      const int32_t *perm, const int32_t *mark, uint64_t *k_out, uint64_t *k_in, Ctl *ctl,
                      hipStream_t st) {
  const int64_t total = n_ins + n_del;
  if (total == 0) return;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_make_keys, dim3(grid), dim3(256), 0, st, ins_s, ins_d, n_ins, del_s, del_d, n_del, n_nodes,
                     b1, undirected, perm, mark, k_out, k_in, ctl);
}

void launch_node_mark(const int32_t *del_nodes, int32_t n_del, const int32_t *perm, const DevGraphView &out,
                      const DevGraphView &in, int undirected, int rows_only, int32_t *mark, int64_t *cnt,
                      hipStream_t st) {
  if (n_del <= 0) return;
  hipLaunchKernelGGL(k_node_mark, dim3((n_del + 255) / 256), dim3(256), 0, st, del_nodes, n_del, perm, out, in,
                     undirected, rows_only, mark, cnt);
}

void launch_node_keys(const int32_t *del_nodes, int32_t n_del, const int64_t *off, int64_t first,
                      const int32_t *perm, const DevGraphView &out, const DevGraphView &in, int undirected,
                      int rows_only, const int32_t *mark, int b1, uint64_t *k_out, uint64_t *k_in, Ctl *ctl,
                      hipStream_t st) {
  if (n_del <= 0) return;
  hipLaunchKernelGGL(k_node_keys, dim3(n_del), dim3(256), 0, st, del_nodes, off, first, perm, out, in, undirected,
                     rows_only, mark, b1, k_out, k_in, ctl);
}

void launch_node_unmark(const int32_t *del_nodes, int32_t n_del, const int32_t *perm, int32_t *mark,
                        hipStream_t st) {
  if (n_del <= 0) return;
  hipLaunchKernelGGL(k_node_unmark, dim3((n_del + 255) / 256), dim3(256), 0, st, del_nodes, n_del, perm, mark);
}

void launch_sort_segment_small(uint64_t *k0, uint64_t *k1, int32_t n_keys, int b1, int32_t *seg0, int32_t *row0,
                               int32_t *seg1, int32_t *row1, int orientations, Ctl *ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_sort_segment_small, dim3(orientations), dim3(1024), 0, st, k0, k1, n_keys, b1, seg0, row0,
                     seg1, row1, ctl);
}

hipError_t sort_segment_large(uint64_t *keys, uint64_t *keys_alt, int32_t n_keys, int b1, int32_t *flags,
                              int32_t *pos, int32_t *seg, int32_t *row, void *temp, size_t temp_bytes, Ctl *ctl,
                              int orient, hipStream_t st) {
  const int end_bit = std::min(64, 2 * b1 + 1);
  size_t bytes = temp_bytes;
  hipError_t err = hipcub::DeviceRadixSort::SortKeys(temp, bytes, keys, keys_alt, n_keys, 0, end_bit, st);
  if (err != hipSuccess) return err;
  const int grid = std::min((n_keys + 255) / 256, 4096);
  hipLaunchKernelGGL(k_heads, dim3(grid), dim3(256), 0, st, keys_alt, n_keys, b1, flags, ctl, orient == 0 ? 1 : 0);
  bytes = temp_bytes;
  err = hipcub::DeviceScan::ExclusiveSum(temp, bytes, flags, pos, n_keys, st);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_segments, dim3(grid), dim3(256), 0, st, keys_alt, n_keys, b1, flags, pos, seg, row, ctl,
                     orient);
  return hipMemcpyAsync(keys, keys_alt, sizeof(uint64_t) * (size_t)n_keys, hipMemcpyDeviceToDevice, st);
}

size_t sort_temp_bytes(int32_t n_keys) {
  size_t a = 0, b = 0;
  (void)hipcub::DeviceRadixSort::SortKeys((void *)nullptr, a, (uint64_t *)nullptr, (uint64_t *)nullptr, n_keys, 0, 64);
  (void)hipcub::DeviceScan::ExclusiveSum((void *)nullptr, b, (int32_t *)nullptr, (int32_t *)nullptr, n_keys);
  return std::max(a, b);
}

void launch_validate_plan(const OrientPair &P, int norient, int b1, Ctl *ctl, int32_t max_rows, hipStream_t st) {
  if (max_rows <= 0) return;
  const int waves_per_block = 4;
  const int grid = (max_rows + waves_per_block - 1) / waves_per_block;
  hipLaunchKernelGGL(k_validate_plan, dim3(grid, norient), dim3(waves_per_block * RWR_WAVE), 0, st, P, b1, ctl);
}

template <int S>
static void offset_seed_s(const uint64_t *keys, const int32_t *seg, const int32_t *row, const int32_t *t_dold,
                          const int32_t *t_dnew, const int32_t *item_off, const DevGraphView &g, const double *r,
                          const double *rsub, double *ybuf, int32_t *stamp, Ctl *ctl, int b1, double c1,
                          int32_t max_rows, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_offset_seed<S>, dim3(grid), dim3(256), 0, st, keys, seg, row, t_dold, t_dnew, item_off, g.off,
                     g.adj, r, rsub, ybuf, stamp, ctl, b1, c1, max_rows);
}

hipError_t launch_offset_seed(int S, const uint64_t *keys, const int32_t *seg, const int32_t *row,
                              const int32_t *t_dold, const int32_t *t_dnew, const DevGraphView &g, const double *r,
                              const double *rsub, double *ybuf, int32_t *stamp, Ctl *ctl, int b1, double c1,
                              int32_t max_rows, int32_t *items, int32_t *item_off, void *temp, size_t temp_bytes,
                              int grid, hipStream_t st) {
  if (max_rows <= 0) return hipSuccess;
  if (max_rows < SEED_SMALL) {
    hipLaunchKernelGGL(k_seed_items_small, dim3(1), dim3(1024), 0, st, t_dold, ctl, max_rows, item_off);
  } else {
    hipLaunchKernelGGL(k_seed_items, dim3(std::min(4096, (max_rows + 256) / 256)), dim3(256), 0, st, t_dold, ctl,
                       max_rows, items);
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(temp, temp_bytes, items, item_off, max_rows + 1, st);
    if (e != hipSuccess) return e;
  }
#define RWR_SEED_CASE(SS)                                                                                        \
  case SS:                                                                                                       \
    offset_seed_s<SS>(keys, seg, row, t_dold, t_dnew, item_off, g, r, rsub, ybuf, stamp, ctl, b1, c1, max_rows, \
                      grid, st);                                                                                 \
    break;
  switch (S) {
    RWR_SEED_CASE(1)
    RWR_SEED_CASE(2)
    RWR_SEED_CASE(4)
    RWR_SEED_CASE(8)
    RWR_SEED_CASE(16)
    RWR_SEED_CASE(32)
    RWR_SEED_CASE(64)
  }
#undef RWR_SEED_CASE
  return hipSuccess;
}

size_t seed_scan_temp_bytes(int32_t max_rows) {
  size_t bytes = 0;
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, (const int32_t *)nullptr, (int32_t *)nullptr, max_rows + 1);
  return bytes;
}

void launch_apply(const OrientPair &P, int norient, int b1, Ctl *ctl, int32_t max_rows, hipStream_t st) {
  if (max_rows <= 0) return;
  const int waves_per_block = 4;
  const int grid = (max_rows + waves_per_block - 1) / waves_per_block;
  hipLaunchKernelGGL(k_apply, dim3(grid, norient), dim3(waves_per_block * RWR_WAVE), 0, st, P, b1, ctl);
}
