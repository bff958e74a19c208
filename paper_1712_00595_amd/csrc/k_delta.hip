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

// seg_find for SEG_W columns at once (a negative column is skipped: -1): the
// searches halve the same range in lockstep, so their loads are in flight
// together.  nq (the same in every lane of a wavefront): only columns
// 0 .. nq-1 are searched, so a short row costs no more than one search.
#define SEG_W 4
__device__ __forceinline__ void seg_find_w(const uint64_t *__restrict__ keys, int32_t b, int32_t e, int32_t r,
                                           const int32_t (&col)[SEG_W], int b1, int32_t (&pos)[SEG_W],
                                           int nq = SEG_W) {
  uint64_t tg[SEG_W];
  int32_t base[SEG_W];
#pragma unroll
  for (int q = 0; q < SEG_W; ++q) {
    tg[q] = ((uint64_t)r << b1) | ((uint64_t)max(col[q], 0) << 1);
    base[q] = b;
    pos[q] = -1;
  }
  if (e <= b) return;
  for (int32_t n = e - b; n > 1;) {
    const int32_t half = n >> 1;
#pragma unroll
    for (int q = 0; q < SEG_W; ++q)
      if (q < nq) base[q] = keys[base[q] + half] < tg[q] ? base[q] + half : base[q];
    n -= half;
  }
#pragma unroll
  for (int q = 0; q < SEG_W; ++q) {
    if (q >= nq) break;
    const uint64_t k = keys[base[q]];
    const int32_t at = k < tg[q] ? base[q] + 1 : base[q];
    if (col[q] >= 0 && at < e && (keys[at] >> 1) == (tg[q] >> 1)) pos[q] = at;
  }
}

__device__ __forceinline__ int32_t grown_cap(int32_t d) { return d + max(4, d >> 2); }

// ------------------------------------------------- validation and planning
// One wavefront per touched row.  For the out orientation (rows of A~) also
// checks the batch against the graph: an inserted edge must be absent
// (EEXIST), a deleted edge present (ENOENT).  Records old/new degree of each
// touched row and the arena demand of rows that outgrow their capacity.
// Both orientations in one launch (blockIdx.y selects one).  With P.big, a
// row above BIG_ROW entries is listed instead for k_validate_big (its check)
// and, when its entries must be compacted or moved, for k_apply_big.
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
  const bool big = P.big && d_old > BIG_ROW;
  int found = 0;
  int exists = 0;
  if (check && !big) {
    // SEG_W x 64 neighbours per step: their loads and searches in flight together
    const int32_t o = off[u];
    for (int32_t i0 = 0; i0 < d_old; i0 += SEG_W * RWR_WAVE) {
      int32_t v[SEG_W], p[SEG_W];
#pragma unroll
      for (int q = 0; q < SEG_W; ++q) {
        const int32_t i = i0 + q * RWR_WAVE + lane;
        v[q] = i < d_old ? adj[o + i] : -1;
      }
      seg_find_w(keys, b, e, u, v, b1, p, (d_old - i0 + RWR_WAVE - 1) / RWR_WAVE);
#pragma unroll
      for (int q = 0; q < SEG_W; ++q)
        if (p[q] >= 0) {
          if (keys[p[q]] & 1ull)
            exists = 1;
          else
            ++found;
        }
    }
    found = wave_xor_sum(found, 1, RWR_WAVE);
    exists = wave_xor_sum(exists, 1, RWR_WAVE);
  }
  if (lane == 0) {
    if (check && !big) {
      if (exists)
        set_error(ctl, ERR_EEXIST);
      else if (found != n_del)
        set_error(ctl, ERR_ENOENT);
    }
    const int32_t d_new = d_old - n_del + n_ins;
    if (big && check) P.bigv[atomicAdd(&ctl->nbig_v, 1)] = t;
    if (big && (n_del > 0 || d_new > cap[u])) P.biga[atomicAdd(&ctl->nbig_a, 1)] = (int32_t)((unsigned)orient << 31) | t;
    t_dold[t] = d_old;
    t_dnew[t] = d_new;
    if (d_new > cap[u]) atomicAdd((unsigned long long *)&ctl->demand[orient], (unsigned long long)grown_cap(d_new));
    if (orient == 0 && P.recs)
      atomicAdd((unsigned long long *)&ctl->seed_recs[blockIdx.x % 32], (unsigned long long)d_old);
    if (heavy_limit > 0 && d_old <= heavy_limit && d_new > heavy_limit) atomicAdd(&ctl->heavy_stale, 1);
  }
}

// ------------------------------------------------- offset seed
// Work items: touched row u of A~ (before the row is rewritten) cut into
// chunks of SEED_CHUNK old neighbours; item 0 of a row also takes the row's
// inserted neighbours.  k_seed_items counts the items of each touched row
// (0 past the touched rows); an exclusive prefix sum gives each row's first
// item, and the total is the entry at index max_rows.  When the seed is
// written as records (sort and reduce, below), a second prefix sum over the
// old degrees gives each row's first record slot: row t owns d_old(t) slots
// for its old neighbours followed by one per key of its batch segment, from
// rec_off[t] + seg[t].
#define SEED_CHUNK 1024

// A record of the seed's sort-and-reduce form: receiving node v above rsh
// bits, touched row t above 2 bits, the term's kind in the low 2 bits.  The
// pad key (kind 3) sorts after every record.
#define SEED_KEPT 0ull  // kept edge: (1-c) r(u) (1/d_new - 1/d_old)
#define SEED_DEL 1ull   // deleted edge: -(1-c) r(u) / d_old
#define SEED_INS 2ull   // inserted edge: (1-c) r(u) / d_new
#define SEED_PAD (~0ull)
__device__ __forceinline__ uint64_t seed_rec_key(int32_t v, int32_t t, uint64_t kind, int rsh) {
  return ((uint64_t)v << rsh) | ((uint64_t)t << 2) | kind;
}

__global__ void k_seed_items(const int32_t *__restrict__ t_dold, const Ctl *__restrict__ ctl, int32_t max_rows,
                             int32_t *__restrict__ items, int32_t *__restrict__ dcnt) {
  const int32_t nT = ctl->err ? 0 : ctl->nT[0];
  for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t <= max_rows; t += gridDim.x * blockDim.x) {
    items[t] = t < nT ? max(1, (t_dold[t] + SEED_CHUNK - 1) / SEED_CHUNK) : 0;
    if (dcnt) dcnt[t] = t < nT ? t_dold[t] : 0;
  }
}

// Small batches (max_rows < SEED_SMALL): counts and the exclusive prefix sum
// in one workgroup of 1024 threads, four consecutive rows per thread (no
// library scan, one launch less).
#define SEED_SMALL 4096
__device__ __forceinline__ int32_t block_exclusive_scan4(const int32_t (&v)[4], int32_t *wsum) {
  const int t = threadIdx.x, lane = t % RWR_WAVE, w = t / RWR_WAVE;
  const int32_t s = v[0] + v[1] + v[2] + v[3];
  int32_t incl = s;
  for (int off = 1; off < RWR_WAVE; off <<= 1) {
    const int32_t y = __shfl_up(incl, off, RWR_WAVE);
    if (lane >= off) incl += y;
  }
  if (lane == RWR_WAVE - 1) wsum[w] = incl;
  __syncthreads();
  int32_t base = incl - s;
  for (int ww = 0; ww < w; ++ww) base += wsum[ww];
  return base;
}

__global__ __launch_bounds__(1024) void k_seed_items_small(const int32_t *__restrict__ t_dold,
                                                           const Ctl *__restrict__ ctl, int32_t max_rows,
                                                           int32_t *__restrict__ item_off,
                                                           int32_t *__restrict__ rec_off) {
  __shared__ int32_t wsum[2][1024 / RWR_WAVE];
  const int32_t nT = ctl->err ? 0 : ctl->nT[0];
  const int t = threadIdx.x;
  int32_t v[4], d[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int32_t i = 4 * t + q;
    v[q] = i < nT ? max(1, (t_dold[i] + SEED_CHUNK - 1) / SEED_CHUNK) : 0;
    d[q] = i < nT ? t_dold[i] : 0;
  }
  int32_t base = block_exclusive_scan4(v, wsum[0]);
  int32_t dbase = rec_off ? block_exclusive_scan4(d, wsum[1]) : 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int32_t i = 4 * t + q;
    if (i <= max_rows) {
      item_off[i] = base;
      if (rec_off) rec_off[i] = dbase;
    }
    base += v[q];
    dbase += d[q];
  }
}

// One wavefront per item, the waves looping over all items.  The item's old
// neighbours are tested 64 at a time, one per lane (is the edge deleted?);
// each lane stamps its receiving node and writes its record slot.  The
// contributions to ybuf (FP64, atomically) then take the lane layout column
// j = lane % S, edge slot p = lane / S, P entries per step.  With ybuf null
// only the stamps (the offset support), the records (rec set: every slot of
// the item gets its record, a structurally nonzero term, or the pad key) and
// the cost model's sums are produced.
template <int S>
__global__ void k_offset_seed(const uint64_t *__restrict__ keys, const int32_t *__restrict__ seg,
                              const int32_t *__restrict__ row, const int32_t *__restrict__ t_dold,
                              const int32_t *__restrict__ t_dnew, const int32_t *__restrict__ item_off,
                              const int32_t *__restrict__ off, const int32_t *__restrict__ adj,
                              const double *__restrict__ r, const double *__restrict__ rsub,
                              double *__restrict__ ybuf, int32_t *__restrict__ stamp, Ctl *ctl, int b1, double c1,
                              int32_t max_rows, uint64_t *__restrict__ rec, const int32_t *__restrict__ rec_off,
                              int rsh, uint64_t rmask) {
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
    // the scores without a carried vector (rsub, in the columns of rmask)
    const double ru = rsub && ((rmask >> j) & 1ull) ? r[col_index(u, S, j)] - rsub[col_index(u, S, j)]
                                                    : r[col_index(u, S, j)];
    const int32_t i1 = min(d_old, (k + 1) * SEED_CHUNK);
    // this item's record slots: old neighbours k*SEED_CHUNK .. i1, and (item
    // 0) the segment's keys
    const int64_t rb = rec ? (int64_t)rec_off[t] + b : 0;
    if (__ballot(ru != 0.0) == 0ull) {
      if (rec) {
        for (int32_t i = k * SEED_CHUNK + lane; i < i1; i += RWR_WAVE) rec[rb + i] = SEED_PAD;
        if (k == 0)
          for (int32_t i = b + lane; i < e; i += RWR_WAVE) rec[rb + d_old + (i - b)] = SEED_PAD;
      }
      continue;
    }
    const double w_old = d_old ? c1 * ru / (double)d_old : 0.0;
    const double w_new = d_new ? c1 * ru / (double)d_new : 0.0;
    const int32_t o = off[u];
    for (int32_t i0 = k * SEED_CHUNK; i0 < i1; i0 += RWR_WAVE) {
      const int32_t il = i0 + lane;
      int32_t vl = 0;
      int dl = 0;
      if (il < i1) {
        vl = adj[o + il];
        dl = seg_find(keys, b, e, u, vl, b1) >= 0;  // validated: a hit is a deletion
        const bool nz = dl || d_new != d_old;
        if (nz) stamp[vl] = st;
        if (rec) rec[rb + il] = nz ? seed_rec_key(vl, t, dl ? SEED_DEL : SEED_KEPT, rsh) : SEED_PAD;
      }
      if (!ybuf) continue;
      const int cnt = min(RWR_WAVE, i1 - i0);
      for (int s0 = 0; s0 < cnt; s0 += P) {
        const int src = s0 + p;
        const int32_t v = __shfl(vl, src, RWR_WAVE);
        const int del = __shfl(dl, src, RWR_WAVE);
        const double contrib = del ? -w_old : (w_new - w_old);
        if (src < cnt && contrib != 0.0) atomic_add_f64(&ybuf[col_index(v, S, j)], contrib);
      }
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
    for (int32_t i = b + lane; i < e; i += RWR_WAVE) {
      const uint64_t kk = keys[i];
      const int32_t v = key_col(kk, b1);
      if (rec) rec[rb + d_old + (i - b)] = (kk & 1ull) ? seed_rec_key(v, t, SEED_INS, rsh) : SEED_PAD;
      if (kk & 1ull) stamp[v] = st;
    }
    if (ybuf && w_new != 0.0)
      for (int32_t i = b + p; i < e; i += P) {
        const uint64_t kk = keys[i];
        if (kk & 1ull) atomic_add_f64(&ybuf[col_index(key_col(kk, b1), S, j)], w_new);
      }
  }
}

// ------------------------------------------- offset seed in a fixed order
// The offset seed without floating-point atomics, for runs that must not
// depend on timing (and for large batches, where it is also faster): the
// support pass writes one record per structurally nonzero term of
// (1-c)(B~^T - A~^T) r_old, the records are radix-sorted, and each node's
// terms are summed in sorted order.  Keys are unique (one term per edge of a
// touched row), so the sorted order, and with it every sum, does not depend
// on the order the records were written in.
//
// The sorted records are cut into chunks of SEED_RED_CH; one group of S lanes
// (lane = column) walks a chunk.  A node whose terms lie inside one chunk is
// stored from there; a node whose terms cross chunk boundaries leaves its
// first chunk's sum in tpart and each later chunk's sum in hpart, and
// k_seed_fixup adds them in chunk order.
#define SEED_RED_CH 128
#define SEED_RED_U 16

template <int S>
__global__ __launch_bounds__(256) void k_seed_reduce(const uint64_t *__restrict__ rec, int32_t n_rec, int rsh,
                                                     uint64_t tmask, const int32_t *__restrict__ row,
                                                     const int32_t *__restrict__ t_dold,
                                                     const int32_t *__restrict__ t_dnew,
                                                     const double *__restrict__ r, const double *__restrict__ rsub,
                                                     uint64_t rmask, double c1, double *__restrict__ ybuf,
                                                     double *__restrict__ hpart, double *__restrict__ tpart,
                                                     const Ctl *ctl) {
  if (ctl->err) return;
  constexpr int G = RWR_WAVE / S;
  constexpr int U = S < SEED_RED_U ? S : SEED_RED_U;
  const int lane = threadIdx.x % RWR_WAVE, j = lane % S, g = lane / S;
  const double *__restrict__ sub = (rmask >> j) & 1ull ? rsub : nullptr;
  const int32_t nch = (n_rec + SEED_RED_CH - 1) / SEED_RED_CH;
  const int64_t ngroups = (int64_t)gridDim.x * (blockDim.x / RWR_WAVE) * G;
  for (int64_t c = (int64_t)((blockIdx.x * blockDim.x + threadIdx.x) / RWR_WAVE) * G + g; c < nch; c += ngroups) {
    const int32_t b = (int32_t)c * SEED_RED_CH, e = min(n_rec, b + SEED_RED_CH);
    if ((rec[b] & 3ull) == 3ull) continue;  // pads only
    int32_t cur = (int32_t)(rec[b] >> rsh);
    const bool open_l = b > 0 && (int32_t)(rec[b - 1] >> rsh) == cur;
    bool first_seg = true, done = false;
    double acc = 0.0;
    for (int32_t i0 = b; i0 < e && !done; i0 += S) {
      // decode S records, one per lane of the group: receiving node (-1 for
      // a pad), source node, coefficient of its score
      const int32_t ir = i0 + j;
      const uint64_t kk = ir < e ? rec[ir] : SEED_PAD;
      int32_t vv = -1, uu = 0;
      double aa = 0.0;
      if ((kk & 3ull) != 3ull) {
        const int32_t t = (int32_t)((kk >> 2) & tmask);
        const uint64_t kind = kk & 3ull;
        vv = (int32_t)(kk >> rsh);
        uu = row[t];
        const int32_t d_old = t_dold[t], d_new = t_dnew[t];
        const double wo = d_old ? c1 / (double)d_old : 0.0, wn = d_new ? c1 / (double)d_new : 0.0;
        aa = kind == SEED_KEPT ? wn - wo : (kind == SEED_DEL ? -wo : wn);
      }
      // then the group's lanes are columns: U records' scores in flight, summed in order
      for (int k0 = 0; k0 < S && !done; k0 += U) {
        int32_t vk[U];
        double ak[U], x[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
          const int src = g * S + k0 + q;
          vk[q] = __shfl(vv, src, RWR_WAVE);
          const int32_t uk = __shfl(uu, src, RWR_WAVE);
          ak[q] = __shfl(aa, src, RWR_WAVE);
          const int64_t kx = col_index(uk, S, j);
          x[q] = vk[q] < 0 ? 0.0 : (sub ? r[kx] - sub[kx] : r[kx]);
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
          if (done || vk[q] < 0) {
            done = true;
            continue;
          }
          if (vk[q] != cur) {
            if (first_seg && open_l)
              hpart[c * S + j] = acc;
            else
              ybuf[col_index(cur, S, j)] = acc;
            first_seg = false;
            cur = vk[q];
            acc = 0.0;
          }
          acc = fma(ak[q], x[q], acc);
        }
      }
    }
    const bool open_r = e < n_rec && (rec[e] & 3ull) != 3ull && (int32_t)(rec[e] >> rsh) == cur;
    if (first_seg && open_l)
      hpart[c * S + j] = acc;
    else if (open_r)
      tpart[c * S + j] = acc;
    else
      ybuf[col_index(cur, S, j)] = acc;
  }
}

// Slots past the last touched row's: the batch's padding keys (entries a
// node deletion skips, an undirected self-loop's second direction) own none,
// so the count read back after validation can exceed the slots written.
__global__ void k_seed_pad_tail(uint64_t *__restrict__ rec, const int32_t *__restrict__ rec_off,
                                const int32_t *__restrict__ seg, const Ctl *ctl, int32_t n_rec) {
  if (ctl->err) return;
  const int32_t nT = ctl->nT[0];
  const int64_t start = (int64_t)rec_off[nT] + seg[nT];
  for (int64_t i = start + blockIdx.x * blockDim.x + threadIdx.x; i < n_rec; i += (int64_t)gridDim.x * blockDim.x)
    rec[i] = SEED_PAD;
}

// One group per chunk whose last node continues into the next chunk and
// began in this one: that node's sum, chunk by chunk in order.
template <int S>
__global__ __launch_bounds__(256) void k_seed_fixup(const uint64_t *__restrict__ rec, int32_t n_rec, int rsh,
                                                    const double *__restrict__ hpart,
                                                    const double *__restrict__ tpart, double *__restrict__ ybuf,
                                                    const Ctl *ctl) {
  if (ctl->err) return;
  constexpr int G = RWR_WAVE / S;
  const int lane = threadIdx.x % RWR_WAVE, j = lane % S, g = lane / S;
  const int32_t nch = (n_rec + SEED_RED_CH - 1) / SEED_RED_CH;
  const int64_t ngroups = (int64_t)gridDim.x * (blockDim.x / RWR_WAVE) * G;
  auto node = [&](int32_t i) -> int64_t {  // -1 for a pad
    const uint64_t k = rec[i];
    return (k & 3ull) == 3ull ? -1 : (int64_t)(k >> rsh);
  };
  for (int64_t c = (int64_t)((blockIdx.x * blockDim.x + threadIdx.x) / RWR_WAVE) * G + g; c < nch; c += ngroups) {
    const int32_t b = (int32_t)c * SEED_RED_CH, e = min(n_rec, b + SEED_RED_CH);
    if (e >= n_rec) continue;
    const int64_t v = node(e - 1);
    if (v < 0 || node(e) != v) continue;                        // the last node ends here
    if (node(b) == v && b > 0 && node(b - 1) == v) continue;  // it began in an earlier chunk
    double s = tpart[c * S + j];
    for (int32_t cc = (int32_t)c + 1; cc < nch; ++cc) {
      s += hpart[(int64_t)cc * S + j];
      const int32_t ee = min(n_rec, (cc + 1) * SEED_RED_CH);
      if (ee >= n_rec || node(ee - 1) != v || node(ee) != v) break;
    }
    ybuf[col_index(v, S, j)] = s;
  }
}

// bits that hold every value in [0, v]
static int width_of(int64_t v) {
  int b = 1;
  while ((1ll << b) <= v) ++b;
  return b;
}

int seed_rec_shift(int32_t max_rows) { return 2 + width_of(std::max(1, max_rows)); }

int64_t seed_part_len(int64_t n_rec, int S) { return (n_rec + SEED_RED_CH - 1) / SEED_RED_CH * S; }

size_t seed_sort_temp_bytes(int64_t n_rec) {
  size_t a = 0;
  (void)hipcub::DeviceRadixSort::SortKeys((void *)nullptr, a, (uint64_t *)nullptr, (uint64_t *)nullptr,
                                          (int)std::min<int64_t>(n_rec, INT32_MAX), 0, 64);
  return a;
}

hipError_t launch_seed_sort_reduce(int S, uint64_t *rec, uint64_t *rec_alt, int32_t n_rec, int32_t max_rows,
                                   int32_t n_nodes, const int32_t *rec_off, const int32_t *seg,
                                   const int32_t *row, const int32_t *t_dold, const int32_t *t_dnew,
                                   const double *r, const double *rsub, uint64_t rmask, double c1, double *ybuf,
                                   double *hpart, double *tpart, void *temp, size_t temp_bytes, const Ctl *ctl,
                                   int grid, hipStream_t st) {
  if (n_rec <= 0) return hipSuccess;
  const int rsh = seed_rec_shift(max_rows);
  const int end_bit = rsh + width_of(std::max(1, n_nodes - 1));
  if (end_bit > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_seed_pad_tail, dim3(64), dim3(256), 0, st, rec, rec_off, seg, ctl, n_rec);
  size_t bytes = temp_bytes;
  hipError_t err = hipcub::DeviceRadixSort::SortKeys(temp, bytes, rec, rec_alt, n_rec, 0, end_bit, st);
  if (err != hipSuccess) return err;
  const uint64_t tmask = (1ull << (rsh - 2)) - 1;
#define RWR_RED_CASE(SS)                                                                                         \
  case SS:                                                                                                       \
    hipLaunchKernelGGL(k_seed_reduce<SS>, dim3(grid), dim3(256), 0, st, rec_alt, n_rec, rsh, tmask, row, t_dold, \
                       t_dnew, r, rsub, rmask, c1, ybuf, hpart, tpart, ctl);                                     \
    hipLaunchKernelGGL(k_seed_fixup<SS>, dim3(grid), dim3(256), 0, st, rec_alt, n_rec, rsh, hpart, tpart, ybuf,  \
                       ctl);                                                                                     \
    break;
  switch (S) {
    RWR_RED_CASE(1)
    RWR_RED_CASE(2)
    RWR_RED_CASE(4)
    RWR_RED_CASE(8)
    RWR_RED_CASE(16)
    RWR_RED_CASE(32)
    RWR_RED_CASE(64)
  }
#undef RWR_RED_CASE
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
  const int32_t n_del = ((e - b) - (d_new - d_old)) / 2;
  if (P.big && d_old > BIG_ROW && (n_del > 0 || move)) return;  // k_apply_big's row
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
  // a row that keeps every entry in place only appends
  const bool scan = move || n_del != 0;
  int32_t w = scan ? 0 : d_old;
  for (int32_t i0 = 0; scan && i0 < d_old; i0 += SEG_W * RWR_WAVE) {
    // SEG_W x 64 entries read before any is written: a kept entry moves to a
    // position at or below its own, which this or an earlier step has read
    int32_t v[SEG_W], p[SEG_W];
#pragma unroll
    for (int q = 0; q < SEG_W; ++q) {
      const int32_t i = i0 + q * RWR_WAVE + lane;
      v[q] = i < d_old ? adj[o + i] : -1;
    }
    seg_find_w(keys, b, e, u, v, b1, p, (d_old - i0 + RWR_WAVE - 1) / RWR_WAVE);
#pragma unroll
    for (int q = 0; q < SEG_W; ++q) {
      const bool keep = v[q] >= 0 && p[q] < 0;
      const uint64_t m = __ballot(keep);
      if (keep) adj[base + w + __popcll(m & lt_mask)] = v[q];
      w += __popcll(m);
    }
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

// ------------------------------------------------- rows above BIG_ROW
#define BIG_BLOCK 1024
#define BIG_WAVES (BIG_BLOCK / RWR_WAVE)

// exclusive prefix of a per-wavefront count over the workgroup's wavefronts
// (cnt: the counts in LDS), and the workgroup's total
__device__ __forceinline__ int32_t big_prefix(const int32_t *cnt, int wid, int32_t &total) {
  int32_t pre = 0, tot = 0;
  for (int ww = 0; ww < BIG_WAVES; ++ww) {
    pre += ww < wid ? cnt[ww] : 0;
    tot += cnt[ww];
  }
  total = tot;
  return pre;
}

// The batch check of listed rows, one workgroup per row.
__global__ __launch_bounds__(BIG_BLOCK) void k_validate_big(OrientPair P, int b1, Ctl *ctl) {
  __shared__ int32_t s_red[3][BIG_WAVES];
  if (ctl->err) return;
  const OrientArgs &q = P.o[0];
  const int tid = threadIdx.x, lane = tid % RWR_WAVE, wid = tid / RWR_WAVE;
  const int32_t nb = ctl->nbig_v;
  for (int32_t i = blockIdx.x; i < nb; i += gridDim.x) {
    const int32_t t = P.bigv[i];
    const int32_t u = q.row[t], b = q.seg[t], e = q.seg[t + 1];
    const int32_t d_old = q.g.len[u], o = q.g.off[u];
    int found = 0, exists = 0, dels = 0;
    for (int32_t k = b + tid; k < e; k += BIG_BLOCK) dels += (int)!(q.keys[k] & 1ull);
    for (int32_t i0 = 0; i0 < d_old; i0 += SEG_W * BIG_BLOCK) {
      int32_t v[SEG_W], p[SEG_W];
#pragma unroll
      for (int w = 0; w < SEG_W; ++w) {
        const int32_t k = i0 + w * BIG_BLOCK + tid;
        v[w] = k < d_old ? q.g.adj[o + k] : -1;
      }
      seg_find_w(q.keys, b, e, u, v, b1, p, (d_old - i0 + BIG_BLOCK - 1) / BIG_BLOCK);
#pragma unroll
      for (int w = 0; w < SEG_W; ++w)
        if (p[w] >= 0) {
          if (q.keys[p[w]] & 1ull)
            exists = 1;
          else
            ++found;
        }
    }
    found = wave_xor_sum(found, 1, RWR_WAVE);
    exists = wave_xor_sum(exists, 1, RWR_WAVE);
    dels = wave_xor_sum(dels, 1, RWR_WAVE);
    if (lane == 0) {
      s_red[0][wid] = found;
      s_red[1][wid] = exists;
      s_red[2][wid] = dels;
    }
    __syncthreads();
    if (tid == 0) {
      int F = 0, X = 0, D = 0;
      for (int ww = 0; ww < BIG_WAVES; ++ww) F += s_red[0][ww], X += s_red[1][ww], D += s_red[2][ww];
      if (X)
        set_error(ctl, ERR_EEXIST);
      else if (F != D)
        set_error(ctl, ERR_ENOENT);
    }
    __syncthreads();
  }
}

// The structural apply of listed rows, one workgroup per row: the kept
// entries compacted in order (in place, or into a fresh arena slot), then the
// inserted ones appended, as k_apply does with one wavefront.
__global__ __launch_bounds__(BIG_BLOCK) void k_apply_big(OrientPair P, int b1, Ctl *ctl) {
  __shared__ int32_t s_cnt[SEG_W][BIG_WAVES];
  __shared__ long long s_pos;
  if (ctl->err) return;
  const int tid = threadIdx.x, lane = tid % RWR_WAVE, wid = tid / RWR_WAVE;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (RWR_WAVE - lane));
  const int32_t nb = ctl->nbig_a;
  for (int32_t i = blockIdx.x; i < nb; i += gridDim.x) {
    const uint32_t ent = (uint32_t)P.biga[i];
    const int orient = (int)(ent >> 31);
    const int32_t t = (int32_t)(ent & 0x7fffffffu);
    const OrientArgs &q = P.o[orient];
    const int32_t u = q.row[t], b = q.seg[t], e = q.seg[t + 1];
    const int32_t d_old = q.t_dold[t], d_new = q.t_dnew[t];
    const int32_t o = q.g.off[u];
    int32_t ncap = q.g.cap[u];
    const bool move = d_new > ncap;
    if (move) ncap = grown_cap(d_new);
    if (tid == 0) {
      long long pos = o;
      if (move) {
        pos = (long long)atomicAdd((unsigned long long *)&ctl->tail[orient], (unsigned long long)ncap);
        // the host sizes the arena from the validated demand; never write past it
        if (pos + ncap > q.e_cap) {
          atomicCAS(&ctl->prop_err, 0, ERR_ENOMEM);
          pos = -1;
        }
      }
      s_pos = pos;
    }
    __syncthreads();
    const long long sp = s_pos;
    if (sp < 0) {
      __syncthreads();
      continue;
    }
    const int32_t base = (int32_t)sp;
    int32_t w = 0;
    for (int32_t i0 = 0; i0 < d_old; i0 += SEG_W * BIG_BLOCK) {
      int32_t v[SEG_W], p[SEG_W];
#pragma unroll
      for (int x = 0; x < SEG_W; ++x) {
        const int32_t k = i0 + x * BIG_BLOCK + tid;
        v[x] = k < d_old ? q.g.adj[o + k] : -1;
      }
      seg_find_w(q.keys, b, e, u, v, b1, p, (d_old - i0 + BIG_BLOCK - 1) / BIG_BLOCK);
      uint64_t m[SEG_W];
#pragma unroll
      for (int x = 0; x < SEG_W; ++x) {
        m[x] = __ballot(v[x] >= 0 && p[x] < 0);
        if (lane == 0) s_cnt[x][wid] = __popcll(m[x]);
      }
      // every read of this step is done before any write: a kept entry
      // moves to a position at or below its own
      __syncthreads();
#pragma unroll
      for (int x = 0; x < SEG_W; ++x) {
        int32_t tot;
        const int32_t pre = big_prefix(s_cnt[x], wid, tot);
        if ((m[x] >> lane) & 1ull) q.g.adj[base + w + pre + __popcll(m[x] & lt_mask)] = v[x];
        w += tot;
      }
      __syncthreads();
    }
    for (int32_t k0 = b; k0 < e; k0 += BIG_BLOCK) {
      const int32_t k = k0 + tid;
      const bool ins = k < e && (q.keys[k] & 1ull);
      const uint64_t mi = __ballot(ins);
      if (lane == 0) s_cnt[0][wid] = __popcll(mi);
      __syncthreads();
      int32_t tot;
      const int32_t pre = big_prefix(s_cnt[0], wid, tot);
      if (ins) q.g.adj[base + w + pre + __popcll(mi & lt_mask)] = key_col(q.keys[k], b1);
      w += tot;
      __syncthreads();
    }
    if (tid == 0) {
      q.g.len[u] = d_new;
      if (move) {
        q.g.off[u] = base;
        q.g.cap[u] = ncap;
      }
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
  for (int i = 0; i < 32; ++i) ctl->seed_recs[i] = 0;
  ctl->nbig_v = 0;
  ctl->nbig_a = 0;
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
  // the listed rows' count is on the device: a grid for many (idle workgroups return at once)
  if (P.big && P.o[0].check) hipLaunchKernelGGL(k_validate_big, dim3(1024), dim3(BIG_BLOCK), 0, st, P, b1, ctl);
}

template <int S>
static void offset_seed_s(const uint64_t *keys, const int32_t *seg, const int32_t *row, const int32_t *t_dold,
                          const int32_t *t_dnew, const int32_t *item_off, const DevGraphView &g, const double *r,
                          const double *rsub, double *ybuf, int32_t *stamp, Ctl *ctl, int b1, double c1,
                          int32_t max_rows, uint64_t *rec, const int32_t *rec_off, int rsh, uint64_t rmask,
                          int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_offset_seed<S>, dim3(grid), dim3(256), 0, st, keys, seg, row, t_dold, t_dnew, item_off, g.off,
                     g.adj, r, rsub, ybuf, stamp, ctl, b1, c1, max_rows, rec, rec_off, rsh, rmask);
}

hipError_t launch_offset_seed(int S, const uint64_t *keys, const int32_t *seg, const int32_t *row,
                              const int32_t *t_dold, const int32_t *t_dnew, const DevGraphView &g, const double *r,
                              const double *rsub, uint64_t rmask, double *ybuf, int32_t *stamp, Ctl *ctl, int b1,
                              double c1, int32_t max_rows, int32_t *items, int32_t *item_off, uint64_t *rec,
                              int32_t *dcnt, int32_t *rec_off, void *temp, size_t temp_bytes, int grid,
                              hipStream_t st) {
  if (max_rows <= 0) return hipSuccess;
  if (max_rows < SEED_SMALL) {
    hipLaunchKernelGGL(k_seed_items_small, dim3(1), dim3(1024), 0, st, t_dold, ctl, max_rows, item_off,
                       rec ? rec_off : nullptr);
  } else {
    hipLaunchKernelGGL(k_seed_items, dim3(std::min(4096, (max_rows + 256) / 256)), dim3(256), 0, st, t_dold, ctl,
                       max_rows, items, rec ? dcnt : nullptr);
    size_t bytes = temp_bytes;
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(temp, bytes, items, item_off, max_rows + 1, st);
    if (e != hipSuccess) return e;
    if (rec) {
      bytes = temp_bytes;
      e = hipcub::DeviceScan::ExclusiveSum(temp, bytes, dcnt, rec_off, max_rows + 1, st);
      if (e != hipSuccess) return e;
    }
  }
  const int rsh = seed_rec_shift(max_rows);
#define RWR_SEED_CASE(SS)                                                                                        \
  case SS:                                                                                                       \
    offset_seed_s<SS>(keys, seg, row, t_dold, t_dnew, item_off, g, r, rsub, ybuf, stamp, ctl, b1, c1, max_rows, \
                      rec, rec_off, rsh, rmask, grid, st);                                                       \
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

void launch_apply(const OrientPair &P, int norient, int b1, Ctl *ctl, int32_t max_rows, int32_t big_rows,
                  hipStream_t st) {
  if (max_rows <= 0) return;
  const int waves_per_block = 4;
  const int grid = (max_rows + waves_per_block - 1) / waves_per_block;
  hipLaunchKernelGGL(k_apply, dim3(grid, norient), dim3(waves_per_block * RWR_WAVE), 0, st, P, b1, ctl);
  if (P.big && big_rows > 0)
    hipLaunchKernelGGL(k_apply_big, dim3(std::min(big_rows, 1024)), dim3(BIG_BLOCK), 0, st, P, b1, ctl);
}
