// Construction and maintenance of the slack adjacency structure on the
// device: build from an edge list (radix sort of (row, col) keys, per-row
// capacity with slack, scatter), relayout when the relocation arena fills,
// export to an edge list, and the heavy-row flags of the dense pull.
#include <hipcub/hipcub.hpp>

#include "rwr_common.h"
#include "rwr_kernels.h"

__global__ void k_fill_i32(int32_t *p, int64_t count, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_zero_u32(uint32_t *p, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

static int fill_grid(int64_t count) { return (int)std::max<int64_t>(1, std::min<int64_t>((count + 255) / 256, 8192)); }

void launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(count)), dim3(256), 0, st, p, count, v);
}
// byte count must be a multiple of 4 (all buffers here are)
void launch_zero_bytes(void *p, size_t bytes, hipStream_t st) {
  const int64_t words = (int64_t)(bytes / 4);
  if (words > 0) hipLaunchKernelGGL(k_zero_u32, dim3(fill_grid(words)), dim3(256), 0, st, (uint32_t *)p, words);
}

// ------------------------------------------------------------------ build
__global__ void k_edge_keys(const int32_t *__restrict__ rows, const int32_t *__restrict__ cols, int64_t m, int32_t n,
                            uint64_t *__restrict__ keys, Ctl *ctl) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = rows[i], c = cols[i];
    if (r < 0 || r >= n || c < 0 || c >= n) {
      set_error(ctl, ERR_EINVAL);
      keys[i] = 0;
    } else {
      keys[i] = ((uint64_t)r << 32) | (uint32_t)c;
    }
  }
}

// row lengths from the sorted keys; a repeated key is a multi-edge (EINVAL)
__global__ void k_count_rows(const uint64_t *__restrict__ keys, int64_t m, int32_t *__restrict__ len, Ctl *ctl) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[i];
    if (i > 0 && keys[i - 1] == k) set_error(ctl, ERR_EINVAL);
    atomicAdd(&len[(int32_t)(k >> 32)], 1);
  }
}

// row capacity with slack: len + max(2, len/8)
__global__ void k_caps(const int32_t *__restrict__ len, int32_t n, int32_t *__restrict__ cap) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const int32_t d = len[v];
    cap[v] = d + max(2, d >> 3);
  }
}

__global__ void k_scatter(const uint64_t *__restrict__ keys, int64_t m, const int32_t *__restrict__ off,
                          const int32_t *__restrict__ sstart, int32_t *__restrict__ adj) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[i];
    const int32_t r = (int32_t)(k >> 32);
    adj[off[r] + (int32_t)(i - sstart[r])] = (int32_t)(uint32_t)(k & 0xffffffffull);
  }
}

size_t build_temp_bytes(int64_t m, int32_t n) {
  size_t a = 0, b = 0;
  (void)hipcub::DeviceRadixSort::SortKeys((void *)nullptr, a, (uint64_t *)nullptr, (uint64_t *)nullptr, (int)m, 0, 64);
  (void)hipcub::DeviceScan::ExclusiveSum((void *)nullptr, b, (int32_t *)nullptr, (int32_t *)nullptr, n);
  return std::max(a, b);
}

// Phase 1 of a build: sort keys, lengths, capacities, offsets.  Returns the
// number of adjacency slots used in *used (host value, after a sync).
hipError_t build_phase1(const int32_t *rows, const int32_t *cols, int64_t m, int32_t n, DevGraphView g, void *temp,
                        size_t temp_bytes, uint64_t *keys, uint64_t *keys_alt, int32_t *sstart, Ctl *ctl,
                        int64_t *used, hipStream_t st) {
  hipError_t err;
  if (m > 0) {
    hipLaunchKernelGGL(k_edge_keys, dim3(fill_grid(m)), dim3(256), 0, st, rows, cols, m, n, keys, ctl);
    int end_bit = 32;
    while ((1ll << (end_bit - 32)) < n) ++end_bit;
    size_t bytes = temp_bytes;
    err = hipcub::DeviceRadixSort::SortKeys(temp, bytes, keys, keys_alt, (int)m, 0, end_bit, st);
    if (err != hipSuccess) return err;
    err = hipMemcpyAsync(keys, keys_alt, sizeof(uint64_t) * (size_t)m, hipMemcpyDeviceToDevice, st);
    if (err != hipSuccess) return err;
  }
  launch_fill_i32(g.len, n, 0, st);
  if (m > 0) hipLaunchKernelGGL(k_count_rows, dim3(fill_grid(m)), dim3(256), 0, st, keys, m, g.len, ctl);
  hipLaunchKernelGGL(k_caps, dim3(fill_grid(n)), dim3(256), 0, st, g.len, n, g.cap);
  size_t bytes = temp_bytes;
  err = hipcub::DeviceScan::ExclusiveSum(temp, bytes, g.cap, g.off, n, st);
  if (err != hipSuccess) return err;
  bytes = temp_bytes;
  err = hipcub::DeviceScan::ExclusiveSum(temp, bytes, g.len, sstart, n, st);
  if (err != hipSuccess) return err;
  int32_t last_off = 0, last_cap = 0;
  err = hipMemcpyAsync(&last_off, g.off + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (err != hipSuccess) return err;
  err = hipMemcpyAsync(&last_cap, g.cap + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (err != hipSuccess) return err;
  err = hipStreamSynchronize(st);
  if (err != hipSuccess) return err;
  *used = (int64_t)last_off + last_cap;
  return hipSuccess;
}

void build_phase2(const uint64_t *keys, int64_t m, DevGraphView g, const int32_t *sstart, hipStream_t st) {
  if (m > 0) hipLaunchKernelGGL(k_scatter, dim3(fill_grid(m)), dim3(256), 0, st, keys, m, g.off, sstart, g.adj);
}

// ------------------------------------------------------------------ relayout
// one wavefront per row copies its entries to the new layout
__global__ void k_copy_rows(const int32_t *__restrict__ off, const int32_t *__restrict__ len,
                            const int32_t *__restrict__ adj, const int32_t *__restrict__ new_off,
                            int32_t *__restrict__ new_adj, int32_t n) {
  const int lane = threadIdx.x % RWR_WAVE;
  const int64_t w0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / RWR_WAVE;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / RWR_WAVE;
  for (int64_t v = w0; v < n; v += nw) {
    const int32_t o = off[v], d = len[v], no = new_off[v];
    for (int32_t e = lane; e < d; e += RWR_WAVE) new_adj[no + e] = adj[o + e];
  }
}

// new capacities (k_caps) and offsets must already be in new_cap / new_off
void launch_copy_rows(const DevGraphView &g, const int32_t *new_off, int32_t *new_adj, int32_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_rows, dim3(fill_grid((int64_t)n * RWR_WAVE)), dim3(256), 0, st, g.off, g.len, g.adj,
                     new_off, new_adj, n);
}

hipError_t relayout_offsets(const int32_t *len, int32_t n, int32_t *new_cap, int32_t *new_off, void *temp,
                            size_t temp_bytes, int64_t *used, hipStream_t st) {
  hipLaunchKernelGGL(k_caps, dim3(fill_grid(n)), dim3(256), 0, st, len, n, new_cap);
  size_t bytes = temp_bytes;
  hipError_t err = hipcub::DeviceScan::ExclusiveSum(temp, bytes, new_cap, new_off, n, st);
  if (err != hipSuccess) return err;
  int32_t last_off = 0, last_cap = 0;
  err = hipMemcpyAsync(&last_off, new_off + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (err != hipSuccess) return err;
  err = hipMemcpyAsync(&last_cap, new_cap + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (err != hipSuccess) return err;
  err = hipStreamSynchronize(st);
  *used = (int64_t)last_off + last_cap;
  return err;
}

// ------------------------------------------------------------------ export
// external ids via inv (internal -> external)
__global__ void k_export(const int32_t *__restrict__ off, const int32_t *__restrict__ len,
                         const int32_t *__restrict__ adj, const int32_t *__restrict__ pos, int32_t n,
                         const int32_t *__restrict__ inv, int32_t *__restrict__ out_src,
                         int32_t *__restrict__ out_dst) {
  const int lane = threadIdx.x % RWR_WAVE;
  const int64_t w0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / RWR_WAVE;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / RWR_WAVE;
  for (int64_t v = w0; v < n; v += nw) {
    const int32_t o = off[v], d = len[v], p = pos[v];
    const int32_t ev = inv[v];
    for (int32_t e = lane; e < d; e += RWR_WAVE) {
      out_src[p + e] = ev;
      out_dst[p + e] = inv[adj[o + e]];
    }
  }
}

hipError_t export_rows(const DevGraphView &g, int32_t n, const int32_t *inv, int32_t *out_src, int32_t *out_dst,
                       int32_t *pos, void *temp, size_t temp_bytes, hipStream_t st) {
  size_t bytes = temp_bytes;
  hipError_t err = hipcub::DeviceScan::ExclusiveSum(temp, bytes, g.len, pos, n, st);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_export, dim3(fill_grid((int64_t)n * RWR_WAVE)), dim3(256), 0, st, g.off, g.len, g.adj, pos, n,
                     inv, out_src, out_dst);
  return hipSuccess;
}

// ------------------------------------------------------------------ heavy rows
// flags[v] = len[v] > limit; flagged ids appended to sel (count in sel_count)
__global__ void k_mark_heavy(const int32_t *__restrict__ len, int32_t n, int32_t limit, uint8_t *__restrict__ flags,
                             int32_t *__restrict__ sel, int32_t *__restrict__ sel_count) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const bool h = len[v] > limit;
    flags[v] = h ? 1 : 0;
    if (h) sel[atomicAdd(sel_count, 1)] = v;
  }
}

void launch_mark_heavy(const int32_t *len, int32_t n, int32_t limit, uint8_t *flags, int32_t *sel,
                       int32_t *sel_count, hipStream_t st) {
  hipLaunchKernelGGL(k_mark_heavy, dim3(fill_grid(n)), dim3(256), 0, st, len, n, limit, flags, sel, sel_count);
}

__global__ void k_gather_i32(const int32_t *__restrict__ src, const int32_t *__restrict__ idx, int32_t count,
                             int32_t *__restrict__ out) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) out[i] = src[idx[i]];
}

void launch_gather_i32(const int32_t *src, const int32_t *idx, int32_t count, int32_t *out, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_gather_i32, dim3(fill_grid(count)), dim3(256), 0, st, src, idx, count, out);
}

// ------------------------------------------------------------------ relabel
// Internal vertex order: descending out-degree (ties by id), so that the
// entries gathered most often during a sweep are contiguous and stay in L2.
__global__ void k_out_degree(const int32_t *__restrict__ src, int64_t m, int32_t *__restrict__ deg) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&deg[src[i]], 1);
}

__global__ void k_degree_keys(const int32_t *__restrict__ deg, int32_t n, uint64_t *__restrict__ keys) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    keys[v] = ((uint64_t)(uint32_t)(INT32_MAX - deg[v]) << 32) | (uint32_t)v;
}

__global__ void k_perm_from_keys(const uint64_t *__restrict__ keys, int32_t n, int32_t *__restrict__ perm,
                                 int32_t *__restrict__ inv) {
  for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)(keys[r] & 0xffffffffull);
    perm[v] = r;
    inv[r] = v;
  }
}

__global__ void k_identity(int32_t *__restrict__ a, int32_t *__restrict__ b, int32_t from, int32_t to) {
  for (int32_t v = from + blockIdx.x * blockDim.x + threadIdx.x; v < to; v += gridDim.x * blockDim.x) {
    a[v] = v;
    b[v] = v;
  }
}

// out[i] = perm[in[i]] for ids in range; ids out of range pass through (the
// builder rejects them afterwards)
__global__ void k_map_ids(const int32_t *__restrict__ in, int64_t m, int32_t n, const int32_t *__restrict__ perm,
                          int32_t *__restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = in[i];
    out[i] = (v >= 0 && v < n) ? perm[v] : v;
  }
}

// perm/inv for n nodes ordered by out-degree; [n, n_cap) identity
hipError_t build_relabel(const int32_t *src, int64_t m, int32_t n, int32_t n_cap, int32_t *perm, int32_t *inv,
                         int32_t *deg_tmp, uint64_t *keys, uint64_t *keys_alt, void *temp, size_t temp_bytes,
                         hipStream_t st) {
  launch_fill_i32(deg_tmp, n, 0, st);
  if (m > 0) hipLaunchKernelGGL(k_out_degree, dim3(fill_grid(m)), dim3(256), 0, st, src, m, deg_tmp);
  hipLaunchKernelGGL(k_degree_keys, dim3(fill_grid(n)), dim3(256), 0, st, deg_tmp, n, keys);
  size_t bytes = temp_bytes;
  hipError_t err = hipcub::DeviceRadixSort::SortKeys(temp, bytes, keys, keys_alt, n, 0, 64, st);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_perm_from_keys, dim3(fill_grid(n)), dim3(256), 0, st, keys_alt, n, perm, inv);
  if (n_cap > n) hipLaunchKernelGGL(k_identity, dim3(fill_grid(n_cap - n)), dim3(256), 0, st, perm, inv, n, n_cap);
  return hipSuccess;
}

void launch_identity(int32_t *perm, int32_t *inv, int32_t from, int32_t to, hipStream_t st) {
  if (to > from) hipLaunchKernelGGL(k_identity, dim3(fill_grid(to - from)), dim3(256), 0, st, perm, inv, from, to);
}

void launch_map_ids(const int32_t *in, int64_t m, int32_t n, const int32_t *perm, int32_t *out, hipStream_t st) {
  if (m > 0) hipLaunchKernelGGL(k_map_ids, dim3(fill_grid(m)), dim3(256), 0, st, in, m, n, perm, out);
}
