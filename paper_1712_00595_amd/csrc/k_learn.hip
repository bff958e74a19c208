// Kernels of the learned warm start's network (layout in gnn.h).
//
// Dense per-row transforms run on the matrix cores: v_mfma_f32_16x16x32_bf16
// with bfloat16 operands (weights, and activations rounded when they enter a
// product) and float32 accumulation.  Aggregation along the region's edges,
// bias, ReLU, loss and the optimiser run in float32.  Every reduction over
// rows (weight gradients, loss) is split into per-workgroup partials that a
// second kernel adds in a fixed order, so results do not depend on timing.
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "gnn.h"

namespace gnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int GB = 256;  // workgroup size of every kernel here
constexpr int WAVE = 64;

Layout::Layout() {
  int64_t o = 0;
  W0 = o;
  o += FEAT * HID;
  b0 = o;
  o += HID;
  for (int l = 0; l < LAYERS; ++l) {
    Wp[l] = o;
    o += HID * MSG;
    Ws[l] = o;
    o += HID * HID;
    Wm[l] = o;
    o += MSG * HID;
    b[l] = o;
    o += HID;
  }
  wo = o;
  o += HID;
  bo = o;
  o += 1;
  total = o;
}
const Layout LAYOUT;

// the ten weight matrices that enter matrix-core products
struct MatTable {
  int64_t off[1 + 3 * LAYERS];
  int32_t K[1 + 3 * LAYERS], N[1 + 3 * LAYERS];
  int64_t fwd[1 + 3 * LAYERS], bwd[1 + 3 * LAYERS];
};
constexpr int NMAT = 1 + 3 * LAYERS;

static __host__ __device__ inline int pad32(int x) { return (x + 31) / 32 * 32; }

static MatTable mat_table() {
  MatTable t{};
  int64_t f = 0, b = 0;
  auto add = [&](int i, int64_t off, int K, int N) {
    t.off[i] = off;
    t.K[i] = K;
    t.N[i] = N;
    t.fwd[i] = f;
    t.bwd[i] = b;
    f += (int64_t)N * pad32(K);
    b += (int64_t)K * pad32(N);
  };
  add(0, LAYOUT.W0, FEAT, HID);
  for (int l = 0; l < LAYERS; ++l) {
    add(1 + 3 * l, LAYOUT.Wp[l], HID, MSG);
    add(2 + 3 * l, LAYOUT.Ws[l], HID, HID);
    add(3 + 3 * l, LAYOUT.Wm[l], MSG, HID);
  }
  return t;
}

// forward operand: Bt[n][pad32(K)] = W[k][n]; backward: B[k][pad32(N)] = W[k][n]
__global__ void k_prep_weights(const float *__restrict__ theta, MatTable t, __bf16 *__restrict__ fwd,
                               __bf16 *__restrict__ bwd) {
  const int i = blockIdx.y;
  const int K = t.K[i], N = t.N[i], KP = pad32(K), NP = pad32(N);
  const float *W = theta + t.off[i];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N * KP; e += gridDim.x * blockDim.x) {
    const int n = e / KP, k = e % KP;
    fwd[t.fwd[i] + e] = (__bf16)(k < K ? W[k * N + n] : 0.0f);
  }
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < K * NP; e += gridDim.x * blockDim.x) {
    const int k = e / NP, n = e % NP;
    bwd[t.bwd[i] + e] = (__bf16)(n < N ? W[k * N + n] : 0.0f);
  }
}

// ------------------------------------------------------------ products
// Y[M x N] = X1[M x K1] B1 (+ X2[M x K2] B2), one wavefront per 16 rows.
// Operand fragments of the 16x16x32 product: lane l holds row (l % 16) of
// the 16-row block and eight consecutive reduction indices 8 (l / 16) ..;
// the B fragment holds the same reduction indices of column (l % 16); the
// result holds rows 4 (l / 16) .. +3 of column (l % 16).
template <int K, int NT>
__device__ __forceinline__ void mma_rows(const float *__restrict__ X, const __bf16 *__restrict__ B, int64_t row,
                                         int64_t M, int g, int r, f32x4 (&acc)[NT]) {
  constexpr int KP = (K + 31) / 32 * 32;
#pragma unroll
  for (int ks = 0; ks < KP; ks += 32) {
    const int kb = ks + 8 * g;
    bf16x8 af;
    if (row < M && kb < K) {
      const float4 x0 = *reinterpret_cast<const float4 *>(X + row * K + kb);
      const float4 x1 = *reinterpret_cast<const float4 *>(X + row * K + kb + 4);
      af = bf16x8{(__bf16)x0.x, (__bf16)x0.y, (__bf16)x0.z, (__bf16)x0.w,
                  (__bf16)x1.x, (__bf16)x1.y, (__bf16)x1.z, (__bf16)x1.w};
    } else {
      af = bf16x8{};
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const bf16x8 bf = *reinterpret_cast<const bf16x8 *>(B + (int64_t)(t * 16 + r) * KP + kb);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf, acc[t], 0, 0, 0);
    }
  }
}

enum { EPI_NONE = 0, EPI_BIAS_RELU = 1, EPI_RELU_MASK = 2 };

template <int K1, int K2, int N, int EPI>
__global__ __launch_bounds__(GB) void k_gemm(int64_t M, const float *__restrict__ X1, const float *__restrict__ X2,
                                             const __bf16 *__restrict__ B1, const __bf16 *__restrict__ B2,
                                             const float *__restrict__ bias, const float *__restrict__ hmask,
                                             float *__restrict__ Y) {
  constexpr int NT = N / 16;
  const int lane = threadIdx.x % WAVE;
  const int r = lane % 16, g = lane / 16;
  const int64_t wave = ((int64_t)blockIdx.x * GB + threadIdx.x) / WAVE;
  const int64_t nwaves = (int64_t)gridDim.x * GB / WAVE;
  for (int64_t m0 = wave * 16; m0 < M; m0 += nwaves * 16) {
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    mma_rows<K1, NT>(X1, B1, m0 + r, M, g, r, acc);
    if constexpr (K2 > 0) mma_rows<K2, NT>(X2, B2, m0 + r, M, g, r, acc);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = t * 16 + r;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t row = m0 + 4 * g + i;
        if (row >= M) continue;
        float v = acc[t][i];
        if constexpr (EPI == EPI_BIAS_RELU) v = fmaxf(v + bias[col], 0.0f);
        if constexpr (EPI == EPI_RELU_MASK) v = hmask[row * N + col] > 0.0f ? v : 0.0f;
        Y[row * N + col] = v;
      }
    }
  }
}

// Partial weight gradient of one wavefront: G[k][n] = sum over its rows of
// X[m][k] D[m][n] (both rounded to bfloat16), on the matrix cores with the
// rows as the reduction index; part row = the wavefront's global index.  No
// LDS, so that many wavefronts stay resident.
template <int K, int N>
__global__ __launch_bounds__(GB) void k_wgrad(int64_t M, const float *__restrict__ X, const float *__restrict__ D,
                                              float *__restrict__ part) {
  constexpr int KT = K / 16, NT = N / 16;
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int r = lane % 16, g = lane / 16;
  f32x4 acc[KT][NT];
#pragma unroll
  for (int a = 0; a < KT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t wave = (int64_t)blockIdx.x * (GB / WAVE) + w;
  const int64_t nwaves = (int64_t)gridDim.x * (GB / WAVE);
  for (int64_t m0 = wave * 32; m0 < M; m0 += nwaves * 32) {
    bf16x8 af[KT], bf[NT];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t m = m0 + 8 * g + e;
      const bool ok = m < M;
#pragma unroll
      for (int a = 0; a < KT; ++a) af[a][e] = (__bf16)(ok ? X[m * K + a * 16 + r] : 0.0f);
#pragma unroll
      for (int b = 0; b < NT; ++b) bf[b][e] = (__bf16)(ok ? D[m * N + b * 16 + r] : 0.0f);
    }
#pragma unroll
    for (int a = 0; a < KT; ++a)
#pragma unroll
      for (int b = 0; b < NT; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bf[b], acc[a][b], 0, 0, 0);
  }
  float *__restrict__ dst = part + wave * (K * N);
#pragma unroll
  for (int a = 0; a < KT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) dst[(a * 16 + 4 * g + i) * N + b * 16 + r] = acc[a][b][i];
}

// Column sums over rows (per workgroup): MODE 0: sum A[m][n]; MODE 1: sum
// bf16(A[m][n]) * bf16(wv[m]).  Each thread owns one column.
template <int N, int MODE>
__global__ __launch_bounds__(GB) void k_colsum(int64_t M, const float *__restrict__ A, const float *__restrict__ wv,
                                               float *__restrict__ part) {
  constexpr int RPB = GB / N;  // row lanes per column
  __shared__ float red[GB];
  const int n = threadIdx.x % N, rl = threadIdx.x / N;
  float s = 0.0f;
  for (int64_t m = (int64_t)blockIdx.x * RPB + rl; m < M; m += (int64_t)gridDim.x * RPB) {
    if constexpr (MODE == 0) {
      s += A[m * N + n];
    } else {
      s += (float)(__bf16)A[m * N + n] * (float)(__bf16)wv[m];
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < N) {
    float t = 0.0f;
    for (int q = 0; q < RPB; ++q) t += red[q * N + threadIdx.x];
    part[(int64_t)blockIdx.x * N + threadIdx.x] = t;
  }
}

// out[i] = sum over b of part[b * count + i], in two fixed-order stages:
// group y of RED_GROUP consecutive partials is summed in order into
// tmp[y * count + i], then the group sums in order into out[i].
#define RED_GROUP 32
__global__ __launch_bounds__(GB) void k_reduce_stage(const float *__restrict__ part, int nb, int count,
                                                     float *__restrict__ out) {
  const int i = blockIdx.x * GB + threadIdx.x;
  if (i >= count) return;
  const int b0 = blockIdx.y * RED_GROUP, b1 = min(nb, b0 + RED_GROUP);
  float s = 0.0f;
  for (int b = b0; b < b1; ++b) s += part[(int64_t)b * count + i];
  out[(int64_t)blockIdx.y * count + i] = s;
}

static void reduce_part(const Net &n, const float *part, int nb, int count, float *out, hipStream_t st) {
  const int ng = (nb + RED_GROUP - 1) / RED_GROUP;
  const int gx = (count + GB - 1) / GB;
  if (ng == 1) {
    hipLaunchKernelGGL(k_reduce_stage, dim3(gx, 1), dim3(GB), 0, st, part, nb, count, out);
    return;
  }
  hipLaunchKernelGGL(k_reduce_stage, dim3(gx, ng), dim3(GB), 0, st, part, nb, count, n.part2);
  hipLaunchKernelGGL(k_reduce_stage, dim3(gx, 1), dim3(GB), 0, st, n.part2, ng, count, out);
}

// ------------------------------------------------------------ aggregation
// Work unit = (item, c) with c = 4 j + q over the 4 S float4 slices of a
// row (node i, column j, message entries 4q .. 4q+3).  Forward (IN = true):
//   Y[i*S+j][.] = sum over in-edges u -> i of dinv[u] M[u*S+j][.]
// backward (IN = false):
//   Y[i*S+j][.] = dinv[i] sum over out-edges i -> v of M[v*S+j][.]
// Four gathers in flight per thread.  A row of several chunks is zeroed
// beforehand and its chunks accumulate with float atomics; with `det` the
// first chunk's thread sums the whole row in edge order instead.
template <bool IN>
__global__ void k_agg(RegionView g, int S, const float *__restrict__ Min, float *__restrict__ Y, int det) {
  const int32_t *items = IN ? g.in_items : g.out_items;
  const int32_t n_items = IN ? g.n_in_items : g.n_out_items;
  const int32_t *item_row = IN ? g.in_item_row : g.out_item_row;
  const int32_t *roff = IN ? g.in_off : g.out_off;
  const int32_t *rlen = IN ? g.in_len : g.out_len;
  const int32_t *radj = IN ? g.in_adj : g.out_adj;
  const int per = 4 * S;
  const int64_t total = (int64_t)n_items * per;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int32_t it = (int32_t)(t / per);
    const int cidx = (int)(t % per);
    const int j = cidx / 4, q = cidx % 4;
    int32_t i;
    if (item_row) {
      i = item_row[it];
    } else {
      int32_t lo = 0, hi = g.nR - 1;
      while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (items[mid] <= it) lo = mid;
        else hi = mid - 1;
      }
      i = lo;
    }
    const int k = it - items[i];
    const int nch = items[i + 1] - items[i];
    if (det && k != 0) continue;
    const int o = roff[i], d = rlen[i];
    const int e0 = k * AGG_CHUNK, e1 = det ? d : min(d, e0 + AGG_CHUNK);
    float4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int e = e0; e < e1; e += 4) {
      int uu[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) uu[x] = e + x < e1 ? radj[o + e + x] : -1;
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        if (uu[x] < 0) continue;
        const float s = IN ? g.dinv[uu[x]] : 1.0f;
        const float4 m = *reinterpret_cast<const float4 *>(Min + ((int64_t)uu[x] * S + j) * MSG + 4 * q);
        acc.x += s * m.x;
        acc.y += s * m.y;
        acc.z += s * m.z;
        acc.w += s * m.w;
      }
    }
    if (!IN) {
      const float s = g.dinv[i];
      acc.x *= s;
      acc.y *= s;
      acc.z *= s;
      acc.w *= s;
    }
    float *dst = Y + ((int64_t)i * S + j) * MSG + 4 * q;
    if (nch == 1 || det) {
      *reinterpret_cast<float4 *>(dst) = acc;
    } else {
      atomicAdd(dst, acc.x);
      atomicAdd(dst + 1, acc.y);
      atomicAdd(dst + 2, acc.z);
      atomicAdd(dst + 3, acc.w);
    }
  }
}

// item_row[it] = the row whose chunk `it` is (items: nR + 1 chunk offsets)
__global__ void k_item_rows(const int32_t *__restrict__ items, int32_t nR, int32_t *__restrict__ item_row) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nR; i += gridDim.x * blockDim.x)
    for (int32_t it = items[i]; it < items[i + 1]; ++it) item_row[it] = i;
}

// zero the rows of several chunks (and rows without edges) before k_agg
template <bool IN>
__global__ void k_agg_zero(RegionView g, int S, float *__restrict__ Y) {
  const int32_t *items = IN ? g.in_items : g.out_items;
  const int64_t total = (int64_t)g.nR * S * MSG;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / ((int64_t)S * MSG));
    if (items[i + 1] - items[i] != 1) Y[e] = 0.0f;
  }
}

// ------------------------------------------------------------ output and loss
__device__ __forceinline__ float rb(float x) { return (float)(__bf16)x; }

// o[m] = sum_k bf16(h[m][k]) bf16(wo[k]) + bo
__global__ void k_out_fwd(int64_t M, const float *__restrict__ h, const float *__restrict__ theta, int64_t wo,
                          int64_t bo, float *__restrict__ o) {
  for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < M; m += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int k = 0; k < HID; k += 4) {
      const float4 x = *reinterpret_cast<const float4 *>(h + m * HID + k);
      s += rb(x.x) * rb(theta[wo + k]) + rb(x.y) * rb(theta[wo + k + 1]) + rb(x.z) * rb(theta[wo + k + 2]) +
           rb(x.w) * rb(theta[wo + k + 3]);
    }
    o[m] = s + theta[bo];
  }
}

// Huber loss per row (column j = m % S counts when active[j]); dL/do and
// per-workgroup loss partials (FP64)
__global__ __launch_bounds__(GB) void k_loss(int64_t M, int S, const float *__restrict__ o, const float *__restrict__ t,
                                             const int32_t *__restrict__ active, float inv_cols, float delta,
                                             float *__restrict__ dout, double *__restrict__ part) {
  __shared__ double red[GB];
  double s = 0.0;
  for (int64_t m = blockIdx.x * (int64_t)GB + threadIdx.x; m < M; m += (int64_t)gridDim.x * GB) {
    const bool act = active[m % S] != 0;
    const float e = o[m] - t[m];
    const float ae = fabsf(e);
    float val, gr;
    if (ae <= delta) {
      val = 0.5f * e * e / delta;
      gr = e / delta;
    } else {
      val = ae - 0.5f * delta;
      gr = e > 0.0f ? 1.0f : -1.0f;
    }
    dout[m] = act ? gr * inv_cols : 0.0f;
    if (act) s += (double)val;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = GB / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_loss_total(const double *__restrict__ part, int nb, double scale, double *__restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[b];
  *out = s * scale;
}

// dz3[m][k] = bf16(do[m]) bf16(wo[k]), kept where h3 > 0
__global__ void k_out_bwd(int64_t M, const float *__restrict__ dout, const float *__restrict__ theta, int64_t wo,
                          const float *__restrict__ h, float *__restrict__ dz) {
  const int64_t total = M * HID;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = e / HID;
    const int k = (int)(e % HID);
    dz[e] = h[e] > 0.0f ? rb(dout[m]) * rb(theta[wo + k]) : 0.0f;
  }
}

// ------------------------------------------------------------ optimiser
// mask (may be null): parameters whose entry is 0 are held (no step, moments
// untouched)
__global__ void k_adamw(int64_t n, float *__restrict__ theta, const float *__restrict__ g, float *__restrict__ m1,
                        float *__restrict__ m2, const float *__restrict__ mask, float lr, float wd, float c1,
                        float c2) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (mask && mask[i] == 0.0f) continue;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gi;
    const float b = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    const float mh = a / c1, vh = b / c2;
    theta[i] -= lr * (mh / (sqrtf(vh) + eps) + wd * theta[i]);
  }
}

// ------------------------------------------------------------ host driver
static int grid_for(int64_t work, int per_block, int cap = 4096) {
  const int64_t g = (work + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

void region_item_rows(const int32_t *items, int32_t nR, int32_t *item_row, hipStream_t st) {
  if (nR > 0) hipLaunchKernelGGL(k_item_rows, dim3(grid_for(nR, GB, 4096)), dim3(GB), 0, st, items, nR, item_row);
}

#define GNN_TRY(x)                   \
  do {                               \
    hipError_t e_ = (x);             \
    if (e_ != hipSuccess) return e_; \
  } while (0)

template <typename T>
static hipError_t dalloc(T **p, int64_t n) {
  return hipMalloc((void **)p, sizeof(T) * std::max<int64_t>(1, n));
}

hipError_t net_alloc(Net &n, int S, int64_t max_rows) {
  n.S = S;
  n.max_rows = max_rows;
  const int64_t P = LAYOUT.total;
  GNN_TRY(dalloc(&n.theta, P));
  GNN_TRY(dalloc(&n.grad, P));
  GNN_TRY(dalloc(&n.m1, P));
  GNN_TRY(dalloc(&n.m2, P));
  const MatTable t = mat_table();
  int64_t f = 0, b = 0;
  for (int i = 0; i < NMAT; ++i) {
    f += (int64_t)t.N[i] * pad32(t.K[i]);
    b += (int64_t)t.K[i] * pad32(t.N[i]);
  }
  GNN_TRY(dalloc(&n.wb.fwd, f));
  GNN_TRY(dalloc(&n.wb.bwd, b));
  GNN_TRY(dalloc(&n.F, max_rows * FEAT));
  for (int l = 0; l <= LAYERS; ++l) GNN_TRY(dalloc(&n.h[l], max_rows * HID));
  for (int l = 0; l < LAYERS; ++l) GNN_TRY(dalloc(&n.a[l], max_rows * MSG));
  GNN_TRY(dalloc(&n.m, max_rows * MSG));
  GNN_TRY(dalloc(&n.o, max_rows));
  GNN_TRY(dalloc(&n.t, max_rows));
  GNN_TRY(dalloc(&n.dh, max_rows * HID));
  GNN_TRY(dalloc(&n.dz, max_rows * HID));
  GNN_TRY(dalloc(&n.da, max_rows * MSG));
  GNN_TRY(dalloc(&n.dm, max_rows * MSG));
  GNN_TRY(dalloc(&n.dout, max_rows));
  n.part_cap = NET_PART_CAP;
  GNN_TRY(dalloc(&n.part, n.part_cap));
  GNN_TRY(dalloc(&n.part2, n.part_cap / RED_GROUP + HID * HID));
  GNN_TRY(dalloc(&n.loss_part, 4096));
  GNN_TRY(dalloc(&n.loss, 1));
  GNN_TRY(dalloc(&n.active, 64));
  return hipSuccess;
}

size_t net_view(Net &n, int S, int64_t max_rows, void *base, size_t bytes, int64_t part_cap) {
  n = Net{};
  n.S = S;
  n.max_rows = max_rows;
  char *p = static_cast<char *>(base);
  size_t used = 0;
  bool fit = true;
  auto take = [&](auto **dst, int64_t count) {
    using T = std::remove_reference_t<decltype(**dst)>;
    const size_t b = ((size_t)count * sizeof(T) + 255) / 256 * 256;
    if (!p) {  // size query
      *dst = nullptr;
      used += b;
      return;
    }
    if (used + b > bytes) {
      fit = false;
      *dst = nullptr;
      return;
    }
    *dst = reinterpret_cast<T *>(p + used);
    used += b;
  };
  const int64_t P = LAYOUT.total;
  take(&n.theta, P);
  take(&n.grad, P);
  take(&n.m1, P);
  take(&n.m2, P);
  const MatTable t = mat_table();
  int64_t f = 0, b = 0;
  for (int i = 0; i < NMAT; ++i) {
    f += (int64_t)t.N[i] * pad32(t.K[i]);
    b += (int64_t)t.K[i] * pad32(t.N[i]);
  }
  take(&n.wb.fwd, f);
  take(&n.wb.bwd, b);
  take(&n.F, max_rows * FEAT);
  for (int l = 0; l <= LAYERS; ++l) take(&n.h[l], max_rows * HID);
  for (int l = 0; l < LAYERS; ++l) take(&n.a[l], max_rows * MSG);
  take(&n.m, max_rows * MSG);
  take(&n.o, max_rows);
  take(&n.t, max_rows);
  take(&n.dh, max_rows * HID);
  take(&n.dz, max_rows * HID);
  take(&n.da, max_rows * MSG);
  take(&n.dm, max_rows * MSG);
  take(&n.dout, max_rows);
  // weight-gradient partials: by default one block of HID x HID per 128
  // rows (the same partition as an allocated network uses for these rows)
  n.part_cap = part_cap > 0 ? part_cap : std::max<int64_t>(1, (max_rows + 127) / 128) * HID * HID;
  take(&n.part, n.part_cap);
  take(&n.part2, n.part_cap / RED_GROUP + HID * HID);
  take(&n.loss_part, 4096);
  take(&n.loss, 1);
  take(&n.active, 64);
  if (!fit) {
    n = Net{};
    return 0;
  }
  if (!p) n = Net{};
  return used;
}

void net_free(Net &n) {
  void *ps[] = {n.theta, n.grad, n.m1, n.m2, n.wb.fwd, n.wb.bwd, n.F, n.m, n.o, n.t, n.dh, n.dz, n.da, n.dm,
                n.dout, n.part, n.part2, n.loss_part, n.loss, n.active, n.mask};
  for (void *p : ps)
    if (p) (void)hipFree(p);
  for (int l = 0; l <= LAYERS; ++l)
    if (n.h[l]) (void)hipFree(n.h[l]);
  for (int l = 0; l < LAYERS; ++l)
    if (n.a[l]) (void)hipFree(n.a[l]);
  n = Net{};
}

void net_prepare_weights(Net &n, hipStream_t st) {
  const MatTable t = mat_table();
  hipLaunchKernelGGL(k_prep_weights, dim3(8, NMAT), dim3(GB), 0, st, n.theta, t, n.wb.fwd, n.wb.bwd);
}

hipError_t net_set_params(Net &n, const float *host, hipStream_t st) {
  const int64_t P = LAYOUT.total;
  GNN_TRY(hipMemcpyAsync(n.theta, host, sizeof(float) * P, hipMemcpyHostToDevice, st));
  GNN_TRY(hipMemsetAsync(n.m1, 0, sizeof(float) * P, st));
  GNN_TRY(hipMemsetAsync(n.m2, 0, sizeof(float) * P, st));
  n.step = 0;
  net_prepare_weights(n, st);
  return hipStreamSynchronize(st);
}

hipError_t net_get_params(const Net &n, float *host, hipStream_t st) {
  GNN_TRY(hipMemcpyAsync(host, n.theta, sizeof(float) * LAYOUT.total, hipMemcpyDeviceToHost, st));
  return hipStreamSynchronize(st);
}

static const __bf16 *fwd_w(const Net &n, int i) { return n.wb.fwd + mat_table().fwd[i]; }
static const __bf16 *bwd_w(const Net &n, int i) { return n.wb.bwd + mat_table().bwd[i]; }

static int gemm_grid(int64_t rows) { return grid_for((rows + 15) / 16, GB / WAVE, 8192); }

template <bool IN>
static void agg(const RegionView &g, int S, int64_t rows, const float *Min, float *Y, int det, hipStream_t st) {
  hipLaunchKernelGGL(k_agg_zero<IN>, dim3(grid_for(rows * MSG, GB)), dim3(GB), 0, st, g, S, Y);
  const int64_t work = (int64_t)(IN ? g.n_in_items : g.n_out_items) * 4 * S;
  if (work > 0)
    hipLaunchKernelGGL(k_agg<IN>, dim3(grid_for(work, GB, 8192)), dim3(GB), 0, st, g, S, Min, Y, det);
}

void net_forward(Net &n, const RegionView &g, int64_t rows, hipStream_t st) {
  const float *th = n.theta;
  const int gg = gemm_grid(rows);
  hipLaunchKernelGGL((k_gemm<FEAT, 0, HID, EPI_BIAS_RELU>), dim3(gg), dim3(GB), 0, st, rows, n.F, nullptr,
                     fwd_w(n, 0), nullptr, th + LAYOUT.b0, nullptr, n.h[0]);
  for (int l = 0; l < LAYERS; ++l) {
    hipLaunchKernelGGL((k_gemm<HID, 0, MSG, EPI_NONE>), dim3(gg), dim3(GB), 0, st, rows, n.h[l], nullptr,
                       fwd_w(n, 1 + 3 * l), nullptr, nullptr, nullptr, n.m);
    agg<true>(g, n.S, rows, n.m, n.a[l], n.det, st);
    hipLaunchKernelGGL((k_gemm<HID, MSG, HID, EPI_BIAS_RELU>), dim3(gg), dim3(GB), 0, st, rows, n.h[l], n.a[l],
                       fwd_w(n, 2 + 3 * l), fwd_w(n, 3 + 3 * l), th + LAYOUT.b[l], nullptr, n.h[l + 1]);
  }
  hipLaunchKernelGGL(k_out_fwd, dim3(grid_for(rows, GB)), dim3(GB), 0, st, rows, n.h[LAYERS], th, LAYOUT.wo,
                     LAYOUT.bo, n.o);
}

void net_loss(Net &n, int64_t rows, int n_active, hipStream_t st) {
  const int nb = grid_for(rows, GB, 4096);
  const float inv = 1.0f / (float)std::max(1, n_active);
  hipLaunchKernelGGL(k_loss, dim3(nb), dim3(GB), 0, st, rows, n.S, n.o, n.t, n.active, inv, 1e-3f, n.dout,
                     n.loss_part);
  hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(64), 0, st, n.loss_part, nb, (double)inv, n.loss);
}

template <int K, int N>
static void wgrad(Net &n, int64_t rows, const float *X, const float *D, float *out, hipStream_t st) {
  // one partial per wavefront, GB / WAVE wavefronts per workgroup
  constexpr int WPB = GB / WAVE;
  const int64_t waves = std::min<int64_t>(std::max<int64_t>(1, (rows + 127) / 128), n.part_cap / (K * N));
  const int nb = (int)std::max<int64_t>(1, waves / WPB);
  hipLaunchKernelGGL((k_wgrad<K, N>), dim3(nb), dim3(GB), 0, st, rows, X, D, n.part);
  reduce_part(n, n.part, nb * WPB, K * N, out, st);
}

template <int N, int MODE>
static void colsum(Net &n, int64_t rows, const float *A, const float *wv, float *out, hipStream_t st) {
  const int nb = (int)std::min<int64_t>(std::max<int64_t>(1, (rows + 255) / 256), 1024);
  hipLaunchKernelGGL((k_colsum<N, MODE>), dim3(nb), dim3(GB), 0, st, rows, A, wv, n.part);
  reduce_part(n, n.part, nb, N, out, st);
}

void net_backward(Net &n, const RegionView &g, int64_t rows, hipStream_t st) {
  float *G = n.grad;
  const float *th = n.theta;
  const int gg = gemm_grid(rows);
  // output layer
  colsum<HID, 1>(n, rows, n.h[LAYERS], n.dout, G + LAYOUT.wo, st);
  colsum<1, 0>(n, rows, n.dout, nullptr, G + LAYOUT.bo, st);
  hipLaunchKernelGGL(k_out_bwd, dim3(grid_for(rows * HID, GB)), dim3(GB), 0, st, rows, n.dout, th, LAYOUT.wo,
                     n.h[LAYERS], n.dz);
  for (int l = LAYERS - 1; l >= 0; --l) {
    // n.dz = dL/dz of layer l+1 (ReLU applied)
    colsum<HID, 0>(n, rows, n.dz, nullptr, G + LAYOUT.b[l], st);
    wgrad<HID, HID>(n, rows, n.h[l], n.dz, G + LAYOUT.Ws[l], st);
    wgrad<MSG, HID>(n, rows, n.a[l], n.dz, G + LAYOUT.Wm[l], st);
    // da = dz Wm^T ; dm = aggregation transpose of da
    hipLaunchKernelGGL((k_gemm<HID, 0, MSG, EPI_NONE>), dim3(gg), dim3(GB), 0, st, rows, n.dz, nullptr,
                       bwd_w(n, 3 + 3 * l), nullptr, nullptr, nullptr, n.da);
    agg<false>(g, n.S, rows, n.da, n.dm, n.det, st);
    wgrad<HID, MSG>(n, rows, n.h[l], n.dm, G + LAYOUT.Wp[l], st);
    // dz of layer l = (dz Ws^T + dm Wp^T) masked by h_l > 0
    hipLaunchKernelGGL((k_gemm<HID, MSG, HID, EPI_RELU_MASK>), dim3(gg), dim3(GB), 0, st, rows, n.dz, n.dm,
                       bwd_w(n, 2 + 3 * l), bwd_w(n, 1 + 3 * l), nullptr, n.h[l], n.dh);
    std::swap(n.dz, n.dh);
  }
  colsum<HID, 0>(n, rows, n.dz, nullptr, G + LAYOUT.b0, st);
  wgrad<FEAT, HID>(n, rows, n.F, n.dz, G + LAYOUT.W0, st);
}

void net_adamw(Net &n, hipStream_t st) {
  ++n.step;
  const float c1 = 1.0f - powf(0.9f, (float)n.step);
  const float c2 = 1.0f - powf(0.999f, (float)n.step);
  // linear warm-up of the step size over the first `warmup` steps
  const float lr = n.warmup > 0 && n.step < n.warmup ? n.lr * (float)n.step / (float)n.warmup : n.lr;
  hipLaunchKernelGGL(k_adamw, dim3(grid_for(LAYOUT.total, GB)), dim3(GB), 0, st, LAYOUT.total, n.theta, n.grad,
                     n.m1, n.m2, n.mask, lr, n.wd, c1, c2);
  net_prepare_weights(n, st);
}

hipError_t net_set_mask(Net &n, const float *host, hipStream_t st) {
  if (!host) {
    if (n.mask) (void)hipFree(n.mask);
    n.mask = nullptr;
    return hipSuccess;
  }
  if (!n.mask) GNN_TRY(dalloc(&n.mask, LAYOUT.total));
  GNN_TRY(hipMemcpyAsync(n.mask, host, sizeof(float) * LAYOUT.total, hipMemcpyHostToDevice, st));
  return hipStreamSynchronize(st);
}

}  // namespace gnn
