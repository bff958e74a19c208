// Device network of the learned warm start: parameter layout, buffers and
// the host-side driver of its kernels (k_learn.hip).
//
// The network predicts the offset result of Section 3.1 on a region around
// the offset seed; the update then propagates only the exact residual of the
// prediction (q_offset - (I - (1-c) B~^T) xhat), so the scores stay those of
// Algorithm 1.  Rows of every activation matrix are (node, column) pairs in
// node-major order, row = local_node * S + column.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace gnn {

constexpr int FEAT = 16;
constexpr int HID = 64;
constexpr int MSG = 16;
constexpr int LAYERS = 3;
constexpr int AGG_CHUNK = 128;  // edges per aggregation work item

// parameter vector layout (float32), in this order:
//   W0[FEAT x HID] b0[HID]  { Wp[HID x MSG] Ws[HID x HID] Wm[MSG x HID] b[HID] } x LAYERS  wo[HID] bo[1]
struct Layout {
  int64_t W0, b0, Wp[LAYERS], Ws[LAYERS], Wm[LAYERS], b[LAYERS], wo, bo, total;
  Layout();
};
extern const Layout LAYOUT;

// bfloat16 copies of the weight matrices in the two operand layouts of the
// matrix-core products: forward (W^T, K padded to 32) and backward (W, N
// padded to 32)
struct WeightsBf16 {
  __bf16 *fwd = nullptr;
  __bf16 *bwd = nullptr;
  int64_t fwd_off[1 + 3 * LAYERS + 1];
  int64_t bwd_off[1 + 3 * LAYERS + 1];
  int64_t total = 0;
};

// Region graph view for aggregation: rows of the region's nodes in some
// adjacency (off/len/adj over ids of that adjacency); loc maps an id of the
// adjacency to its local index plus one (0: not in the region), or is NULL
// when the ids are already local.  nodes[i] is the adjacency id of local
// node i (NULL: identity).
struct RegionView {
  const int32_t *in_off, *in_len, *in_adj;     // in-rows (forward aggregation)
  const int32_t *out_off, *out_len, *out_adj;  // out-rows (backward aggregation)
  // work items: rows cut into AGG_CHUNK-edge chunks; *_items[i] = first item
  // of local row i (exclusive prefix of the chunk counts, nR + 1 entries),
  // n_*_items the total.  Rows of one chunk are written, rows of several
  // chunks accumulated.
  const int32_t *in_items, *out_items;
  int32_t n_in_items, n_out_items;
  // row of each item (n_*_items entries; null: found by binary search)
  const int32_t *in_item_row, *out_item_row;
  const int32_t *loc;
  const int32_t *nodes;
  const float *dinv;  // 1/d_out of each local node (0 for dead ends)
  int32_t nR;
};

struct Net {
  int S = 1;
  int64_t max_rows = 0;  // capacity in (node, column) rows
  // parameters, gradients, AdamW moments (float32) and bf16 copies
  float *theta = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
  WeightsBf16 wb;
  int64_t step = 0;
  float lr = 1e-3f, wd = 1e-4f;
  int64_t warmup = 0;      // steps of linear step-size warm-up
  float *mask = nullptr;   // trainable parameters (1) and held ones (0); null: all train
  int det = 0;             // 1: each aggregation row summed by one thread in edge order
  // activations
  float *F = nullptr;                 // rows x FEAT
  float *h[LAYERS + 1] = {};          // rows x HID
  float *a[LAYERS] = {};              // rows x MSG
  float *m = nullptr;                 // rows x MSG
  float *o = nullptr, *t = nullptr;   // rows
  float *dh = nullptr, *dz = nullptr; // rows x HID
  float *da = nullptr, *dm = nullptr; // rows x MSG
  float *dout = nullptr;              // rows
  float *part = nullptr;              // partial sums of weight gradients
  int64_t part_cap = 0;
  float *part2 = nullptr;             // first-stage sums of those (part_cap / 32 + HID * HID)
  double *loss_part = nullptr;        // per-workgroup loss partials
  double *loss = nullptr;             // device scalar
  int32_t *active = nullptr;          // per column: 1 when it counts in the loss
};

hipError_t net_alloc(Net &n, int S, int64_t max_rows);
// item_row[it] = row of chunk it, from the chunk offsets items[0..nR]
void region_item_rows(const int32_t *items, int32_t nR, int32_t *item_row, hipStream_t st);
void net_free(Net &n);
// Lay the buffers of a network for up to max_rows rows over caller memory
// (device address base, `bytes` available) instead of allocating them.
// Returns the bytes taken, or 0 (and an empty Net) when they do not fit;
// base null: the bytes it would take (n left empty).  part_cap: floats of
// weight-gradient partials (0: one HID x HID block per 128 rows).  Its
// mask is the caller's to set.  Such a Net must not be passed to net_free or
// net_set_mask.
size_t net_view(Net &n, int S, int64_t max_rows, void *base, size_t bytes, int64_t part_cap = 0);
// weight-gradient partials of an allocated network (floats)
constexpr int64_t NET_PART_CAP = 4096 * HID * HID;
// copy host parameters (float32, LAYOUT.total) and reset the optimiser
hipError_t net_set_params(Net &n, const float *host, hipStream_t st);
hipError_t net_get_params(const Net &n, float *host, hipStream_t st);
void net_prepare_weights(Net &n, hipStream_t st);
// forward over rows = nR * S; o = output
void net_forward(Net &n, const RegionView &g, int64_t rows, hipStream_t st);
// loss and dL/do from n.o, n.t and n.active (n_active columns counted)
void net_loss(Net &n, int64_t rows, int n_active, hipStream_t st);
// gradients into n.grad (overwritten)
void net_backward(Net &n, const RegionView &g, int64_t rows, hipStream_t st);
// one AdamW step from n.grad (masked parameters are held)
void net_adamw(Net &n, hipStream_t st);
// trainable-parameter mask (host, LAYOUT.total floats; null: every parameter trains)
hipError_t net_set_mask(Net &n, const float *host, hipStream_t st);

}  // namespace gnn
