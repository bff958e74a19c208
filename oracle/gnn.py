"""CPU oracle of the learned warm start -- TEST INFRASTRUCTURE ONLY.

The paper has no learned component.  The warm start predicts the offset
result r_offset = sum_i x^(i) of Section 3.1 from local features, and the
update then propagates only the residual of that prediction, so OSP's
exactness (Theorem 1) and OSP-T's bound (Theorem 3) are untouched:

    rho = q_offset - (I - (1-c) B~^T) xhat,   r_offset = xhat + sum_i ((1-c) B~^T)^i rho.

This module is the plain numpy definition of the network, its loss and its
gradients (float64 throughout; optionally with the operands of every matrix
product rounded to bfloat16, the precision the device's matrix cores take),
plus the residual identity above written out with dense operators.

Model (one region of nR nodes, S seed columns, features F[nR, S, 16]):
    h0 = relu(F W0 + b0)
    for l = 1..3:  m = h_{l-1} Wp_l                  (64 -> 16)
                   a[v] = sum_{u -> v in region} m[u] / d_out(u)
                   h_l = relu(h_{l-1} Ws_l + a Wm_l + b_l)
    o = h_3 wo + bo,   xhat[v, j] = ||q_offset[:, j]||_1 * o[v, j]
Loss: mean over active columns of sum_v huber(o[v, j] - t[v, j]; delta) with
t = r_offset / ||q_offset||_1 on the region.
"""

from __future__ import annotations

import numpy as np

FEAT = 16
HID = 64
MSG = 16
LAYERS = 3
HUBER_DELTA = 1e-3

# parameter vector layout (float32 on the device, float64 here)
_SHAPES = [("W0", (FEAT, HID)), ("b0", (HID,))]
for _l in range(1, LAYERS + 1):
    _SHAPES += [(f"Wp{_l}", (HID, MSG)), (f"Ws{_l}", (HID, HID)), (f"Wm{_l}", (MSG, HID)), (f"b{_l}", (HID,))]
_SHAPES += [("wo", (HID,)), ("bo", (1,))]
SHAPES = dict(_SHAPES)
ORDER = [k for k, _ in _SHAPES]
N_PARAMS = int(sum(int(np.prod(s)) for _, s in _SHAPES))


def unpack(theta: np.ndarray) -> dict:
    theta = np.asarray(theta, dtype=np.float64)
    if theta.shape != (N_PARAMS,):
        raise ValueError(f"expected {N_PARAMS} parameters")
    out, o = {}, 0
    for k in ORDER:
        s = SHAPES[k]
        n = int(np.prod(s))
        out[k] = theta[o:o + n].reshape(s)
        o += n
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], np.float64).reshape(-1) for k in ORDER])


def init_params(seed: int = 5) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = {}
    for k in ORDER:
        s = SHAPES[k]
        if k.startswith("b"):
            p[k] = np.zeros(s)
        else:
            fan_in = s[0]
            p[k] = rng.uniform(-1.0, 1.0, size=s) / np.sqrt(fan_in)
    return pack(p).astype(np.float32).astype(np.float64)


def bf16(x: np.ndarray) -> np.ndarray:
    """Round float64 values to bfloat16 (round to nearest, ties to even),
    through float32 as the device does."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _mm(x, w, rnd):
    if rnd:
        return bf16(x) @ bf16(w)
    return x @ w


def aggregate(m: np.ndarray, src: np.ndarray, dst: np.ndarray, dinv: np.ndarray, nR: int) -> np.ndarray:
    """a[v] = sum over region edges u -> v of m[u] / d_out(u)."""
    a = np.zeros((nR,) + m.shape[1:])
    np.add.at(a, dst, m[src] * dinv[src][:, None, None])
    return a


def aggregate_t(da: np.ndarray, src: np.ndarray, dst: np.ndarray, dinv: np.ndarray, nR: int) -> np.ndarray:
    """Transpose of :func:`aggregate`: dm[u] = sum over u -> v of da[v] / d_out(u)."""
    dm = np.zeros((nR,) + da.shape[1:])
    np.add.at(dm, src, da[dst] * dinv[src][:, None, None])
    return dm


def forward(theta, F, src, dst, dinv, *, rnd=False):
    """Network output o[nR, S] and the activations the backward pass needs.

    ``src``/``dst`` are the region's edges in local ids, ``dinv`` = 1/d_out of
    each region node in the whole graph (0 for dead ends)."""
    p = unpack(theta)
    F = np.asarray(F, np.float64)
    nR = F.shape[0]
    z0 = _mm(F, p["W0"], rnd) + p["b0"]
    h = [np.maximum(z0, 0.0)]
    a_s = []
    for l in range(1, LAYERS + 1):
        m = _mm(h[-1], p[f"Wp{l}"], rnd)
        a = aggregate(m, src, dst, dinv, nR)
        a_s.append(a)
        z = _mm(h[-1], p[f"Ws{l}"], rnd) + _mm(a, p[f"Wm{l}"], rnd) + p[f"b{l}"]
        h.append(np.maximum(z, 0.0))
    o = _mm(h[-1], p["wo"][:, None], rnd)[..., 0] + p["bo"][0]
    return o, {"h": h, "a": a_s}


def huber(e: np.ndarray, delta: float = HUBER_DELTA):
    ae = np.abs(e)
    val = np.where(ae <= delta, 0.5 * e * e / delta, ae - 0.5 * delta)
    grad = np.where(ae <= delta, e / delta, np.sign(e))
    return val, grad


def loss(o, t, active, delta: float = HUBER_DELTA):
    """Mean over active columns of the summed Huber error, and dL/do."""
    active = np.asarray(active, bool)
    C = max(1, int(active.sum()))
    val, g = huber(o - t, delta)
    val = val * active[None, :]
    g = g * active[None, :] / C
    return float(val.sum() / C), g


def backward(theta, F, src, dst, dinv, cache, do, *, rnd=False):
    """Gradient of the loss w.r.t. the parameter vector, given dL/do."""
    p = unpack(theta)
    F = np.asarray(F, np.float64)
    nR = F.shape[0]
    h, a_s = cache["h"], cache["a"]
    g = {k: np.zeros(SHAPES[k]) for k in ORDER}
    r = bf16 if rnd else (lambda x: x)

    def wgrad(x, dz):
        # sum over nodes and columns of x^T dz
        return np.einsum("vsk,vsn->kn", r(x), r(dz))

    g["wo"] = np.einsum("vsk,vs->k", r(h[-1]), r(do))
    g["bo"] = np.array([do.sum()])
    dh = r(do)[..., None] * r(p["wo"])[None, None, :]
    for l in range(LAYERS, 0, -1):
        dz = dh * (h[l] > 0)
        g[f"b{l}"] = dz.sum(axis=(0, 1))
        g[f"Ws{l}"] = wgrad(h[l - 1], dz)
        g[f"Wm{l}"] = wgrad(a_s[l - 1], dz)
        da = _mm(dz, p[f"Wm{l}"].T, rnd)
        dm = aggregate_t(da, src, dst, dinv, nR)
        g[f"Wp{l}"] = wgrad(h[l - 1], dm)
        dh = _mm(dz, p[f"Ws{l}"].T, rnd) + _mm(dm, p[f"Wp{l}"].T, rnd)
    dz0 = dh * (h[0] > 0)
    g["b0"] = dz0.sum(axis=(0, 1))
    g["W0"] = wgrad(F, dz0)
    return pack(g)


def adamw(theta, grad, m, v, step, *, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, wd=1e-4):
    """One AdamW step (decoupled weight decay), step counted from 1."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    theta = theta - lr * (mh / (np.sqrt(vh) + eps) + wd * theta)
    return theta, m, v


# ------------------------------------------------------------ the warm start

def residual(q, xhat, P):
    """rho = q - (I - P) xhat for a dense propagation operator P = (1-c) B~^T."""
    return q - xhat + P @ xhat


def region(n, src, dst, start, hops: int, cap: int):
    """Nodes within `hops` out-hops of `start` (breadth first, level by
    level); a level that would take the region past `cap` nodes is not
    added.  Returns (nodes in order of discovery, hop of each)."""
    out = [[] for _ in range(n)]
    for u, v in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()):
        out[u].append(v)
    hop = {int(v): 0 for v in start}
    level = sorted(hop)
    order = list(level)
    for h in range(1, hops + 1):
        nxt = sorted({v for u in level for v in out[u] if v not in hop})
        if len(order) + len(nxt) > cap:
            break
        for v in nxt:
            hop[v] = h
        order += nxt
        level = nxt
    return np.array(order, dtype=np.int64), np.array([hop[v] for v in order], dtype=np.int64)


# ------------------------------------------------------------ inside an update
#
# What an update computes when the warm start is on, written out plainly for
# one batch: the region around the offset seed, the network's inputs, the
# prediction with its mass correction, the exact residual and the training
# loss with its gradient.  Row order: region node i, seed column j at
# row i * S + j; nodes are the graph's own ids.

def propagation_operator(n, src, dst, c):
    """P = (1-c) B~^T as a sparse matrix: P[v, u] = (1-c) / d_out(u) for every
    edge u -> v (Section 2.1's row normalisation; dead-end rows are zero)."""
    import scipy.sparse as sp

    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    deg = np.bincount(src, minlength=n).astype(np.float64)
    return sp.csr_matrix(((1.0 - c) / deg[src], (dst, src)), shape=(n, n))


def offset_support(old, new, r_old):
    """Level 0 of the region: every node v whose coefficient B~[u, v] -
    A~[u, v] is non-zero for some row u that the batch changed and whose old
    score is non-zero in some column (Section 3.1: these are the nodes the
    offset seed q = (1-c)(B~^T - A~^T) r_old can reach in one step).  ``old``
    and ``new`` are (n, src, dst); r_old has old-n rows (one column per seed,
    or a vector)."""
    import scipy.sparse as sp

    n0, s0, d0 = old
    n1, s1, d1 = new

    def normalised(n, s, d):
        s = np.asarray(s, dtype=np.int64)
        d = np.asarray(d, dtype=np.int64)
        deg = np.bincount(s, minlength=n).astype(np.float64)
        return sp.csr_matrix((1.0 / deg[s], (s, d)), shape=(n1, n1))

    delta = (normalised(n1, s1, d1) - normalised(n0, s0, d0)).tocoo()
    r = np.zeros((n1,) + np.shape(r_old)[1:])
    r[:n0] = np.asarray(r_old, np.float64)
    live_row = np.any(r.reshape(n1, -1) != 0.0, axis=1)
    keep = (delta.data != 0.0) & live_row[delta.row]
    return np.unique(delta.col[keep])


def features(n_total, src, dst, nodes, hop, q, r_old, sigma, seeds):
    """The sixteen inputs of every (region node, column) row, as float32:
    0 log(1+d_in)/8, 1 log(1+d_out)/8, 2 q/||q_j||_1, 3 |q|/||q_j||_1,
    4 log(1 + max(0, n r_old/sigma_j))/8, 5..8 hop 0, 1, 2, >=3 (one-hot),
    9 dead end, 10 seed of the column, 11 1/d_out (0 for a dead end),
    12 1/d_in (0 without in-edges), 13 input 3 * input 0, 14 input 3 *
    input 1, 15 input 2 * input 0 (in float32).  Degrees are those of the
    graph after the batch; q is the offset seed (n x S), r_old the scores
    before the batch (n x S, rows of new nodes zero), sigma their column
    sums."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    nodes = np.asarray(nodes, dtype=np.int64)
    n = q.shape[0]
    S = q.shape[1]
    dout = np.bincount(src, minlength=n)[nodes].astype(np.float64)
    din = np.bincount(dst, minlength=n)[nodes].astype(np.float64)
    qn = np.abs(q).sum(axis=0)
    F = np.zeros((nodes.shape[0], S, FEAT))
    F[:, :, 0] = (np.log1p(din) / 8.0)[:, None]
    F[:, :, 1] = (np.log1p(dout) / 8.0)[:, None]
    qq = np.where(qn > 0, q[nodes] / np.where(qn > 0, qn, 1.0), 0.0)
    F[:, :, 2] = qq
    F[:, :, 3] = np.abs(qq)
    rn = np.where(sigma != 0, r_old[nodes] / np.where(sigma != 0, sigma, 1.0), 0.0)
    F[:, :, 4] = np.log1p(np.maximum(0.0, rn * n_total)) / 8.0
    for k in range(4):
        F[:, :, 5 + k] = ((hop == k) if k < 3 else (hop >= 3))[:, None]
    F[:, :, 9] = (dout == 0)[:, None]
    F[:, :, 10] = nodes[:, None] == np.asarray(seeds, np.int64)[None, :]
    F[:, :, 11] = np.where(dout > 0, 1.0 / np.maximum(dout, 1.0), 0.0)[:, None]
    F[:, :, 12] = np.where(din > 0, 1.0 / np.maximum(din, 1.0), 0.0)[:, None]
    F = F.astype(np.float32)
    F[:, :, 13] = F[:, :, 3] * F[:, :, 0]
    F[:, :, 14] = F[:, :, 3] * F[:, :, 1]
    F[:, :, 15] = F[:, :, 2] * F[:, :, 0]
    return F.astype(np.float64)


def local_edges(src, dst, nodes):
    """Edges of the graph with both ends in the region, in local ids."""
    loc = -np.ones(int(max(np.max(src), np.max(dst), np.max(nodes))) + 1, dtype=np.int64)
    loc[np.asarray(nodes, np.int64)] = np.arange(len(nodes))
    ls, ld = loc[np.asarray(src, np.int64)], loc[np.asarray(dst, np.int64)]
    keep = (ls >= 0) & (ld >= 0)
    return ls[keep], ld[keep]


def mass_correction(xhat, live, c, qsum):
    """The prediction corrected so that its residual sums to zero in every
    column.  The column sums of I - (1-c) B~^T are w_v = 1 - (1-c) [v is not
    a dead end], so sum(rho) = sum(q) - f(xhat) with f(x) = sum_v w_v x_v;
    xhat' = xhat - beta |xhat| with beta = (f(xhat) - sum(q)) / f(|xhat|)
    (beta = 0 when f(|xhat|) = 0).  Returns (xhat', beta, f(|xhat|), w)."""
    w = 1.0 - (1.0 - c) * np.asarray(live, np.float64)
    fx = (w[:, None] * xhat).sum(axis=0)
    fa = (w[:, None] * np.abs(xhat)).sum(axis=0)
    beta = np.where(fa > 0, (fx - qsum) / np.where(fa > 0, fa, 1.0), 0.0)
    return xhat - beta[None, :] * np.abs(xhat), beta, fa, w


def residual_loss(theta, F, lsrc, ldst, dinv, nodes, q, P, live, c, *, follow=True, rnd=False):
    """Training loss of the warm start inside an update and its gradient.

    xhat = ||q_j||_1 o on the region rows (o the network output), corrected
    by :func:`mass_correction`, zero elsewhere; rho = q - (I - P) xhat' on
    every node; over the active columns (||q_j||_1 > 0),
    L = sum_j ||rho_j||_1 / sum_j ||q_j||_1 and dL/dxhat' = (-(I - P)^T
    sign(rho)) / Q with Q = sum_j ||q_j||_1.
    With follow=True the gradient goes through the correction exactly:
      dL/dxhat_v = (1 - beta s_v) (dL/dxhat'_v - w_v K / f(|xhat|)),
      K = sum_u dL/dxhat'_u |xhat_u|,  s = sign(xhat);
    with follow=False the correction is held fixed (dL/dxhat = dL/dxhat').
    Then dL/do = ||q_j||_1 dL/dxhat and the network's backward pass gives
    dL/dtheta.  ``P`` is :func:`propagation_operator` of the graph after the
    batch, ``live`` marks region nodes that are not dead ends."""
    nodes = np.asarray(nodes, np.int64)
    o, cache = forward(theta, F, lsrc, ldst, dinv, rnd=rnd)
    qn = np.abs(q).sum(axis=0)
    qsum = q[nodes].sum(axis=0)
    active = qn > 0
    Q = float(qn[active].sum())
    xhat = qn[None, :] * o
    xc, beta, fa, w = mass_correction(xhat, live, c, qsum)
    X = np.zeros_like(q)
    X[nodes] = xc
    rho = q - X + P @ X
    L = float(np.abs(rho).sum(axis=0)[active].sum() / Q) if Q > 0 else 0.0
    sg = np.sign(rho)
    gprime = ((-sg + P.T @ sg)[nodes]) * np.where(active, 1.0 / Q if Q > 0 else 0.0, 0.0)[None, :]
    if follow:
        K = (gprime * np.abs(xhat)).sum(axis=0)
        corr = np.where(fa > 0, K / np.where(fa > 0, fa, 1.0), 0.0)
        gx = (1.0 - beta[None, :] * np.sign(xhat)) * (gprime - w[:, None] * corr[None, :])
    else:
        gx = gprime
    do = qn[None, :] * gx
    grad = backward(theta, F, lsrc, ldst, dinv, cache, do, rnd=rnd)
    return {"loss": L, "grad": grad, "do": do, "o": o, "rho": rho, "xhat": xc, "beta": beta, "active": active}
