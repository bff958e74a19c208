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
