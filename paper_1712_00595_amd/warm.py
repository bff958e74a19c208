"""Parameter initialisation of the warm-start network (host side, seeded).

The parameter vector layout is the one ``include/rwr.h`` states for
``rwr_model_set``.  Initialisation draws uniform weights in +-1/sqrt(fan-in)
from a seeded numpy generator and then sets a few units to a prior, so that
the untrained network already predicts something useful:

* ``prior="propagation"`` (default): the network computes the first four
  terms of the offset series, xhat = sum_{k=0..3} ((1-c) B~^T)^k q.  The
  aggregation a(v) = sum over in-edges u -> v of m(u) / d_out(u) is B~^T
  applied to the messages, so each layer can take one more power.  Since q
  has both signs and the units pass through ReLU, the positive and negative
  parts of q travel in separate units (the operator is non-negative, so
  each part stays non-negative): units 0/1 carry the current power of q+ /
  q-, units 2/3 the running sums; o = (unit 2) - (unit 3).  The residual of
  that prediction is ((1-c) B~^T)^4 q: four iterations are skipped.
* ``prior="copy"``: units 0 and 1 carry +q and -q to the output, so the
  prediction is q itself and its residual (1-c) B~^T q (one iteration).
* ``prior="none"``: the random draw only.

Every other unit starts silent at the output (wo = 0): even a small output on
each of many region nodes would add up to more than ||q||.

For the same reason the trainable network is kept positively homogeneous in
the offset seed (``trainable_mask``): biases stay zero and only the inputs
that scale with q (2, 3 and the q-scaled degrees 13-15) have weights, so
every unit's activation, and the prediction, grows with q.  A unit driven by
the degree inputs alone would add the same amount on every region node
whatever the seed, which no training signal can keep in check.
"""

from __future__ import annotations

import numpy as np

FEAT, HID, MSG, LAYERS = 16, 64, 16, 3

# inputs 2 and 3 of a row: q / ||q|| and |q| / ||q||; 13-15 q-scaled degrees
_Q, _QABS = 2, 3
Q_INPUTS = (2, 3, 13, 14, 15)


def layout():
    """(name, shape) of each tensor, in order."""
    out = [("W0", (FEAT, HID)), ("b0", (HID,))]
    for l in range(1, LAYERS + 1):
        out += [(f"Wp{l}", (HID, MSG)), (f"Ws{l}", (HID, HID)), (f"Wm{l}", (MSG, HID)), (f"b{l}", (HID,))]
    return out + [("wo", (HID,)), ("bo", (1,))]


def init_params(seed: int = 5, prior: str = "propagation", c: float = 0.15, scale: float = 1.0) -> np.ndarray:
    if prior not in ("propagation", "copy", "none"):
        raise ValueError(f"unknown prior {prior!r}")
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = {}
    for name, shape in layout():
        if name.startswith("b"):
            parts[name] = np.zeros(shape)
        else:
            parts[name] = scale * rng.uniform(-1.0, 1.0, size=shape) / np.sqrt(shape[0])
    if prior == "none":
        return np.concatenate([parts[n].reshape(-1) for n, _ in layout()]).astype(np.float32)
    # homogeneous in q: no weight on the inputs that do not scale with it
    for f in range(FEAT):
        if f not in Q_INPUTS:
            parts["W0"][f, :] = 0.0
    k = 4 if prior == "propagation" else 2  # units reserved for the prior
    # reserved units take input only from the prior's own paths
    parts["W0"][:, :k] = 0.0
    parts["b0"][:k] = 0.0
    for l in range(1, LAYERS + 1):
        ws, wm, wp = parts[f"Ws{l}"], parts[f"Wm{l}"], parts[f"Wp{l}"]
        ws[:, :k] = 0.0
        ws[:k, :] = 0.0
        wm[:, :k] = 0.0
        parts[f"b{l}"][:k] = 0.0
        if prior == "propagation":
            wp[:, :2] = 0.0
            wp[:2, :] = 0.0
            wm[:2, :] = 0.0
    parts["wo"][:] = 0.0
    parts["bo"][:] = 0.0
    W0 = parts["W0"]
    if prior == "copy":
        # units 0 and 1: +q and -q through every layer
        W0[_Q, 0], W0[_Q, 1] = 1.0, -1.0
        for l in range(1, LAYERS + 1):
            parts[f"Ws{l}"][0, 0] = parts[f"Ws{l}"][1, 1] = 1.0
        parts["wo"][0], parts["wo"][1] = 1.0, -1.0
    else:
        # q+ = (|q| + q) / 2 and q- = (|q| - q) / 2 start both the current
        # power (units 0, 1) and the running sums (units 2, 3)
        for u, sgn in ((0, 1.0), (1, -1.0), (2, 1.0), (3, -1.0)):
            W0[_QABS, u] = 0.5
            W0[_Q, u] = 0.5 * sgn
        c1 = 1.0 - c
        for l in range(1, LAYERS + 1):
            wp, ws, wm = parts[f"Wp{l}"], parts[f"Ws{l}"], parts[f"Wm{l}"]
            # messages 0, 1: the current powers; a = B~^T m
            wp[0, 0] = wp[1, 1] = 1.0
            # next power (1-c) a, and the running sums take it too
            wm[0, 0] = wm[1, 1] = c1
            wm[0, 2] = wm[1, 3] = c1
            ws[2, 2] = ws[3, 3] = 1.0
        parts["wo"][2], parts["wo"][3] = 1.0, -1.0
    return np.concatenate([parts[n].reshape(-1) for n, _ in layout()]).astype(np.float32)


def trainable_mask() -> np.ndarray:
    """1 for the parameters the optimiser may step, 0 for the ones held at
    zero so that the network stays positively homogeneous in q: every bias
    and the first-layer weights of the inputs that do not scale with q."""
    parts = {name: np.ones(shape) for name, shape in layout()}
    for name in parts:
        if name.startswith("b"):
            parts[name][:] = 0.0
    for f in range(FEAT):
        if f not in Q_INPUTS:
            parts["W0"][f, :] = 0.0
    return np.concatenate([parts[n].reshape(-1) for n, _ in layout()]).astype(np.float32)
