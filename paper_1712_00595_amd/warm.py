"""Parameter initialisation of the warm-start network (host side, seeded).

The parameter vector layout is the one ``include/rwr.h`` states for
``rwr_model_set``.  Initialisation draws uniform weights in +-1/sqrt(fan-in)
from a seeded numpy generator; with ``copy_prior`` two hidden units carry the
input q_offset/||q|| straight to the output (ReLU(x) - ReLU(-x) = x), the
other units start small, so that the untrained network already predicts the
offset seed itself (whose residual is (1-c) B~^T q, smaller than q).
"""

from __future__ import annotations

import numpy as np

FEAT, HID, MSG, LAYERS = 16, 64, 16, 3


def layout():
    """(name, shape) of each tensor, in order."""
    out = [("W0", (FEAT, HID)), ("b0", (HID,))]
    for l in range(1, LAYERS + 1):
        out += [(f"Wp{l}", (HID, MSG)), (f"Ws{l}", (HID, HID)), (f"Wm{l}", (MSG, HID)), (f"b{l}", (HID,))]
    return out + [("wo", (HID,)), ("bo", (1,))]


def init_params(seed: int = 5, copy_prior: bool = True, scale: float = 1.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = {}
    for name, shape in layout():
        if name.startswith("b"):
            parts[name] = np.zeros(shape)
        else:
            parts[name] = scale * rng.uniform(-1.0, 1.0, size=shape) / np.sqrt(shape[0])
    if copy_prior:
        # units 0 and 1 carry +q and -q (input 2) through every layer
        parts["W0"][:, :2] = 0.0
        parts["W0"][2, 0], parts["W0"][2, 1] = 1.0, -1.0
        for l in range(1, LAYERS + 1):
            ws = parts[f"Ws{l}"]
            ws[:, :2] = 0.0
            ws[:2, :] = 0.0
            ws[0, 0] = ws[1, 1] = 1.0
            parts[f"Wm{l}"][:, :2] = 0.0
        # the other units start silent at the output: even a small output on
        # each of many region nodes would add up to more than ||q||
        parts["wo"][:] = 0.0
        parts["wo"][0], parts["wo"][1] = 1.0, -1.0
    return np.concatenate([parts[n].reshape(-1) for n, _ in layout()]).astype(np.float32)
