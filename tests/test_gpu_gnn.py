"""GPU parity of the warm-start network: forward output, loss, every
parameter gradient and one AdamW step of the HIP kernels (rwr_gnn_eval)
against the CPU oracle (oracle/gnn.py) with the same bfloat16 rounding of
product operands.  The oracle's own gradients are pinned by central
differences in tests/test_oracle_gnn.py."""

import numpy as np
import pytest

from oracle import gnn

pytestmark = pytest.mark.gpu

rwr = pytest.importorskip("paper_1712_00595_amd.rwr")


def _case(seed, nR, S, m):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, nR, m)
    dst = rng.integers(0, nR, m)
    deg = rng.integers(0, 40, nR)
    dinv = np.where(deg > 0, 1.0 / np.maximum(deg, 1), 0.0).astype(np.float32).astype(np.float64)
    F = rng.normal(size=(nR, S, gnn.FEAT)).astype(np.float32).astype(np.float64)
    theta = gnn.init_params(seed + 5)
    p = gnn.unpack(theta)
    for k in gnn.ORDER:
        if k.startswith("b"):
            p[k] = rng.normal(scale=0.1, size=p[k].shape)
    theta = gnn.pack(p).astype(np.float32).astype(np.float64)
    t = rng.normal(scale=0.3, size=(nR, S)).astype(np.float32).astype(np.float64)
    active = np.ones(S, bool)
    if S > 1:
        active[1] = False
    return theta, src, dst, dinv, F, t, active


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("seed,nR,S,m", [(0, 300, 3, 2500), (1, 5000, 16, 60000), (2, 64, 1, 300)])
def test_network_matches_oracle(seed, nR, S, m):
    print(f"[gnn] seed={seed} nR={nR} S={S} m={m}", flush=True)
    theta, src, dst, dinv, F, t, active = _case(seed, nR, S, m)
    res = rwr.gnn_eval(theta, nR, S, src, dst, dinv, F, t, active, adam_step=True)
    o_ref, cache = gnn.forward(theta, F, src, dst, dinv, rnd=True)
    L_ref, do = gnn.loss(o_ref, t, active)
    g_ref = gnn.backward(theta, F, src, dst, dinv, cache, do, rnd=True)
    # forward output and loss
    assert _rel(res["out"], o_ref) < 2e-3, _rel(res["out"], o_ref)
    assert abs(res["loss"] - L_ref) <= 2e-3 * abs(L_ref) + 1e-9
    # gradient, block by block
    g = res["grad"].astype(np.float64)
    off = 0
    for k in gnn.ORDER:
        n = int(np.prod(gnn.SHAPES[k]))
        gb, rb = g[off:off + n], g_ref[off:off + n]
        assert _rel(gb, rb) < 1e-2 or np.linalg.norm(gb - rb) < 1e-6 * np.linalg.norm(g_ref), (k, _rel(gb, rb))
        off += n
    assert _rel(g, g_ref) < 5e-3
    # AdamW from zero moments, applied to the device's own gradient
    th_ref, _, _ = gnn.adamw(theta, g, np.zeros_like(theta), np.zeros_like(theta), 1)
    assert np.abs(res["params_after"] - th_ref).max() < 1e-6


def test_rejects_malformed_region():
    theta, src, dst, dinv, F, t, active = _case(3, 10, 1, 20)
    with pytest.raises((ValueError, rwr.RwrError)):
        rwr.gnn_eval(theta[:-1], 10, 1, src, dst, dinv, F)
    with pytest.raises(rwr.RwrError):
        rwr.gnn_eval(theta, 10, 1, np.append(src, 10), np.append(dst, 0), dinv, F)
