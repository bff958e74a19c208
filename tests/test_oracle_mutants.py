"""Plant plausible mistakes in a private copy of the C oracle and check that
the closed-form pins reject every mutant (CPU only; the oracle source file in
the repository is not modified)."""

import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from oracle.core import _ptr

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "rwr_oracle.c")

MUTANTS = {
    "dropped_decay": ("for (int64_t v = 0; v < n; ++v) y[v] *= (1.0 - c);", ""),
    "transposed": ("y[dst[e]] += x[u] / (double)deg[u];", "y[u] += x[dst[e]] / (double)deg[u];"),
    "no_degree_normalisation": ("y[dst[e]] += x[u] / (double)deg[u];", "y[dst[e]] += x[u];"),
    "no_dead_end_rescale": ("for (int64_t v = 0; v < n; ++v) r[v] /= s;", ""),
    "offset_without_x0": ("for (int64_t v = 0; v < n_new; ++v) roff[v] = x[v];",
                          "for (int64_t v = 0; v < n_new; ++v) roff[v] = 0.0;"),
    "offset_sign_flip": ("x[v] = qb[v] - qa[v];", "x[v] = qa[v] - qb[v];"),
    "stop_before_first_step": ("if (nrm <= tol) {", "if (nrm <= tol || i >= 1) {"),
}


def _build(mutant: str, tmp: str) -> ctypes.CDLL:
    text = open(SRC).read()
    old, new = MUTANTS[mutant]
    assert text.count(old) >= 1, mutant
    text = text.replace(old, new)
    path = os.path.join(tmp, f"{mutant}.c")
    open(path, "w").write(text)
    so = os.path.join(tmp, f"{mutant}.so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", so, path, "-lm"])
    L = ctypes.CDLL(so)
    i64, i32, dbl, p = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
    L.orc_rwr.argtypes = [i64, i64, p, p, i32, dbl, dbl, i32, p, p]
    L.orc_osp.argtypes = [i64, i64, p, p, i64, i64, p, p, p, dbl, dbl, i32, i32, i32, p, p, p, p]
    return L


def _rwr(L, n, src, dst, s, c):
    r = np.zeros(n)
    it = ctypes.c_int32(0)
    L.orc_rwr(n, src.size, _ptr(src), _ptr(dst), s, c, 1e-14, 100000, _ptr(r), ctypes.byref(it))
    return r


def _pins_pass(L) -> bool:
    c = 0.15
    # directed cycle closed form
    n = 7
    src = np.arange(n, dtype=np.int32)
    dst = ((src + 1) % n).astype(np.int32)
    expect = np.array([c * (1 - c) ** k / (1 - (1 - c) ** n) for k in range(n)])
    if np.abs(_rwr(L, n, src, dst, 0, c) - expect).sum() > 1e-12:
        return False
    # two-node dead end closed form
    s2, d2 = np.array([0], np.int32), np.array([1], np.int32)
    if np.abs(_rwr(L, 2, s2, d2, 0, c) - [1 / (2 - c), (1 - c) / (2 - c)]).sum() > 1e-12:
        return False
    # star: the centre has 4 out-edges (degree normalisation matters)
    a = np.zeros(4, np.int32)
    b = np.arange(1, 5, dtype=np.int32)
    ss, dd = np.concatenate([a, b]), np.concatenate([b, a])
    r = _rwr(L, 5, ss, dd, 0, c)
    if abs(r[0] - 1 / (2 - c)) > 1e-12 or abs(r[1] - (1 - c) / (4 * (2 - c))) > 1e-12:
        return False
    # Theorem 1 against the dense solve of the updated graph
    rng = np.random.default_rng(1)
    n = 40
    e = set()
    while len(e) < 160:
        u, v = int(rng.integers(n)), int(rng.integers(n))
        if u != v:
            e.add((u, v))
    e = np.array(sorted(e), np.int32)
    src, dst = e[:, 0].copy(), e[:, 1].copy()
    r_old = oracle.rwr_dense(n, src, dst, 0, c)
    src2, dst2 = src[5:].copy(), dst[5:].copy()  # delete five edges
    src2 = np.concatenate([src2, [3, 7]]).astype(np.int32)
    dst2 = np.concatenate([dst2, [0, 0]]).astype(np.int32)
    keys = set(zip(src2.tolist(), dst2.tolist()))
    if len(keys) != src2.size:
        return True  # degenerate draw; cannot judge
    r_new = np.zeros(n)
    norms = np.zeros(100001)
    it = ctypes.c_int32(0)
    L.orc_osp(n, src.size, _ptr(src), _ptr(dst), n, src2.size, _ptr(src2), _ptr(dst2), _ptr(r_old), c, 1e-16,
              100000, 1, 0, _ptr(r_new), None, _ptr(norms), ctypes.byref(it))
    exact = oracle.rwr_dense(n, src2, dst2, 0, c)
    if np.abs(r_new - exact).sum() > 1e-12:
        return False
    return True


def test_unmutated_copy_passes():
    with tempfile.TemporaryDirectory() as tmp:
        MUTANTS["identity"] = ("#include <math.h>", "#include <math.h>")
        try:
            assert _pins_pass(_build("identity", tmp))
        finally:
            MUTANTS.pop("identity")


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_mutant_is_caught(mutant):
    with tempfile.TemporaryDirectory() as tmp:
        assert not _pins_pass(_build(mutant, tmp))
