"""ctypes front end of the C oracle plus the numpy parts of the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rwr_oracle.c")
_LIB = os.path.join(_HERE, "librwr_oracle.so")
_lock = threading.Lock()
_lib = None


class OracleError(RuntimeError):
    pass


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
            p = ctypes.c_void_p
            L.orc_cpi.argtypes = [i64, i64, p, p, p, dbl, dbl, i32, p, p, p]
            L.orc_cpi.restype = ctypes.c_int
            L.orc_rwr.argtypes = [i64, i64, p, p, i32, dbl, dbl, i32, p, p]
            L.orc_rwr.restype = ctypes.c_int
            L.orc_dead_end_reachable.argtypes = [i64, i64, p, p, i32]
            L.orc_dead_end_reachable.restype = ctypes.c_int
            L.orc_osp.argtypes = [i64, i64, p, p, i64, i64, p, p, p, dbl, dbl, i32, i32, i32, p, p, p, p]
            L.orc_osp.restype = ctypes.c_int
            _lib = L
    return _lib


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


STATIC_TOL = 1e-14
STATIC_MAX_ITERS = 100000


def cpi(n, src, dst, q, c, tol, max_iter=STATIC_MAX_ITERS, *, with_norms=False, allow_noconv=False):
    """Cumulative power iteration of Section 2.2 from seed vector ``q``."""
    src, dst, q = _i32(src), _i32(dst), _f64(q)
    r = np.zeros(n, dtype=np.float64)
    norms = np.zeros(max_iter + 1, dtype=np.float64) if with_norms else None
    it = ctypes.c_int32(0)
    st = lib().orc_cpi(
        n, src.shape[0], _ptr(src), _ptr(dst), _ptr(q), c, tol, max_iter, _ptr(r),
        _ptr(norms) if norms is not None else None, ctypes.byref(it),
    )
    if st != 0 and not (allow_noconv and st == -6):
        raise OracleError(f"orc_cpi failed: {st}")
    if with_norms:
        return r, it.value, norms[: it.value + 1]
    return r, it.value


def rwr_static(n, src, dst, seed, c, tol=STATIC_TOL, max_iter=STATIC_MAX_ITERS):
    """Static RWR scores of Eq. (1) with Theorem 4's dead-end handling."""
    src, dst = _i32(src), _i32(dst)
    r = np.zeros(n, dtype=np.float64)
    it = ctypes.c_int32(0)
    st = lib().orc_rwr(n, src.shape[0], _ptr(src), _ptr(dst), int(seed), c, tol, max_iter, _ptr(r), ctypes.byref(it))
    if st != 0:
        raise OracleError(f"orc_rwr failed: {st}")
    return r


def dead_end_reachable(n, src, dst, seed) -> bool:
    src, dst = _i32(src), _i32(dst)
    v = lib().orc_dead_end_reachable(n, src.shape[0], _ptr(src), _ptr(dst), int(seed))
    if v < 0:
        raise OracleError("out of memory")
    return bool(v)


RENORM_PAPER, RENORM_ALWAYS, RENORM_NEVER = 0, 1, 2


def osp(old, new, r_old, c, eps, *, max_iter=STATIC_MAX_ITERS, renorm=RENORM_PAPER, seed=-1):
    """One OSP / OSP-T update (Section 3.1, Algorithm 1).

    ``old`` and ``new`` are ``(n, src, dst)`` triples.  Returns a dict with
    ``r_new``, ``q_off``, ``iters`` and ``norms`` (||x^(i)||_1, i = 0..iters).
    """
    n0, s0, d0 = old
    n1, s1, d1 = new
    s0, d0, s1, d1 = _i32(s0), _i32(d0), _i32(s1), _i32(d1)
    r_old = _f64(r_old)
    if r_old.shape[0] != n0:
        raise ValueError("r_old length must equal the old node count")
    r_new = np.zeros(n1, dtype=np.float64)
    q_off = np.zeros(n1, dtype=np.float64)
    norms = np.zeros(max_iter + 1, dtype=np.float64)
    it = ctypes.c_int32(0)
    st = lib().orc_osp(
        n0, s0.shape[0], _ptr(s0), _ptr(d0), n1, s1.shape[0], _ptr(s1), _ptr(d1), _ptr(r_old), c, eps,
        max_iter, renorm, int(seed), _ptr(r_new), _ptr(q_off), _ptr(norms), ctypes.byref(it),
    )
    if st not in (0, -6):
        raise OracleError(f"orc_osp failed: {st}")
    return {
        "r_new": r_new,
        "q_off": q_off,
        "iters": it.value,
        "norms": norms[: it.value + 1].copy(),
        "converged": st == 0,
    }


def row_normalised_dense(n, src, dst) -> np.ndarray:
    """Dense A~ (Section 2.1): A~[u, v] = 1/d_out(u) per edge, dead-end rows 0."""
    A = np.zeros((n, n), dtype=np.float64)
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    np.add.at(A, (src, dst), 1.0)
    deg = A.sum(axis=1)
    nz = deg > 0
    A[nz] /= deg[nz, None]
    return A


def rwr_dense(n, src, dst, seed, c) -> np.ndarray:
    """Static RWR by an LU solve of (I - (1-c) A~^T) r = c e_s, then
    Theorem 4's normalisation when a dead end is reachable from the seed."""
    A = row_normalised_dense(n, src, dst)
    M = np.eye(n) - (1.0 - c) * A.T
    b = np.zeros(n)
    b[seed] = c
    r = np.linalg.solve(M, b)
    if dead_end_reachable(n, src, dst, seed):
        r = r / np.abs(r).sum()
    return r


def reachable_from(n, src, dst, sources) -> np.ndarray:
    """Boolean mask of the nodes reachable from any node in ``sources``
    (breadth-first over out-edges, plain numpy)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    order = np.argsort(src, kind="stable")
    dsorted = dst[order]
    start = np.concatenate([[0], np.cumsum(np.bincount(src, minlength=n))])
    seen = np.zeros(n, dtype=bool)
    front = np.unique(np.asarray(sources, dtype=np.int64))
    seen[front] = True
    while front.shape[0]:
        lens = start[front + 1] - start[front]
        idx = np.repeat(start[front], lens) + (np.arange(lens.sum()) - np.repeat(np.cumsum(lens) - lens, lens))
        nxt = np.unique(dsorted[idx])
        nxt = nxt[~seen[nxt]]
        seen[nxt] = True
        front = nxt
    return seen


def rwr_static_vector(n, src, dst, q, c, tol=STATIC_TOL, max_iter=STATIC_MAX_ITERS):
    """Static scores for a general restart vector q (Eq. (1) with q in place
    of e_s; q = 1/n is global PageRank): CPI of Section 2.2 from c q, then
    Theorem 4's normalisation when a dead end is reachable from the support
    of q."""
    q = _f64(q)
    r, _ = cpi(n, src, dst, c * q, c, tol, max_iter)
    deg = np.bincount(np.asarray(src, dtype=np.int64), minlength=n)
    if np.any(reachable_from(n, src, dst, np.flatnonzero(q != 0.0)) & (deg == 0)):
        r = r / r.sum()
    return r


def delta_weight(old, new, r_old) -> float:
    """||D r_old||_1 of the section on the effects of Delta G (Section 3.3):
    D is diagonal with D_uu = sum_v |B~[u,v] - A~[u,v]|, the L1 norm of the
    change of u's row of the row-normalised adjacency, so that
    ||q_offset||_1 <= (1-c) ||D r_old||_1.  Old rows are padded to the new
    node count as empty rows, r_old with zeros.  Plain definition with scipy
    sparse matrices (no reuse of the update arithmetic).  Parity pinned by
    closed forms for single-edge edits and by the inequality above."""
    import scipy.sparse as sp

    n0, s0, d0 = old
    n1, s1, d1 = new

    def normalised(n, s, d):
        s = np.asarray(s, dtype=np.int64)
        d = np.asarray(d, dtype=np.int64)
        deg = np.bincount(s, minlength=n).astype(np.float64)
        return sp.csr_matrix((1.0 / deg[s], (s, d)), shape=(n1, n1))

    delta = normalised(n1, s1, d1) - normalised(n0, s0, d0)
    D = np.asarray(abs(delta).sum(axis=1)).ravel()
    r = np.zeros(n1, dtype=np.float64)
    r[:n0] = np.abs(_f64(r_old))
    return float(D @ r)


KEY = np.int64(1) << np.int64(32)


def apply_batch(n, src, dst, batch, *, undirected=False, del_nodes=(), rows_only=False):
    """Edge list of G + Delta G.

    ``batch`` has ``ins_src, ins_dst, del_src, del_dst, n_new_nodes``.  Raises
    :class:`OracleError` (with code 'EINVAL', 'EEXIST' or 'ENOENT') for an
    invalid batch.  New nodes get ids n..n+k-1 (Section 3.4.1).  A deleted
    node (an existing id, listed once, not named by the batch's edge
    entries) loses every incident edge: its row and column become zero
    (reading G9); with ``rows_only`` it loses its out-edges only, the zero
    row Section 3.4.1 states, and keeps its in-edges (a directed graph's
    reading; undirected graphs lose every pair either way).
    Undirected graphs store both directions of each pair; batch pairs are
    given once.
    """
    n_new = int(n) + int(getattr(batch, "n_new_nodes", 0))
    s = np.asarray(src, dtype=np.int64)
    d = np.asarray(dst, dtype=np.int64)
    ins_s = np.asarray(batch.ins_src, dtype=np.int64)
    ins_d = np.asarray(batch.ins_dst, dtype=np.int64)
    del_s = np.asarray(batch.del_src, dtype=np.int64)
    del_d = np.asarray(batch.del_dst, dtype=np.int64)
    for a in (ins_s, ins_d, del_s, del_d):
        if a.size and (a.min() < 0 or a.max() >= n_new):
            raise OracleError("EINVAL")
    if undirected:
        def canon(a, b):
            return np.minimum(a, b) * KEY + np.maximum(a, b)
        cur = np.unique(canon(s, d))
        ik, dk = canon(ins_s, ins_d), canon(del_s, del_d)
    else:
        cur = s * KEY + d
        ik, dk = ins_s * KEY + ins_d, del_s * KEY + del_d
    allk = np.concatenate([ik, dk])
    if np.unique(allk).shape[0] != allk.shape[0]:
        raise OracleError("EINVAL")
    if dk.size and not np.isin(dk, cur).all():
        raise OracleError("ENOENT")
    if ik.size and np.isin(ik, cur).any():
        raise OracleError("EEXIST")
    keep = ~np.isin(cur, dk)
    newk = np.concatenate([cur[keep], ik])
    if len(del_nodes) == 0:
        del_nodes = getattr(batch, "del_nodes", ())
    dn = np.asarray(del_nodes, dtype=np.int64)
    if dn.size:
        # deleted nodes: distinct existing nodes, not named by the batch's
        # own edge entries
        if dn.min() < 0 or dn.max() >= n or np.unique(dn).shape[0] != dn.shape[0]:
            raise OracleError("EINVAL")
        if np.isin(np.concatenate([ins_s, ins_d, del_s, del_d]), dn).any():
            raise OracleError("EINVAL")
        a, b = newk // KEY, newk % KEY
        inc = np.isin(a, dn) if (rows_only and not undirected) else (np.isin(a, dn) | np.isin(b, dn))
        newk = newk[~inc]
    a = (newk // KEY).astype(np.int32)
    b = (newk % KEY).astype(np.int32)
    if undirected:
        loop = a == b
        src2 = np.concatenate([a, b[~loop]])
        dst2 = np.concatenate([b, a[~loop]])
        return n_new, src2, dst2
    return n_new, a, b


def apply_stream(n, src, dst, batches):
    """Edge list after applying ``batches`` in order (directed graphs).

    Each batch is validated against the graph it is applied to (inserted
    edges absent, deleted edges present, no repeats), exactly as
    :func:`apply_batch` does, but the state is kept as the initial sorted key
    array plus a dictionary of changed keys, so a long stream of small
    batches costs one pass over the edge list.
    """
    s0 = np.asarray(src, dtype=np.int64)
    d0 = np.asarray(dst, dtype=np.int64)
    init = np.sort(s0 * KEY + d0)
    changed = {}
    n_cur = int(n)

    def present(k):
        if k in changed:
            return changed[k]
        i = int(np.searchsorted(init, k))
        return i < init.shape[0] and int(init[i]) == k

    for b in batches:
        if len(getattr(b, "del_nodes", ())):
            raise ValueError("apply_stream takes edge batches only; use apply_batch for node deletions")
        n_cur += int(getattr(b, "n_new_nodes", 0))
        ik = [int(u) * int(KEY) + int(v) for u, v in zip(b.ins_src, b.ins_dst)]
        dk = [int(u) * int(KEY) + int(v) for u, v in zip(b.del_src, b.del_dst)]
        for u, v in list(zip(b.ins_src, b.ins_dst)) + list(zip(b.del_src, b.del_dst)):
            if not (0 <= u < n_cur and 0 <= v < n_cur):
                raise OracleError("EINVAL")
        if len(set(ik + dk)) != len(ik) + len(dk):
            raise OracleError("EINVAL")
        if any(not present(k) for k in dk):
            raise OracleError("ENOENT")
        if any(present(k) for k in ik):
            raise OracleError("EEXIST")
        for k in dk:
            changed[k] = False
        for k in ik:
            changed[k] = True
    gone = np.array(sorted(k for k, p in changed.items() if not p), dtype=np.int64)
    added = np.array(sorted(k for k, p in changed.items() if p), dtype=np.int64)
    keys = s0 * KEY + d0
    keep = ~np.isin(keys, gone) if gone.size else np.ones(keys.shape[0], bool)
    fresh = added[~np.isin(added, init)] if added.size else added
    allk = np.concatenate([keys[keep], fresh])
    return n_cur, (allk // KEY).astype(np.int32), (allk % KEY).astype(np.int32)
