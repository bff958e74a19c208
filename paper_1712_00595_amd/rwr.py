"""Python binding of the HIP dynamic-RWR library (``librwr.so``).

Argument marshalling only: every step of the update runs in the library's HIP
kernels.  Arrays may be numpy arrays (host) or torch CUDA tensors (device);
the library must have been built (``__graft_entry__.build()``) -- there is no
fallback path.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librwr.so")

STATUS = {
    0: "RWR_OK",
    -1: "RWR_EINVAL",
    -2: "RWR_ENOMEM",
    -3: "RWR_EHIP",
    -4: "RWR_EEXIST",
    -5: "RWR_ENOENT",
    -6: "RWR_ENOCONV",
    -7: "RWR_ENUMERIC",
    -8: "RWR_ESTATE",
    -9: "RWR_EIO",
}

EXPORTED = [
    "rwr_config_default",
    "rwr_build",
    "rwr_build_vectors",
    "rwr_update",
    "rwr_refine",
    "rwr_scores",
    "rwr_graph_size",
    "rwr_graph_export",
    "rwr_last_norms",
    "rwr_sweep_shape",
    "rwr_profile",
    "rwr_profile_read",
    "rwr_destroy",
    "rwr_last_error",
    "rwr_gnn_num_params",
    "rwr_gnn_eval",
    "rwr_model_set",
    "rwr_model_get",
    "rwr_warm_start",
    "rwr_warm_inspect",
    "rwr_model_trainable",
    "rwr_gnn_eval_noalloc",
    "rwr_scores_set",
    "rwr_save",
    "rwr_load",
    "rwr_context_info",
]


class RwrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        self.code = code
        self.name = STATUS.get(code, str(code))
        super().__init__(f"{self.name}: {msg}")


class Config(ctypes.Structure):
    _fields_ = [
        ("c", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("err_budget", ctypes.c_double),
        ("build_tol", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("undirected", ctypes.c_int32),
        ("max_iters", ctypes.c_int32),
        ("pull_ratio", ctypes.c_int32),
        ("reorder", ctypes.c_int32),
        ("autotune", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("deterministic", ctypes.c_int32),
        ("node_deletion", ctypes.c_int32),
        ("phase_timing", ctypes.c_int32),
        ("dev_alloc", ctypes.c_void_p),
        ("dev_free", ctypes.c_void_p),
        ("alloc_user", ctypes.c_void_p),
    ]


class BatchStruct(ctypes.Structure):
    _fields_ = [
        ("n_ins", ctypes.c_int64),
        ("ins_src", ctypes.c_void_p),
        ("ins_dst", ctypes.c_void_p),
        ("n_del", ctypes.c_int64),
        ("del_src", ctypes.c_void_p),
        ("del_dst", ctypes.c_void_p),
        ("n_new_nodes", ctypes.c_int32),
        ("n_del_nodes", ctypes.c_int32),
        ("del_nodes", ctypes.c_void_p),
        ("on_device", ctypes.c_int32),
    ]


class StatsStruct(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("dense_iters", ctypes.c_int32),
        ("refined", ctypes.c_int32),
        ("checked", ctypes.c_int32),
        ("visited_edges", ctypes.c_int64),
        ("touched_rows", ctypes.c_int64),
        ("q_off_l1", ctypes.c_double),
        ("last_x_l1", ctypes.c_double),
        ("err_bound", ctypes.c_double),
        ("residual_l1", ctypes.c_double),
        ("ms_total", ctypes.c_double),
        ("ws_region", ctypes.c_int32),
        ("ws_accepted", ctypes.c_int32),
        ("ws_resid_ratio", ctypes.c_double),
        ("ws_loss", ctypes.c_double),
        ("ms_warm", ctypes.c_double),
        ("dr_l1", ctypes.c_double),
        ("carry_l1", ctypes.c_double),
        ("fallback", ctypes.c_int32),
        ("flushed", ctypes.c_int32),
        ("ms_delta", ctypes.c_double),
        ("ms_seed", ctypes.c_double),
        ("ms_model", ctypes.c_double),
        ("ms_prop", ctypes.c_double),
        ("ms_merge", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load ``librwr.so``; raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    L = ctypes.CDLL(path)
    p, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.rwr_config_default.argtypes = [ctypes.POINTER(Config)]
    L.rwr_build.argtypes = [ctypes.POINTER(Config), i32, i64, p, p, i32, p, i32, ctypes.POINTER(p)]
    L.rwr_build_vectors.argtypes = [ctypes.POINTER(Config), i32, i64, p, p, i32, p, i32, ctypes.POINTER(p)]
    L.rwr_update.argtypes = [p, ctypes.POINTER(BatchStruct), ctypes.POINTER(StatsStruct)]
    L.rwr_refine.argtypes = [p, ctypes.POINTER(StatsStruct)]
    L.rwr_scores.argtypes = [p, i32, p, i64, i32]
    L.rwr_graph_size.argtypes = [p, ctypes.POINTER(i32), ctypes.POINTER(i64)]
    L.rwr_graph_export.argtypes = [p, p, p, i64, ctypes.POINTER(i64), p]
    L.rwr_last_norms.argtypes = [p, i32, p, i32, ctypes.POINTER(i32)]
    L.rwr_sweep_shape.argtypes = [p, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
    L.rwr_profile.argtypes = [p, i32]
    L.rwr_profile_read.argtypes = [p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), ctypes.POINTER(i64), i32]
    L.rwr_destroy.argtypes = [p]
    L.rwr_destroy.restype = None
    L.rwr_last_error.argtypes = [p]
    L.rwr_last_error.restype = ctypes.c_char_p
    L.rwr_gnn_num_params.argtypes = []
    L.rwr_gnn_num_params.restype = i64
    L.rwr_gnn_eval.argtypes = [p, i32, i32, p, p, p, i64, p, p, p, i64, p, p, p, p, p, p, p, p]
    L.rwr_model_set.argtypes = [p, p, i64]
    L.rwr_model_get.argtypes = [p, p, i64]
    L.rwr_warm_start.argtypes = [p, i32, i32, i64, ctypes.c_float, ctypes.c_float]
    L.rwr_warm_inspect.argtypes = [p, p, p, p, p, p, i64, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.rwr_model_trainable.argtypes = [p, p, i64, i32]
    L.rwr_scores_set.argtypes = [p, i32, p, i64, i32]
    L.rwr_gnn_eval_noalloc.argtypes = [p, i32, i32, p, p, p, i64, p, p, p, i64, p, p, p, p, p, p, p, p, p]
    L.rwr_save.argtypes = [p, ctypes.c_char_p]
    L.rwr_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(Config), ctypes.POINTER(p)]
    L.rwr_context_info.argtypes = [p, ctypes.POINTER(Config), ctypes.POINTER(i32), p]
    for name in EXPORTED:
        f = getattr(L, name)
        if name not in ("rwr_destroy", "rwr_last_error", "rwr_gnn_num_params"):
            f.restype = ctypes.c_int
    _lib = L
    return L


# allocator hooks of rwr_config (dev_alloc / dev_free)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class TorchAllocator:
    """Device memory of a context from torch's caching allocator, on the
    context's own stream.  Keeps the callbacks alive while a context uses
    them; ``live`` counts the blocks the context holds."""

    def __init__(self):
        import torch

        self._torch = torch
        self.device = torch.cuda.current_device()
        self.live = 0
        self.allocs = 0
        self.alloc_fn = ALLOC_FN(self._alloc)
        self.free_fn = FREE_FN(self._free)

    def _alloc(self, nbytes, stream, user):
        try:
            ptr = self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device, int(stream or 0) or None)
        except Exception:  # out of memory: the library reports RWR_ENOMEM
            return None
        self.live += 1
        self.allocs += 1
        return ptr

    def _free(self, ptr, stream, user):
        if ptr:
            self._torch.cuda.caching_allocator_delete(int(ptr))
            self.live -= 1

    def install(self, cfg: "Config") -> None:
        cfg.dev_alloc = ctypes.cast(self.alloc_fn, ctypes.c_void_p)
        cfg.dev_free = ctypes.cast(self.free_fn, ctypes.c_void_p)
        cfg.alloc_user = None


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


class _Arr:
    """Pointer to an int32 array: numpy on the host or a torch CUDA tensor."""

    def __init__(self, a, on_device: bool):
        if a is None:
            self.keep = None
            self.ptr = None
            self.n = 0
        elif on_device:
            import torch

            if not _is_torch(a):
                a = torch.as_tensor(np.asarray(a, dtype=np.int32), device="cuda")
            t = a if a.dtype == torch.int32 else a.to(torch.int32)
            self.keep = t.contiguous()
            self.ptr = self.keep.data_ptr()
            self.n = self.keep.numel()
        else:
            self.keep = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
            self.ptr = self.keep.ctypes.data
            self.n = int(self.keep.shape[0])


def _check(lib, ctx, code: int):
    if code != 0:
        msg = lib.rwr_last_error(ctx)
        raise RwrError(code, msg.decode() if msg else "")


def _make_allocator(kind: Optional[str]):
    if kind is None:
        return None
    if kind == "torch":
        return TorchAllocator()
    raise ValueError(f"unknown allocator {kind!r} (None or 'torch')")


@dataclasses.dataclass
class Update:
    ins_src: object = None
    ins_dst: object = None
    del_src: object = None
    del_dst: object = None
    n_new_nodes: int = 0


class Context:
    """One dynamic-RWR context on the current GPU."""

    def __init__(
        self,
        n: int,
        src,
        dst,
        seeds=None,
        *,
        q=None,
        c: float = 0.15,
        eps: float = 1e-9,
        err_budget: float = 0.0,
        build_tol: float = 0.0,
        precision: str = "fp32",
        undirected: bool = False,
        max_iters: int = 10000,
        pull_ratio: int = 0,
        reorder: bool = True,
        autotune: bool = True,
        stream: Optional[int] = None,
        deterministic: bool = False,
        node_deletion: str = "incident",
        phase_timing: bool = False,
        allocator: Optional[str] = None,
    ):
        self._lib = load_library()
        self._ctx = ctypes.c_void_p(None)
        self.allocator = _make_allocator(allocator)
        cfg = Config()
        self._lib.rwr_config_default(ctypes.byref(cfg))
        cfg.c = c
        cfg.eps = eps
        cfg.err_budget = err_budget
        cfg.build_tol = build_tol
        cfg.precision = {"fp32": 0, "fp64": 1}[precision]
        cfg.undirected = 1 if undirected else 0
        cfg.max_iters = max_iters
        cfg.pull_ratio = pull_ratio
        cfg.reorder = 1 if reorder else 0
        cfg.autotune = 1 if autotune else 0
        cfg.stream = stream
        cfg.deterministic = 1 if deterministic else 0
        cfg.node_deletion = {"incident": 0, "row": 1}[node_deletion]
        cfg.phase_timing = 1 if phase_timing else 0
        if self.allocator is not None:
            self.allocator.install(cfg)
        on_dev = _is_torch(src)
        s = _Arr(src, on_dev)
        d = _Arr(dst, on_dev)
        out = ctypes.c_void_p(None)
        if q is not None:
            # seed vectors: n x S (or n) restart distributions, each summing to 1
            qa = np.asarray(q, dtype=np.float64)
            if qa.ndim == 1:
                qa = qa[:, None]
            qa = np.ascontiguousarray(qa)
            code = self._lib.rwr_build_vectors(
                ctypes.byref(cfg), int(n), s.n, s.ptr, d.ptr, int(qa.shape[1]), qa.ctypes.data, 1 if on_dev else 0,
                ctypes.byref(out),
            )
            sd = np.full(qa.shape[1], -1, np.int32)
        else:
            sd = np.ascontiguousarray(np.asarray(seeds, dtype=np.int32))
            code = self._lib.rwr_build(
                ctypes.byref(cfg), int(n), s.n, s.ptr, d.ptr, int(sd.shape[0]), sd.ctypes.data, 1 if on_dev else 0,
                ctypes.byref(out),
            )
        _check(self._lib, None, code)
        self._ctx = out
        self.n_seeds = int(sd.shape[0])
        self.seeds = sd.copy()
        self.c = c
        self.eps = eps

    # -- checkpoint
    def save(self, path: str) -> None:
        """Write the context's state to ``path`` (rwr_save)."""
        _check(self._lib, self._ctx, self._lib.rwr_save(self._ctx, os.fsencode(path)))

    @classmethod
    def load(cls, path: str, *, stream: Optional[int] = None, allocator: Optional[str] = None,
             phase_timing: bool = False) -> "Context":
        """A context continuing from a checkpoint (rwr_load); the configuration
        comes from the file, except the runtime fields given here."""
        self = cls.__new__(cls)
        self._lib = load_library()
        self._ctx = ctypes.c_void_p(None)
        self.allocator = _make_allocator(allocator)
        rt = Config()
        self._lib.rwr_config_default(ctypes.byref(rt))
        rt.stream = stream
        rt.phase_timing = 1 if phase_timing else 0
        if self.allocator is not None:
            self.allocator.install(rt)
        out = ctypes.c_void_p(None)
        _check(self._lib, None, self._lib.rwr_load(os.fsencode(path), ctypes.byref(rt), ctypes.byref(out)))
        self._ctx = out
        cfg = Config()
        ns = ctypes.c_int32(0)
        sd = np.zeros(64, np.int32)
        _check(self._lib, self._ctx, self._lib.rwr_context_info(self._ctx, ctypes.byref(cfg), ctypes.byref(ns),
                                                                sd.ctypes.data))
        self.n_seeds = int(ns.value)
        self.seeds = sd[: self.n_seeds].copy()
        self.c = cfg.c
        self.eps = cfg.eps
        return self

    def config(self) -> dict:
        cfg = Config()
        _check(self._lib, self._ctx, self._lib.rwr_context_info(self._ctx, ctypes.byref(cfg), None, None))
        return {f: getattr(cfg, f) for f, _ in Config._fields_}

    # -- lifetime
    def close(self):
        if self._ctx:
            self._lib.rwr_destroy(self._ctx)
            self._ctx = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- updates
    def update(self, ins_src=None, ins_dst=None, del_src=None, del_dst=None, n_new_nodes: int = 0,
               del_nodes=None) -> dict:
        arrays = (ins_src, ins_dst, del_src, del_dst, del_nodes)
        on_dev = any(_is_torch(x) for x in arrays if x is not None)
        a = [_Arr(x, on_dev) for x in arrays]
        if a[0].n != a[1].n or a[2].n != a[3].n:
            raise ValueError("source and destination arrays differ in length")
        b = BatchStruct()
        b.n_ins = a[0].n
        b.ins_src, b.ins_dst = a[0].ptr, a[1].ptr
        b.n_del = a[2].n
        b.del_src, b.del_dst = a[2].ptr, a[3].ptr
        b.n_new_nodes = int(n_new_nodes)
        b.n_del_nodes = a[4].n
        b.del_nodes = a[4].ptr
        b.on_device = 1 if on_dev else 0
        st = StatsStruct()
        code = self._lib.rwr_update(self._ctx, ctypes.byref(b), ctypes.byref(st))
        _check(self._lib, self._ctx, code)
        return st.as_dict()

    def update_batch(self, batch) -> dict:
        return self.update(batch.ins_src, batch.ins_dst, batch.del_src, batch.del_dst, batch.n_new_nodes,
                           getattr(batch, "del_nodes", None))

    # -- learned warm start
    def model_set(self, params) -> None:
        th = np.ascontiguousarray(np.asarray(params, np.float32))
        _check(self._lib, self._ctx, self._lib.rwr_model_set(self._ctx, th.ctypes.data, th.shape[0]))

    def model_get(self) -> np.ndarray:
        n = int(self._lib.rwr_gnn_num_params())
        out = np.zeros(n, np.float32)
        _check(self._lib, self._ctx, self._lib.rwr_model_get(self._ctx, out.ctypes.data, n))
        return out

    def model_trainable(self, mask=None, warmup: int = 0) -> None:
        """Parameters the optimiser steps (mask 1) or holds (0); None: all.
        warmup: steps of linear step-size warm-up."""
        if mask is None:
            _check(self._lib, self._ctx, self._lib.rwr_model_trainable(self._ctx, None, 0, int(warmup)))
            return
        mk = np.ascontiguousarray(np.asarray(mask, np.float32))
        _check(self._lib, self._ctx, self._lib.rwr_model_trainable(self._ctx, mk.ctypes.data, mk.shape[0],
                                                                    int(warmup)))

    def warm_start(self, mode: str = "predict", hops: int = 3, max_rows: int = 0, lr: float = 1e-5,
                   weight_decay: float = 1e-4) -> None:
        """mode: 'off', 'predict', 'train' or 'predict+train'."""
        m = {"off": 0, "predict": 1, "train": 2, "predict+train": 3}[mode]
        _check(self._lib, self._ctx, self._lib.rwr_warm_start(self._ctx, m, int(hops), int(max_rows), float(lr),
                                                               float(weight_decay)))

    def warm_inspect(self, with_grad: bool = True) -> dict:
        """What the warm start of the last update computed: region nodes (in
        the network's row order) and their hops, the output o and dL/do
        (region node x padded seed columns) and the parameter gradient of
        its training step (when with_grad)."""
        nR = ctypes.c_int32(0)
        cols = ctypes.c_int32(0)
        _check(self._lib, self._ctx, self._lib.rwr_warm_inspect(self._ctx, None, None, None, None, None, 0,
                                                                 ctypes.byref(nR), ctypes.byref(cols)))
        n, S = nR.value, cols.value
        nodes = np.zeros(n, np.int32)
        hops = np.zeros(n, np.int32)
        o = np.zeros((n, S), np.float32)
        dout = np.zeros((n, S), np.float32)
        grad = np.zeros(int(self._lib.rwr_gnn_num_params()), np.float32)
        if n:
            _check(self._lib, self._ctx, self._lib.rwr_warm_inspect(
                self._ctx, nodes.ctypes.data, hops.ctypes.data, o.ctypes.data,
                dout.ctypes.data if with_grad else None, grad.ctypes.data if with_grad else None, n,
                ctypes.byref(nR), ctypes.byref(cols)))
        return {"nodes": nodes, "hops": hops, "o": o, "dout": dout, "grad": grad}

    def refine(self) -> dict:
        st = StatsStruct()
        _check(self._lib, self._ctx, self._lib.rwr_refine(self._ctx, ctypes.byref(st)))
        return st.as_dict()

    # -- queries
    @property
    def n(self) -> int:
        n = ctypes.c_int32(0)
        m = ctypes.c_int64(0)
        _check(self._lib, self._ctx, self._lib.rwr_graph_size(self._ctx, ctypes.byref(n), ctypes.byref(m)))
        return n.value

    @property
    def m(self) -> int:
        """Stored directed edges (an undirected pair counts twice, a self-loop once)."""
        n = ctypes.c_int32(0)
        m = ctypes.c_int64(0)
        _check(self._lib, self._ctx, self._lib.rwr_graph_size(self._ctx, ctypes.byref(n), ctypes.byref(m)))
        return m.value

    def sweep_shape(self) -> dict:
        lanes = ctypes.c_int32(0)
        groups = ctypes.c_int32(0)
        ms = ctypes.c_double(0.0)
        _check(self._lib, self._ctx, self._lib.rwr_sweep_shape(self._ctx, ctypes.byref(lanes), ctypes.byref(groups),
                                                                ctypes.byref(ms)))
        return {"lanes_per_row": lanes.value, "workgroups": groups.value, "tuned_ms": ms.value}

    def scores(self, j: int = 0) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.float64)
        _check(self._lib, self._ctx, self._lib.rwr_scores(self._ctx, int(j), out.ctypes.data, out.shape[0], 0))
        return out

    def scores_set(self, j: int, values) -> None:
        """Replace column j's scores (normalised, caller ids); see rwr_scores_set."""
        v = np.ascontiguousarray(np.asarray(values, np.float64))
        _check(self._lib, self._ctx, self._lib.rwr_scores_set(self._ctx, int(j), v.ctypes.data, v.shape[0], 0))

    def scores_device(self, j: int, out) -> None:
        """Write column j into a float64 CUDA tensor of at least n elements."""
        _check(self._lib, self._ctx, self._lib.rwr_scores(self._ctx, int(j), out.data_ptr(), out.numel(), 1))

    def export(self):
        m = ctypes.c_int64(0)
        n = self.n
        deg = np.zeros(n, dtype=np.int32)
        _check(self._lib, self._ctx,
               self._lib.rwr_graph_export(self._ctx, None, None, 0, ctypes.byref(m), deg.ctypes.data))
        src = np.zeros(m.value, dtype=np.int32)
        dst = np.zeros(m.value, dtype=np.int32)
        _check(self._lib, self._ctx,
               self._lib.rwr_graph_export(self._ctx, src.ctypes.data, dst.ctypes.data, m.value, ctypes.byref(m),
                                          None))
        return src, dst, deg

    def profile(self, enable: bool = True) -> None:
        _check(self._lib, self._ctx, self._lib.rwr_profile(self._ctx, 1 if enable else 0))

    def profile_read(self, reset: bool = False) -> dict:
        ms = ctypes.c_double(0.0)
        sweeps = ctypes.c_int64(0)
        idle = ctypes.c_int64(0)
        _check(self._lib, self._ctx, self._lib.rwr_profile_read(self._ctx, ctypes.byref(ms), ctypes.byref(sweeps),
                                                                ctypes.byref(idle), 1 if reset else 0))
        return {"dense_ms": ms.value, "dense_sweeps": sweeps.value, "idle_launches": idle.value}

    def last_norms(self, j: int = 0) -> np.ndarray:
        ln = ctypes.c_int32(0)
        self._lib.rwr_last_norms(self._ctx, int(j), None, 0, ctypes.byref(ln))
        out = np.zeros(ln.value, dtype=np.float64)
        _check(self._lib, self._ctx,
               self._lib.rwr_last_norms(self._ctx, int(j), out.ctypes.data, ln.value, ctypes.byref(ln)))
        return out


def _csr(n: int, a: np.ndarray, b: np.ndarray):
    """Rows of the edges (a[e], b[e]) grouped by a, in edge order: off, len, adj."""
    a = np.asarray(a, np.int64)
    b = np.asarray(b, np.int32)
    order = np.argsort(a, kind="stable")
    cnt = np.bincount(a, minlength=n).astype(np.int32)
    off = np.concatenate([[0], np.cumsum(cnt)[:-1]]).astype(np.int32)
    return off, cnt, np.ascontiguousarray(b[order])


def gnn_eval(params, nR: int, S: int, src, dst, dinv, feats, target=None, active=None, *, adam_step: bool = False,
             noalloc: bool = False, stream: Optional[int] = None):
    """Run the warm-start network on one explicit region (see rwr_gnn_eval).

    ``src``/``dst`` are the region's edges u -> v in local ids.  Returns a
    dict with ``out`` (nR, S) and, with a target, ``loss``, ``grad`` and (if
    ``adam_step``) ``params_after``.  ``noalloc`` calls
    rwr_gnn_eval_noalloc instead (no device allocation; on ``stream``, a
    hipStream_t handle, or the default stream)."""
    L = load_library()
    P = int(L.rwr_gnn_num_params())
    th = np.ascontiguousarray(np.asarray(params, np.float32))
    if th.shape != (P,):
        raise ValueError(f"expected {P} parameters")
    in_off, in_len, in_adj = _csr(nR, dst, src)   # in-row of v lists its sources u
    out_off, out_len, out_adj = _csr(nR, src, dst)
    dv = np.ascontiguousarray(np.asarray(dinv, np.float32))
    F = np.ascontiguousarray(np.asarray(feats, np.float32).reshape(nR * S, -1))
    out = np.zeros(nR * S, np.float32)
    res = {}
    tg = act = grad = loss = after = None
    if target is not None:
        tg = np.ascontiguousarray(np.asarray(target, np.float32).reshape(-1))
        act = np.ascontiguousarray(np.asarray(active, np.int32))
        grad = np.zeros(P, np.float32)
        loss = ctypes.c_double(0.0)
        if adam_step:
            after = np.zeros(P, np.float32)

    def ptr(x):
        return None if x is None else x.ctypes.data

    args = (
        ptr(th), int(nR), int(S), ptr(in_off), ptr(in_len), ptr(in_adj), int(in_adj.shape[0]), ptr(out_off),
        ptr(out_len), ptr(out_adj), int(out_adj.shape[0]), ptr(dv), ptr(F), ptr(tg), ptr(act), ptr(out),
        ptr(grad), ctypes.byref(loss) if loss is not None else None, ptr(after),
    )
    if noalloc:
        code = L.rwr_gnn_eval_noalloc(*args, stream)
    else:
        code = L.rwr_gnn_eval(*args)
    _check(L, None, code)
    res["out"] = out.reshape(nR, S)
    if target is not None:
        res["loss"] = loss.value
        res["grad"] = grad
        if adam_step:
            res["params_after"] = after
    return res
