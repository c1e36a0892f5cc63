"""Python binding of libdumato_mi (C ABI in include/dm.h).

Argument marshalling only: every step of the counting path runs in the HIP
library.  The raw entry points are exposed under their C names
(``dm_load_csr``, ``dm_count_cliques``, ``dm_count_motifs``, ``dm_batch``, ...)
and wrapped by small helpers that accept numpy arrays or torch tensors.  torch
is used for device memory and streams only.

If the shared library has not been built, importing the helpers raises
``ImportError`` — there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libdumato_mi.so")

DM_OK, DM_E_ARG, DM_E_CSR, DM_E_K, DM_E_OVERFLOW, DM_E_NOMEM, DM_E_HIP, DM_E_BUFSZ, DM_E_MODEL = range(9)
DM_CSR_HOST, DM_CSR_DEVICE, DM_CSR_TRUSTED, DM_CSR_ORIENT, DM_CSR_RANK = 0, 1, 2, 4, 8
DM_SCHED_PLAIN, DM_SCHED_LEARNED, DM_SCHED_AUTOTUNE, DM_RECORD_ROOTS, DM_NO_DONATION = 0, 1, 2, 4, 8
DM_SCHED_COST = 16
DM_IMPL_DFS = 32
DM_SCHED_HOST_BALANCE = 64
DM_OP_CLIQUE, DM_OP_MOTIF = 0, 1
DM_PATTERN_INDUCED, DM_PATTERN_DIRECTED = 1, 2
DM_MLP_NET = 4 * 64 + 64 + 64 * 64 + 64 + 64 + 1  # 4 -> 64 -> 64 -> 1 weights
DM_MLP_NPARAMS = DM_MLP_NET + 8                     # + feature mean[4], std[4]

EXPORTS = [
    "dm_load_csr", "dm_free", "dm_graph_info", "dm_count_cliques", "dm_motif_num_classes",
    "dm_motif_class_mask", "dm_motif_class_table", "dm_motif_class_table16", "dm_count_motifs",
    "dm_count_motifs_static", "dm_batch", "dm_list", "dm_induced_subgraph", "dm_count_quasi_cliques",
    "dm_load_digraph", "dm_digraph_info", "dm_motif_directed_num_classes", "dm_motif_directed_class_code",
    "dm_motif_directed_class_table", "dm_count_motifs_directed", "dm_count_pattern",
    "dm_strerror", "dm_last_error", "dm_last_launch_count", "dm_features", "dm_mlp_init", "dm_mlp_fit_normalizer",
    "dm_mlp_forward", "dm_mlp_targets", "dm_mlp_loss_grad", "dm_mlp_adam_step", "dm_mlp_train", "dm_autotune",
]


class dm_tuning(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_uint32), ("rebalance", ctypes.c_float), ("waves_per_cu", ctypes.c_uint32),
                ("ms", ctypes.c_float)]


class dm_options(ctypes.Structure):
    _fields_ = [
        ("size", ctypes.c_uint32),
        ("sched", ctypes.c_uint32),
        ("stream", ctypes.c_void_p),
        ("chunk", ctypes.c_uint32),
        ("rebalance", ctypes.c_float),
        ("waves_per_cu", ctypes.c_uint32),
        ("mlp", ctypes.c_void_p),
        ("roots", ctypes.c_void_p),
        ("num_roots", ctypes.c_int64),
        ("root_stats", ctypes.c_void_p),
        ("wave_stats", ctypes.c_void_p),
        ("wave_stats_len", ctypes.c_uint32),
        ("counter_bias", ctypes.c_uint64),
        ("wait_limit_us", ctypes.c_uint32),
        ("root_cost", ctypes.c_void_p),
    ]


# void (*dm_sink_fn)(const int32_t* rows, uint64_t nrows, int width, void* user)
SINK_FN = ctypes.CFUNCTYPE(None, ctypes.POINTER(ctypes.c_int32), ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p)


class DMError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


_lib = None


def lib():
    """Load the shared library (raises ImportError when it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2212_04551_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    L.dm_load_csr.restype = ctypes.c_int
    L.dm_load_csr.argtypes = [i32, vp, vp, u32, vp, ctypes.POINTER(vp)]
    L.dm_free.restype = None
    L.dm_free.argtypes = [vp]
    L.dm_graph_info.restype = ctypes.c_int
    L.dm_graph_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64)]
    L.dm_count_cliques.restype = ctypes.c_int
    L.dm_count_cliques.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(dm_options)]
    L.dm_motif_num_classes.restype = ctypes.c_int
    L.dm_motif_num_classes.argtypes = [ctypes.c_int]
    L.dm_motif_class_mask.restype = ctypes.c_int
    L.dm_motif_class_mask.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(u32)]
    L.dm_motif_class_table.restype = ctypes.c_int
    L.dm_motif_class_table.argtypes = [ctypes.c_int, vp, ctypes.c_size_t]
    L.dm_motif_class_table16.restype = ctypes.c_int
    L.dm_motif_class_table16.argtypes = [ctypes.c_int, vp, ctypes.c_size_t]
    L.dm_count_motifs.restype = ctypes.c_int
    L.dm_count_motifs.argtypes = [vp, ctypes.c_int, vp, ctypes.c_size_t, ctypes.POINTER(dm_options)]
    L.dm_count_motifs_static.restype = ctypes.c_int
    L.dm_count_motifs_static.argtypes = [vp, ctypes.c_int, vp, ctypes.c_size_t, ctypes.POINTER(dm_options)]
    L.dm_list.restype = ctypes.c_int
    L.dm_list.argtypes = [vp, ctypes.c_int, ctypes.c_int, SINK_FN, vp, ctypes.POINTER(ctypes.c_uint64),
                          ctypes.POINTER(dm_options)]
    L.dm_induced_subgraph.restype = ctypes.c_int
    L.dm_induced_subgraph.argtypes = [vp, vp, vp, ctypes.POINTER(vp)]
    L.dm_load_digraph.restype = ctypes.c_int
    L.dm_load_digraph.argtypes = [i32, vp, vp, u32, vp, ctypes.POINTER(vp)]
    L.dm_digraph_info.restype = ctypes.c_int
    L.dm_digraph_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64)]
    L.dm_motif_directed_num_classes.restype = i32
    L.dm_motif_directed_num_classes.argtypes = [ctypes.c_int]
    L.dm_motif_directed_class_code.restype = ctypes.c_int
    L.dm_motif_directed_class_code.argtypes = [ctypes.c_int, i32, ctypes.POINTER(u32)]
    L.dm_motif_directed_class_table.restype = ctypes.c_int
    L.dm_motif_directed_class_table.argtypes = [ctypes.c_int, vp, ctypes.c_size_t]
    L.dm_count_motifs_directed.restype = ctypes.c_int
    L.dm_count_motifs_directed.argtypes = [vp, ctypes.c_int, vp, ctypes.c_size_t, ctypes.POINTER(dm_options)]
    L.dm_count_pattern.restype = ctypes.c_int
    L.dm_count_pattern.argtypes = [vp, ctypes.c_int, u32, u32, ctypes.POINTER(ctypes.c_uint64),
                                   ctypes.POINTER(dm_options)]
    L.dm_count_quasi_cliques.restype = ctypes.c_int
    L.dm_count_quasi_cliques.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.POINTER(dm_options)]
    L.dm_batch.restype = ctypes.c_int
    L.dm_batch.argtypes = [ctypes.POINTER(vp), i32, ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t,
                           ctypes.POINTER(dm_options)]
    L.dm_last_launch_count.restype = ctypes.c_int
    L.dm_last_launch_count.argtypes = []
    L.dm_strerror.restype = ctypes.c_char_p
    L.dm_strerror.argtypes = [ctypes.c_int]
    L.dm_last_error.restype = ctypes.c_char_p
    L.dm_last_error.argtypes = []
    for name, args in (
        ("dm_features", [vp, vp, vp]),
        ("dm_mlp_init", [vp, ctypes.c_uint64, vp]),
        ("dm_mlp_fit_normalizer", [vp, vp, i64, vp]),
        ("dm_mlp_forward", [vp, vp, i64, vp, vp]),
        ("dm_mlp_targets", [vp, i64, vp, vp]),
        ("dm_mlp_loss_grad", [vp, vp, vp, i64, vp, ctypes.POINTER(ctypes.c_float), vp]),
        ("dm_mlp_adam_step", [vp, vp, vp, vp, i64, ctypes.c_float, vp]),
        ("dm_mlp_train", [vp, vp, vp, i64, ctypes.c_int, ctypes.c_int, ctypes.c_float, ctypes.c_uint64, vp, vp]),
        ("dm_autotune", [ctypes.POINTER(vp), i32, ctypes.c_int, ctypes.c_int, ctypes.POINTER(dm_options),
                         ctypes.POINTER(dm_tuning)]),
    ):
        f = getattr(L, name)
        f.restype = ctypes.c_int
        f.argtypes = args
    _lib = L
    return L


def _check(status: int):
    if status != DM_OK:
        L = lib()
        msg = L.dm_strerror(status).decode()
        detail = L.dm_last_error().decode()
        raise DMError(status, f"{msg}: {detail}" if detail else msg)


def _ptr(x) -> Optional[int]:
    """Address of a numpy array or torch tensor (None passes through)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, int):
        return x
    raise TypeError(f"cannot take the address of {type(x)}")


def _stream(s) -> Optional[int]:
    if s is None:
        return None
    if hasattr(s, "cuda_stream"):
        return s.cuda_stream
    return int(s)


def make_options(sched: int = 0, stream=None, chunk: int = 0, rebalance: float = 0.0, waves_per_cu: int = 0,
                 mlp=None, roots=None, root_stats=None, wave_stats=None, counter_bias: int = 0,
                 wait_limit_us: int = 0, root_cost=None):
    """Build a dm_options struct; returns (struct, keep-alive list)."""
    keep = []
    o = dm_options()
    o.size = ctypes.sizeof(dm_options)
    o.sched = sched
    o.stream = _stream(stream)
    o.chunk = chunk
    o.rebalance = rebalance
    o.waves_per_cu = waves_per_cu
    o.mlp = _ptr(mlp)
    if roots is not None:
        r = np.ascontiguousarray(roots, dtype=np.int32)
        keep.append(r)
        o.roots = r.ctypes.data
        o.num_roots = r.size
    if root_stats is not None:
        o.root_stats = _ptr(root_stats)
        o.sched |= DM_RECORD_ROOTS
    if wave_stats is not None:
        o.wave_stats = _ptr(wave_stats)
        o.wave_stats_len = int(wave_stats.numel() // 4) if hasattr(wave_stats, "numel") else int(wave_stats.size // 4)
    o.counter_bias = counter_bias
    o.wait_limit_us = wait_limit_us
    if root_cost is not None:
        o.root_cost = _ptr(root_cost)
        o.sched |= DM_SCHED_COST
    keep.append(mlp)
    keep.append(root_cost)
    return o, keep


class DMGraph:
    """A graph loaded into the library (owns the dm_graph handle)."""

    def __init__(self, handle: int):
        self.handle = ctypes.c_void_p(handle)
        n = ctypes.c_int32(0)
        nnz = ctypes.c_int64(0)
        _check(lib().dm_graph_info(self.handle, ctypes.byref(n), ctypes.byref(nnz)))
        self.n, self.nnz = n.value, nnz.value

    def close(self):
        if self.handle:
            lib().dm_free(self.handle)
            self.handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def load_csr(n: int, row_ptr, col, device: bool = False, trusted: bool = False, stream=None,
             orient: bool = False, rank: bool = False) -> DMGraph:
    """dm_load_csr on numpy arrays (host) or torch CUDA tensors (device=True)."""
    if not device:
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        if col.size == 0:
            col = np.zeros(1, dtype=np.int32)
    flags = (DM_CSR_DEVICE if device else DM_CSR_HOST) | (DM_CSR_TRUSTED if trusted else 0)
    flags |= DM_CSR_ORIENT if orient else 0
    flags |= DM_CSR_RANK if rank else 0
    h = ctypes.c_void_p(None)
    _check(lib().dm_load_csr(n, _ptr(row_ptr), _ptr(col), flags, _stream(stream), ctypes.byref(h)))
    return DMGraph(h.value)


def graph_info(g: DMGraph):
    """(n, nnz) of a loaded graph."""
    n = ctypes.c_int32(0)
    nnz = ctypes.c_int64(0)
    _check(lib().dm_graph_info(g.handle, ctypes.byref(n), ctypes.byref(nnz)))
    return int(n.value), int(nnz.value)


def load_graph(g, **kw) -> DMGraph:
    """Load a graphgen.Graph (host arrays)."""
    return load_csr(g.n, g.row_ptr, g.col, **kw)


def _check_stats(g: DMGraph, opt: dict):
    st = opt.get("root_stats")
    if st is None:
        return
    rows = len(opt["roots"]) if opt.get("roots") is not None else g.n
    size = st.numel() if hasattr(st, "numel") else st.size
    if size < 3 * rows:
        raise ValueError(f"root_stats needs {3 * rows} uint64 entries, got {size}")


def count_cliques(g: DMGraph, k: int, **opt) -> int:
    _check_stats(g, opt)
    o, keep = make_options(**opt)
    out = ctypes.c_uint64(0)
    _check(lib().dm_count_cliques(g.handle, k, ctypes.byref(out), ctypes.byref(o)))
    del keep
    return int(out.value)


def last_launch_count() -> int:
    """Kernel launches of this thread's last counting call (host-driven balancing relaunches)."""
    return int(lib().dm_last_launch_count())


def motif_num_classes(k: int) -> int:
    return int(lib().dm_motif_num_classes(k))


def motif_class_mask(k: int, cls: int) -> int:
    m = ctypes.c_uint32(0)
    _check(lib().dm_motif_class_mask(k, cls, ctypes.byref(m)))
    return int(m.value)


def motif_class_table(k: int) -> np.ndarray:
    if not 3 <= k <= 6:
        _check(lib().dm_motif_class_table(k, None, 0))  # raises DM_E_K
    n = 1 << (k * (k - 1) // 2 - 1)
    out = np.zeros(n, dtype=np.uint8)
    _check(lib().dm_motif_class_table(k, out.ctypes.data, n))
    return out


def motif_class_table16(k: int) -> np.ndarray:
    if motif_num_classes(k) < 0:
        _check(lib().dm_motif_class_table16(k, None, 0))  # raises DM_E_K
    n = 1 << (k * (k - 1) // 2 - 1)
    out = np.zeros(n, dtype=np.uint16)
    _check(lib().dm_motif_class_table16(k, out.ctypes.data, n))
    return out


def count_motifs(g: DMGraph, k: int, **opt) -> np.ndarray:
    ncls = motif_num_classes(k)
    if ncls < 0:
        _check(DM_E_K)
    out = np.zeros(ncls, dtype=np.uint64)
    _check_stats(g, opt)
    o, keep = make_options(**opt)
    _check(lib().dm_count_motifs(g.handle, k, out.ctypes.data, ncls, ctypes.byref(o)))
    del keep
    return out


def count_motifs_static(g: DMGraph, k: int, **opt) -> np.ndarray:
    """dm_count_motifs_static: the motif count with no device allocation."""
    ncls = motif_num_classes(k)
    if ncls < 0:
        _check(DM_E_K)
    out = np.zeros(ncls, dtype=np.uint64)
    _check_stats(g, opt)
    o, keep = make_options(**opt)
    _check(lib().dm_count_motifs_static(g.handle, k, out.ctypes.data, ncls, ctypes.byref(o)))
    del keep
    return out


def list_subgraphs(g: DMGraph, op: int, k: int, sink=None, **opt):
    """dm_list (aggregate_store).  With no `sink`, returns every row as one
    int32 array [rows, width] (cliques: k vertex ids; motifs: k vertex ids in
    traversal order, then the class id).  With a `sink(rows)` callable, hands
    it each batch (a numpy view valid only during the call) and returns the
    row count."""
    parts = []

    def _cb(ptr, nrows, width, _user):
        arr = np.ctypeslib.as_array(ptr, shape=(int(nrows), int(width)))
        if sink is None:
            parts.append(arr.copy())
        else:
            sink(arr)

    cb = SINK_FN(_cb)
    total = ctypes.c_uint64(0)
    o, keep = make_options(**opt)
    _check(lib().dm_list(g.handle, op, k, cb, None, ctypes.byref(total), ctypes.byref(o)))
    del keep
    if sink is not None:
        return int(total.value)
    width = k if op == DM_OP_CLIQUE else k + 1
    out = np.concatenate(parts) if parts else np.zeros((0, width), dtype=np.int32)
    assert out.shape[0] == total.value
    return out


def induced_subgraph(g: DMGraph, keep, stream=None) -> DMGraph:
    """dm_induced_subgraph: the subgraph on the vertices with keep[v] (host bool / uint8 array)."""
    k = np.ascontiguousarray(np.asarray(keep, dtype=np.uint8))
    h = ctypes.c_void_p(None)
    _check(lib().dm_induced_subgraph(g.handle, k.ctypes.data if k.size else None, _stream(stream), ctypes.byref(h)))
    return DMGraph(h.value)


def count_quasi_cliques(g: DMGraph, k: int, min_edges: int, **opt) -> int:
    """dm_count_quasi_cliques: connected induced k-subgraphs with >= min_edges edges."""
    o, keep = make_options(**opt)
    out = ctypes.c_uint64(0)
    _check(lib().dm_count_quasi_cliques(g.handle, k, min_edges, ctypes.byref(out), ctypes.byref(o)))
    del keep
    return int(out.value)


def batch(graphs: Sequence[DMGraph], op: int, k: int, **opt) -> np.ndarray:
    """dm_batch: returns [num_graphs, width] uint64."""
    width = 1 if op == DM_OP_CLIQUE else motif_num_classes(k)
    if width < 0:
        _check(DM_E_K)
    arr = (ctypes.c_void_p * len(graphs))(*[g.handle.value for g in graphs])
    out = np.zeros((len(graphs), width), dtype=np.uint64)
    o, keep = make_options(**opt)
    _check(lib().dm_batch(arr, len(graphs), op, k, out.ctypes.data, out.size, ctypes.byref(o)))
    del keep
    return out


def autotune(graphs: Sequence[DMGraph], op: int, k: int, **opt) -> dict:
    """dm_autotune over one graph or a batch; returns the chosen knobs."""
    arr = (ctypes.c_void_p * len(graphs))(*[g.handle.value for g in graphs])
    o, keep = make_options(**opt)
    t = dm_tuning()
    _check(lib().dm_autotune(arr, len(graphs), op, k, ctypes.byref(o), ctypes.byref(t)))
    del keep
    return {"chunk": t.chunk, "rebalance": float(t.rebalance), "waves_per_cu": t.waves_per_cu, "ms": float(t.ms)}


# ------------------------------------------------------------------ learned ordering
# Device buffers are torch CUDA tensors: features int64 [n, 4], parameters
# float32 [DM_MLP_NPARAMS], predictions / targets float32 [n].

def _cur_stream(stream):
    if stream is not None:
        return _stream(stream)
    import torch
    return torch.cuda.current_stream().cuda_stream


def features(g: DMGraph, stream=None):
    import torch
    out = torch.empty((g.n, 4), dtype=torch.int64, device="cuda")
    _check(lib().dm_features(g.handle, out.data_ptr(), _cur_stream(stream)))
    return out


def mlp_new(seed: int = 0, stream=None):
    import torch
    p = torch.empty(DM_MLP_NPARAMS, dtype=torch.float32, device="cuda")
    _check(lib().dm_mlp_init(p.data_ptr(), seed, _cur_stream(stream)))
    return p


def mlp_fit_normalizer(params, feats, stream=None):
    _check(lib().dm_mlp_fit_normalizer(params.data_ptr(), feats.data_ptr(), feats.shape[0], _cur_stream(stream)))


def mlp_forward(params, feats, stream=None):
    import torch
    out = torch.empty(feats.shape[0], dtype=torch.float32, device="cuda")
    _check(lib().dm_mlp_forward(params.data_ptr(), feats.data_ptr(), feats.shape[0], out.data_ptr(),
                                _cur_stream(stream)))
    return out


def mlp_targets(root_stats, stream=None):
    import torch
    n = root_stats.shape[0]
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    _check(lib().dm_mlp_targets(root_stats.data_ptr(), n, out.data_ptr(), _cur_stream(stream)))
    return out


def mlp_loss_grad(params, feats, targets, stream=None):
    import torch
    grad = torch.empty(DM_MLP_NET, dtype=torch.float32, device="cuda")
    loss = ctypes.c_float(0.0)
    _check(lib().dm_mlp_loss_grad(params.data_ptr(), feats.data_ptr(), targets.data_ptr(), feats.shape[0],
                                  grad.data_ptr(), ctypes.byref(loss), _cur_stream(stream)))
    return float(loss.value), grad


def mlp_adam_step(params, grad, m, v, t: int, lr: float, stream=None):
    _check(lib().dm_mlp_adam_step(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), t, lr,
                                  _cur_stream(stream)))


def mlp_train(params, feats, targets, epochs: int, batch: int = 4096, lr: float = 1e-3, seed: int = 0,
              stream=None) -> np.ndarray:
    hist = np.zeros(max(epochs, 1), dtype=np.float32)
    _check(lib().dm_mlp_train(params.data_ptr(), feats.data_ptr(), targets.data_ptr(), feats.shape[0], epochs,
                              batch, lr, seed, hist.ctypes.data, _cur_stream(stream)))
    return hist[:epochs]


# C names re-exported for callers that want the raw ABI
def __getattr__(name):
    if name in EXPORTS:
        return getattr(lib(), name)
    raise AttributeError(name)


# ------------------------------------------------------------------ directed graphs

def load_digraph_csr(n: int, row_ptr, col, device: bool = False, trusted: bool = False, stream=None,
                     orient: bool = False, rank: bool = False) -> DMGraph:
    """dm_load_digraph: arcs as sorted out-lists (numpy, or torch CUDA tensors with device=True)."""
    if not device:
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        if col.size == 0:
            col = np.zeros(1, dtype=np.int32)
    flags = (DM_CSR_DEVICE if device else DM_CSR_HOST) | (DM_CSR_TRUSTED if trusted else 0)
    flags |= DM_CSR_ORIENT if orient else 0
    flags |= DM_CSR_RANK if rank else 0
    h = ctypes.c_void_p(None)
    _check(lib().dm_load_digraph(n, _ptr(row_ptr), _ptr(col), flags, _stream(stream), ctypes.byref(h)))
    return DMGraph(h.value)


def load_digraph(d, **kw) -> DMGraph:
    """Load a graphgen.Digraph (host arrays)."""
    return load_digraph_csr(d.n, d.row_ptr, d.col, **kw)


def load_digraph_device(n: int, row_ptr, col, **kw) -> DMGraph:
    return load_digraph_csr(n, row_ptr, col, device=True, **kw)


def digraph_info(g: DMGraph):
    """(1, arcs) for a digraph handle, (0, 0) otherwise."""
    d = ctypes.c_int32(0)
    a = ctypes.c_int64(0)
    _check(lib().dm_digraph_info(g.handle, ctypes.byref(d), ctypes.byref(a)))
    return int(d.value), int(a.value)


def motif_directed_num_classes(k: int) -> int:
    return int(lib().dm_motif_directed_num_classes(k))


def motif_directed_class_code(k: int, cls: int) -> int:
    c = ctypes.c_uint32(0)
    _check(lib().dm_motif_directed_class_code(k, cls, ctypes.byref(c)))
    return int(c.value)


def motif_directed_class_table(k: int) -> np.ndarray:
    """Class of every directed code on k vertices (0xFFFF: not weakly connected)."""
    if motif_directed_num_classes(k) < 0:
        _check(lib().dm_motif_directed_class_table(k, None, 0))
    out = np.zeros(1 << (k * (k - 1)), dtype=np.uint16)
    _check(lib().dm_motif_directed_class_table(k, out.ctypes.data, out.size))
    return out


def count_motifs_directed(g: DMGraph, k: int, **opt) -> np.ndarray:
    """dm_count_motifs_directed: per-class counts of weakly connected induced k-subdigraphs."""
    nc = motif_directed_num_classes(k)
    out = np.zeros(max(nc, 1), dtype=np.uint64)
    o, keep = make_options(**opt)
    _check(lib().dm_count_motifs_directed(g.handle, k, out.ctypes.data, out.size if nc > 0 else 0, ctypes.byref(o)))
    del keep
    return out[:nc]


def count_pattern(g: DMGraph, k: int, code: int, induced: bool = False, directed: bool = False, **opt) -> int:
    """dm_count_pattern: copies of a connected pattern (its pair-bitmap code on k vertices)."""
    flags = (DM_PATTERN_INDUCED if induced else 0) | (DM_PATTERN_DIRECTED if directed else 0)
    out = ctypes.c_uint64(0)
    o, keep = make_options(**opt)
    _check(lib().dm_count_pattern(g.handle, k, ctypes.c_uint32(code), flags, ctypes.byref(out), ctypes.byref(o)))
    del keep
    return int(out.value)
