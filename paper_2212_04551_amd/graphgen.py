"""Seeded synthetic input graphs.

This module is the input side only: it draws graphs and builds CSR arrays and
holds none of the enumeration arithmetic.  The random families (G(n,m),
Chung-Lu, preferential attachment, planted-partition SBM) run in a small C
library (``gen/graphgen.c``); the structured families with known subgraph
counts (complete, bipartite, multipartite, paths, cycles, stars, hypercubes)
are written here with numpy.

Every graph is returned as :class:`Graph` — an undirected simple graph in CSR
form with ``row_ptr`` int64 of length n+1 and ``col`` int32 of length nnz,
each adjacency list sorted strictly ascending.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Iterable, List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen", "graphgen.c")
_LIB_PATH = os.path.join(_HERE, "gen", "libgraphgen.so")
_lib = None


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # int64, n+1
    col: np.ndarray  # int32, nnz

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def neighbors(self, v: int) -> np.ndarray:
        return self.col[self.row_ptr[v]:self.row_ptr[v + 1]]


def build_library(force: bool = False) -> str:
    """Compile the generator library with gcc (in-tree)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build_library()
    lib = ctypes.CDLL(_LIB_PATH)
    vp = ctypes.c_void_p
    lib.gg_erdos_renyi.restype = vp
    lib.gg_erdos_renyi.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64]
    lib.gg_chung_lu.restype = vp
    lib.gg_chung_lu.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
    lib.gg_barabasi_albert.restype = vp
    lib.gg_barabasi_albert.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64]
    lib.gg_sbm.restype = vp
    lib.gg_sbm.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64]
    lib.gg_n.restype = ctypes.c_int32
    lib.gg_n.argtypes = [vp]
    lib.gg_nnz.restype = ctypes.c_int64
    lib.gg_nnz.argtypes = [vp]
    lib.gg_copy.restype = None
    lib.gg_copy.argtypes = [vp, vp, vp]
    lib.gg_free.restype = None
    lib.gg_free.argtypes = [vp]
    lib.gg_fnv1a64.restype = ctypes.c_uint64
    lib.gg_fnv1a64.argtypes = [ctypes.c_int32, vp, vp]
    lib.gg_batch_params.restype = None
    lib.gg_batch_params.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_int32)]
    _lib = lib
    return lib


def _take(handle) -> Graph:
    lib = _load()
    if not handle:
        raise ValueError("generator rejected its parameters")
    n = lib.gg_n(handle)
    nnz = lib.gg_nnz(handle)
    rp = np.empty(n + 1, dtype=np.int64)
    col = np.empty(max(nnz, 1), dtype=np.int32)
    lib.gg_copy(handle, rp.ctypes.data, col.ctypes.data)
    lib.gg_free(handle)
    return Graph(n, rp, col[:nnz].copy())


# ---------------------------------------------------------------- random families

def erdos_renyi(n: int, m: int, seed: int) -> Graph:
    """G(n, m): m distinct uniform pairs (capped at n(n-1)/2)."""
    return _take(_load().gg_erdos_renyi(n, m, seed))


def chung_lu(n: int, m: int, gamma: float, wmax: float, seed: int) -> Tuple[Graph, float]:
    """Chung-Lu graph with weights w_i = wmax*((i+i0)/i0)^(-1/(gamma-1)).

    i0 is found by bisection so that the mean weight is 2m/n; endpoints are drawn
    proportionally to weight (alias method) and loops / repeats are rejected
    until exactly m edges exist.  Returns (graph, i0).
    """
    i0 = ctypes.c_double(0.0)
    g = _take(_load().gg_chung_lu(n, m, gamma, wmax, seed, ctypes.byref(i0)))
    return g, i0.value


def barabasi_albert(n: int, m0: int, seed: int) -> Graph:
    """Preferential attachment: a clique on m0+1 vertices, then each new vertex
    joins m0 distinct targets drawn in proportion to degree."""
    return _take(_load().gg_barabasi_albert(n, m0, seed))


def sbm(blocks: int, block_size: int, p_in: float, p_out: float, seed: int) -> Graph:
    """Planted-partition stochastic block model with equal blocks."""
    return _take(_load().gg_sbm(blocks, block_size, p_in, p_out, seed))


def fnv1a64(g: Graph) -> int:
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.int32)
    return int(_load().gg_fnv1a64(g.n, rp.ctypes.data, col.ctypes.data))


# ---------------------------------------------------------------- structured families

def from_edges(n: int, edges: Iterable[Tuple[int, int]]) -> Graph:
    """CSR from an undirected edge list (duplicates and loops removed)."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    if e.size:
        e = e[e[:, 0] != e[:, 1]]
        a = np.minimum(e[:, 0], e[:, 1])
        b = np.maximum(e[:, 0], e[:, 1])
        e = np.unique(np.stack([a, b], axis=1), axis=0)
    src = np.concatenate([e[:, 0], e[:, 1]]) if e.size else np.zeros(0, np.int64)
    dst = np.concatenate([e[:, 1], e[:, 0]]) if e.size else np.zeros(0, np.int64)
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, src + 1, 1)
    rp = np.cumsum(rp).astype(np.int64)
    return Graph(n, rp, dst.astype(np.int32))


def from_dense(adj: np.ndarray) -> Graph:
    a = np.asarray(adj, dtype=bool)
    iu = np.argwhere(np.triu(a, 1))
    return from_edges(a.shape[0], iu)


def hub_graph(roots: int, base: int, hub_degree: int, seed: int) -> Graph:
    """Sparse base with three high-degree hubs and a few low-rank roots.

    Vertices 0..roots-1 are the roots: each is adjacent to the three hubs only
    (degree 3, the lowest (degree, id) ranks).  Vertices roots..roots+base-1
    form a cycle plus a seeded perfect matching (degree 3 each, ranked above
    the roots).  The hubs are the last three vertices: hub 0 ~ hub 1 and
    hub 1 ~ hub 2 are edges, hub 0 and hub 2 are not; each hub is adjacent to
    `hub_degree` seeded base vertices, 10% of them shared with the next hub.
    A traversal made of a root and two (three) hubs has a list of about
    2 (3) x hub_degree entries above the root."""
    rng = np.random.default_rng(seed)
    n = roots + base + 3
    hubs = [roots + base, roots + base + 1, roots + base + 2]
    edges = []
    b = np.arange(roots, roots + base)
    edges += [(int(b[i]), int(b[(i + 1) % base])) for i in range(base)]
    perm = rng.permutation(b)
    edges += [(int(perm[2 * i]), int(perm[2 * i + 1])) for i in range(base // 2)]
    for r in range(roots):
        edges += [(r, h) for h in hubs]
    edges += [(hubs[0], hubs[1]), (hubs[1], hubs[2])]
    prev = None
    for h in hubs:
        own = rng.choice(b, hub_degree, replace=False)
        if prev is not None:
            own[: hub_degree // 10] = prev[: hub_degree // 10]
        own = np.unique(own)
        edges += [(int(x), h) for x in own]
        prev = rng.permutation(own)
    return from_edges(n, edges)


def complete(n: int) -> Graph:
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def complete_multipartite(parts: Sequence[int]) -> Graph:
    label = np.repeat(np.arange(len(parts)), parts)
    n = int(label.size)
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n) if label[i] != label[j]])


def complete_bipartite(a: int, b: int) -> Graph:
    return complete_multipartite([a, b])


def cocktail_party(r: int) -> Graph:
    """K_{2,2,...,2} with r parts."""
    return complete_multipartite([2] * r)


def path(n: int) -> Graph:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)])


def cycle(n: int) -> Graph:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)])


def star(leaves: int) -> Graph:
    """K_{1,leaves} with the centre at vertex 0."""
    return from_edges(leaves + 1, [(0, i) for i in range(1, leaves + 1)])


def hypercube(d: int) -> Graph:
    n = 1 << d
    return from_edges(n, [(v, v ^ (1 << b)) for v in range(n) for b in range(d) if v < v ^ (1 << b)])


def empty(n: int) -> Graph:
    return from_edges(n, [])


def relabel(g: Graph, perm: np.ndarray) -> Graph:
    """Apply the vertex map v -> perm[v]."""
    perm = np.asarray(perm, dtype=np.int64)
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    e = np.stack([perm[src], perm[g.col.astype(np.int64)]], axis=1)
    return from_edges(g.n, e[e[:, 0] < e[:, 1]])


def disjoint_union(graphs: Sequence[Graph]) -> Tuple[Graph, np.ndarray]:
    """Concatenate graphs; returns (union, vertex offsets of length len+1)."""
    offs = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        offs[i + 1] = offs[i] + g.n
    rp = [np.zeros(1, dtype=np.int64)]
    cols = []
    base = 0
    for i, g in enumerate(graphs):
        rp.append(g.row_ptr[1:] + base)
        cols.append(g.col.astype(np.int64) + offs[i])
        base += g.nnz
    col = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    return Graph(int(offs[-1]), np.concatenate(rp), col), offs


# ---------------------------------------------------------------- named workloads

def batch_params(i: int, nlo: int = 20, nhi: int = 2000, dlo: float = 4.0, dhi: float = 16.0,
                 mlo: int = 2, mhi: int = 6) -> Tuple[str, int, int]:
    """(kind, n, m-or-m0) of graph i in the uneven batch: even i -> G(n,m), odd -> BA."""
    n = ctypes.c_int32(0)
    m = ctypes.c_int64(0)
    m0 = ctypes.c_int32(0)
    _load().gg_batch_params(i, nlo, nhi, dlo, dhi, mlo, mhi, ctypes.byref(n), ctypes.byref(m), ctypes.byref(m0))
    if i % 2 == 0:
        return "er", n.value, m.value
    return "ba", n.value, m0.value


def batch_graph(i: int, **kw) -> Graph:
    kind, n, x = batch_params(i, **kw)
    if kind == "er":
        return erdos_renyi(n, x, seed=i)
    return barabasi_albert(n, x, seed=i)


def batch_graphs(count: int, **kw) -> List[Graph]:
    return [batch_graph(i, **kw) for i in range(count)]


WORKLOADS = {
    "er516": "G(n=516, m=1200) uniform pairs",
    "cl1m": "Chung-Lu n=1e6 m=2e7 gamma=2.1 wmax=1e4",
    "cl100k": "Chung-Lu n=1e5 m=1e6 gamma=2.3",
    "batch4096": "4096 graphs, n~U{20..2000}, even: G(n, n*d/2) d~U[4,16), odd: BA m0~U{2..6}",
    "sbm200x60": "SBM 200 blocks x 60, p_in=0.45, p_out=0.0005",
}


def workload_graph(name: str, seed: int = 0, **kw) -> Graph:
    if name == "er516":
        return erdos_renyi(516, 1200, seed)
    if name == "cl1m":
        return chung_lu(1_000_000, 20_000_000, 2.1, kw.get("wmax", 1.0e4), seed)[0]
    if name == "cl100k":
        return chung_lu(100_000, 1_000_000, 2.3, kw.get("wmax", 1414.0), seed)[0]
    if name == "sbm200x60":
        return sbm(200, 60, 0.45, 0.0005, seed)
    raise KeyError(name)


# ---------------------------------------------------------------- directed graphs

@dataclass
class Digraph:
    """Arcs as sorted out-lists: row_ptr[n+1] (int64), col[arcs] (int32)."""
    n: int
    row_ptr: np.ndarray
    col: np.ndarray

    @property
    def arcs(self) -> int:
        return int(self.row_ptr[-1])


def digraph_from_arcs(n: int, arcs: Iterable[Tuple[int, int]]) -> Digraph:
    a = np.asarray(list(arcs), dtype=np.int64).reshape(-1, 2)
    a = a[a[:, 0] != a[:, 1]]
    key = np.unique(a[:, 0] * max(n, 1) + a[:, 1]) if a.size else np.zeros(0, np.int64)
    src = key // max(n, 1)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=rp[1:])
    return Digraph(n, rp, (key % max(n, 1)).astype(np.int32))


def orient(g: Graph, seed: int, both: float = 0.2) -> Digraph:
    """Each edge {u, v} of g becomes an arc u->v or v->u (fair coin), or both
    arcs with probability `both` (seeded)."""
    rng = np.random.default_rng(seed)
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    dst = g.col.astype(np.int64)
    keep = src < dst
    u, v = src[keep], dst[keep]
    r = rng.random(u.size)
    fwd = (r < both) | (r >= both + (1.0 - both) / 2)
    bwd = r < both + (1.0 - both) / 2
    arcs = np.concatenate([np.stack([u[fwd], v[fwd]], 1), np.stack([v[bwd], u[bwd]], 1)])
    return digraph_from_arcs(g.n, arcs)


def random_digraph(n: int, m: int, seed: int, both: float = 0.2) -> Digraph:
    """An orientation of the Erdos-Renyi G(n, m) graph."""
    return orient(erdos_renyi(n, m, seed), seed + 1, both)


def symmetric(g: Graph) -> Digraph:
    """Every edge as two opposite arcs."""
    return Digraph(g.n, g.row_ptr.copy(), g.col.copy())


def transitive_tournament(n: int) -> Digraph:
    return digraph_from_arcs(n, [(a, b) for a in range(n) for b in range(a + 1, n)])


def directed_cycle(n: int) -> Digraph:
    return digraph_from_arcs(n, [(a, (a + 1) % n) for a in range(n)])


def reverse(d: Digraph) -> Digraph:
    src = np.repeat(np.arange(d.n, dtype=np.int64), np.diff(d.row_ptr))
    return digraph_from_arcs(d.n, np.stack([d.col.astype(np.int64), src], 1))
