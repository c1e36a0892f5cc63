"""CPU oracle — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and the
oracle never imports the product: the two share no code.  What each function
computes, and which passage of DuMato (Ferraz et al., arXiv 2212.04551) it
follows, is stated in ``oracle.c`` and in the docstrings below.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (in-tree)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    L = ctypes.CDLL(_LIB)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    L.or_canon.restype = u32
    L.or_canon.argtypes = [ctypes.c_int, u32]
    L.or_num_classes.restype = ctypes.c_int
    L.or_num_classes.argtypes = [ctypes.c_int]
    L.or_class_canon.restype = ctypes.c_int
    L.or_class_canon.argtypes = [ctypes.c_int, vp, ctypes.c_int]
    L.or_num_connected_labelled.restype = i64
    L.or_num_connected_labelled.argtypes = [ctypes.c_int]
    L.or_class_of_code.restype = ctypes.c_int
    L.or_class_of_code.argtypes = [ctypes.c_int, u32]
    L.or_class_of_codes.restype = None
    L.or_class_of_codes.argtypes = [ctypes.c_int, vp, i64, vp]
    L.or_canon_methods_agree.restype = ctypes.c_int
    L.or_canon_methods_agree.argtypes = [ctypes.c_int]
    L.or_clique_brute.restype = ctypes.c_int
    L.or_clique_brute.argtypes = [i32, vp, vp, ctypes.c_int, vp, vp]
    L.or_motif_brute.restype = ctypes.c_int
    L.or_motif_brute.argtypes = [i32, vp, vp, ctypes.c_int, vp, vp]
    L.or_clique_roots.restype = ctypes.c_int
    L.or_clique_roots.argtypes = [i32, vp, vp, ctypes.c_int, vp, i64, ctypes.c_int, vp, vp, vp, vp,
                                  ctypes.c_double, vp]
    L.or_motif_roots.restype = ctypes.c_int
    L.or_motif_roots.argtypes = [i32, vp, vp, ctypes.c_int, vp, i64, ctypes.c_int, vp, vp, vp, vp,
                                 ctypes.c_double, vp, vp]
    for f in (L.or_clique_timed, L.or_motif_timed):
        f.restype = ctypes.c_uint64
        f.argtypes = [i32, vp, vp, ctypes.c_int, vp, i64, ctypes.c_int, ctypes.c_double,
                      ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]
    L.or_twohop.restype = None
    L.or_twohop.argtypes = [i32, vp, vp, vp]
    L.or_triangles.restype = None
    L.or_triangles.argtypes = [i32, vp, vp, vp]
    L.or_core.restype = None
    L.or_core.argtypes = [i32, vp, vp, vp]
    L.or_dcanon.restype = u32
    L.or_dcanon.argtypes = [ctypes.c_int, u32]
    L.or_dnum_classes.restype = ctypes.c_int
    L.or_dnum_classes.argtypes = [ctypes.c_int]
    L.or_dclass_canon.restype = ctypes.c_int
    L.or_dclass_canon.argtypes = [ctypes.c_int, vp, ctypes.c_int]
    L.or_dclass_of_code.restype = ctypes.c_int
    L.or_dclass_of_code.argtypes = [ctypes.c_int, u32]
    L.or_dnum_connected_labelled.restype = i64
    L.or_dnum_connected_labelled.argtypes = [ctypes.c_int]
    L.or_dclass_table.restype = ctypes.c_int
    L.or_dclass_table.argtypes = [ctypes.c_int, vp, i64]
    L.or_dmotif_brute.restype = ctypes.c_int
    L.or_dmotif_brute.argtypes = [i32, vp, vp, ctypes.c_int, vp]
    L.or_dmotif_esu.restype = ctypes.c_int
    L.or_dmotif_esu.argtypes = [i32, vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, vp]
    _lib = L
    return L


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.int32)
    return rp, col


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


# ------------------------------------------------------------------ classes

def canon(k: int, code: int) -> int:
    """Minimum edge bitmap over all k! relabellings (bit i(i-1)/2+t = edge t<i)."""
    return int(_load().or_canon(k, code))


def num_classes(k: int) -> int:
    return int(_load().or_num_classes(k))


def class_canon(k: int) -> np.ndarray:
    """Canonical codes of the connected classes, in class-id order."""
    L = _load()
    ncls = L.or_num_classes(k)
    out = np.zeros(max(ncls, 1), dtype=np.uint32)
    L.or_class_canon(k, out.ctypes.data, ncls)
    return out[:ncls]


def num_connected_labelled(k: int) -> int:
    return int(_load().or_num_connected_labelled(k))


def canon_methods_agree(k: int) -> bool:
    """The orbit-labelling method (used for k = 7) reproduces the per-code
    minimum over all k! relabellings on every code on k <= 6 vertices."""
    return _load().or_canon_methods_agree(k) == 1


def class_of_code(k: int, code: int) -> int:
    """Class id of a full edge bitmap on k vertices, or -1 if disconnected."""
    return int(_load().or_class_of_code(k, code))


def class_of_codes(k: int, codes) -> np.ndarray:
    """class_of_code over an array of full edge bitmaps."""
    c = np.ascontiguousarray(codes, dtype=np.int64)
    out = np.empty(c.size, dtype=np.int64)
    _load().or_class_of_codes(k, c.ctypes.data, c.size, out.ctypes.data)
    return out


def code_of(adj: np.ndarray) -> int:
    """Full edge bitmap of a k x k adjacency matrix (column order)."""
    k = adj.shape[0]
    c = 0
    for i in range(1, k):
        for t in range(i):
            if adj[t, i]:
                c |= 1 << (i * (i - 1) // 2 + t)
    return c


# ------------------------------------------------------------------ L1

def clique_brute(g, k: int, per_root: bool = False):
    """Number of k-subsets that are cliques (definition, every subset)."""
    rp, col = _csr(g)
    tot = np.zeros(1, dtype=np.uint64)
    pr = np.zeros(max(g.n, 1), dtype=np.uint64) if per_root else None
    rc = _load().or_clique_brute(g.n, rp.ctypes.data, col.ctypes.data, k, tot.ctypes.data, _ptr(pr))
    if rc != 0:
        raise ValueError("bad arguments")
    return (int(tot[0]), pr[:g.n]) if per_root else int(tot[0])


def motif_brute(g, k: int, per_root: bool = False):
    """Per-class counts of connected induced k-subsets (definition, every subset)."""
    rp, col = _csr(g)
    ncls = num_classes(k)
    out = np.zeros(ncls, dtype=np.uint64)
    pr = np.zeros(max(g.n, 1), dtype=np.uint64) if per_root else None
    rc = _load().or_motif_brute(g.n, rp.ctypes.data, col.ctypes.data, k, out.ctypes.data, _ptr(pr))
    if rc != 0:
        raise ValueError("bad arguments")
    return (out, pr[:g.n]) if per_root else out


# ------------------------------------------------------------------ listings

def _adjsets(g):
    return [set(int(x) for x in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]) for v in range(g.n)]


def clique_list(g, k: int) -> np.ndarray:
    """Every k-clique (Section IV-C aggregate_store: the subgraphs themselves
    rather than their number) as a row of its k vertex ids in ascending order,
    rows sorted.  Backtracking over increasing ids: a set grows only by a
    larger vertex adjacent to all its members, so each clique appears once.
    Pure Python: small graphs only."""
    adj = _adjsets(g)
    rows = []

    def grow(sub, cand):
        if len(sub) == k:
            rows.append(tuple(sub))
            return
        for u in sorted(cand):
            grow(sub + [u], {w for w in cand if w > u and w in adj[u]})

    if k >= 1:
        for v in range(g.n):
            grow([v], {w for w in adj[v] if w > v})
    out = np.array(sorted(rows), dtype=np.int64).reshape(-1, k)
    return out


def motif_list(g, k: int) -> np.ndarray:
    """Every connected induced k-subset (Section IV-E, motif counting; listed
    as aggregate_store would) as a row of its k vertex ids in ascending order
    followed by its class id (class_of_code of its adjacency in that order),
    rows sorted.  Connected sets are grown from their smallest vertex by
    adding any larger neighbour of the set, duplicates removed by set
    membership.  Pure Python: small graphs only."""
    adj = _adjsets(g)
    found = set()
    for r in range(g.n):
        frontier = {frozenset([r])}
        for _ in range(k - 1):
            nxt = set()
            for S in frontier:
                nb = set()
                for v in S:
                    nb |= adj[v]
                for w in nb:
                    if w > r and w not in S:
                        nxt.add(S | {w})
            frontier = nxt
        found |= frontier
    rows = []
    for S in found:
        vs = sorted(S)
        a = np.zeros((k, k), dtype=np.uint8)
        for i in range(k):
            for j in range(i + 1, k):
                if vs[j] in adj[vs[i]]:
                    a[i, j] = a[j, i] = 1
        rows.append(tuple(vs) + (class_of_code(k, code_of(a)),))
    return np.array(sorted(rows), dtype=np.int64).reshape(-1, k + 1)


# ------------------------------------------------------------------ property filters

def quasi_clique_brute(g, k: int, min_edges: int) -> int:
    """Connected k-subsets whose induced subgraph has at least min_edges
    edges (Section II's property P as a density threshold), by the definition:
    every k-subset is checked.  Pure Python: tiny graphs only."""
    import itertools
    adj = _adjsets(g)
    cnt = 0
    for S in itertools.combinations(range(g.n), k):
        e = sum(1 for i in range(k) for j in range(i + 1, k) if S[j] in adj[S[i]])
        if e < min_edges:
            continue
        seen, stack = {S[0]}, [S[0]]
        while stack:
            x = stack.pop()
            for y in S:
                if y not in seen and y in adj[x]:
                    seen.add(y)
                    stack.append(y)
        cnt += len(seen) == k
    return cnt


def quasi_clique_count(g, k: int, min_edges: int, threads: int = 1, class_counts=None) -> int:
    """The same from the ESU class counts: the classes whose canonical
    pattern has at least min_edges edges.  class_counts: motif_count(g, k)
    when the caller already has it (several thresholds on one graph)."""
    c = motif_count(g, k, threads=threads) if class_counts is None else np.asarray(class_counts)
    edges = np.array([bin(int(x)).count("1") for x in class_canon(k)])
    return int(c[edges >= min_edges].sum())


def induced(g, keep) -> "object":
    """The subgraph induced by the vertices with keep[v], renumbered in id
    order (a Graph-like object with n, row_ptr, col)."""
    keep = np.asarray(keep, dtype=bool)
    newid = np.cumsum(keep) - keep
    rows, cols = [], []
    rp = [0]
    for v in range(g.n):
        if not keep[v]:
            continue
        nb = g.col[g.row_ptr[v]:g.row_ptr[v + 1]]
        nb = nb[keep[nb]]
        cols.append(newid[nb])
        rp.append(rp[-1] + len(nb))
    col = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)

    class _G:
        pass

    h = _G()
    h.n = int(keep.sum())
    h.row_ptr = np.array(rp, dtype=np.int64)
    h.col = col
    h.nnz = int(len(col))
    return h


# ------------------------------------------------------------------ L2

def _roots(roots):
    if roots is None:
        return None, 0
    r = np.ascontiguousarray(roots, dtype=np.int32)
    return r, r.size


def clique_count(g, k: int, roots=None, threads: int = 1, per_root: bool = False):
    """k-cliques by rank-ordered backtracking.

    With ``roots`` only cliques credited to those roots (lowest (degree, id) rank)
    are counted.  With ``per_root`` returns (total, leaves, nodes, reads) arrays
    aligned with the root list.  Raises OverflowError on a uint64 wrap.
    """
    rp, col = _csr(g)
    r, nr = _roots(roots)
    cnt = nr if r is not None else g.n
    tot = np.zeros(1, dtype=np.uint64)
    arrs = [np.zeros(max(cnt, 1), dtype=np.uint64) for _ in range(3)] if per_root else [None] * 3
    rc = _load().or_clique_roots(g.n, rp.ctypes.data, col.ctypes.data, k, _ptr(r), nr, threads,
                                 tot.ctypes.data, *[_ptr(a) for a in arrs], 0.0, None)
    if rc < 0:
        raise ValueError("bad arguments")
    if rc == 1:
        raise OverflowError("uint64 overflow")
    if per_root:
        return (int(tot[0]),) + tuple(a[:cnt] for a in arrs)
    return int(tot[0])


def clique_budgeted(g, k: int, roots, threads: int, root_budget: float):
    """Per-root clique records with a time budget per root.

    Returns (done, leaves, nodes, reads) aligned with ``roots``: done[i] is
    True when root i finished within ``root_budget`` seconds; the records of
    the other roots are partial and must not be used."""
    rp, col = _csr(g)
    r, nr = _roots(roots)
    tot = np.zeros(1, dtype=np.uint64)
    arrs = [np.zeros(max(nr, 1), dtype=np.uint64) for _ in range(3)]
    done = np.zeros(max(nr, 1), dtype=np.uint8)
    rc = _load().or_clique_roots(g.n, rp.ctypes.data, col.ctypes.data, k, _ptr(r), nr, threads,
                                 tot.ctypes.data, *[_ptr(a) for a in arrs], float(root_budget), done.ctypes.data)
    if rc != 0:
        raise ValueError("bad arguments or overflow")
    return (done[:nr].astype(bool),) + tuple(a[:nr] for a in arrs)


def motif_count(g, k: int, roots=None, threads: int = 1, per_root: bool = False):
    """Per-class connected induced k-set counts by ESU (Wernicke 2006).

    With ``roots`` only sets whose lowest (degree, id) vertex is listed are
    counted.  With ``per_root`` returns (counts, leaves, nodes, reads).
    """
    rp, col = _csr(g)
    r, nr = _roots(roots)
    cnt = nr if r is not None else g.n
    out = np.zeros(num_classes(k), dtype=np.uint64)
    arrs = [np.zeros(max(cnt, 1), dtype=np.uint64) for _ in range(3)] if per_root else [None] * 3
    rc = _load().or_motif_roots(g.n, rp.ctypes.data, col.ctypes.data, k, _ptr(r), nr, threads,
                                out.ctypes.data, *[_ptr(a) for a in arrs], 0.0, None, None)
    if rc < 0:
        raise ValueError("bad arguments")
    if rc == 1:
        raise OverflowError("uint64 overflow")
    if per_root:
        return (out,) + tuple(a[:cnt] for a in arrs)
    return out


def motif_budgeted(g, k: int, roots, threads: int, root_budget: float):
    """Per-root motif records with a time budget per root.

    Returns (done, counts, leaves, nodes, reads): done as in clique_budgeted,
    counts[i] the class counts of root i (nroots x ncls)."""
    rp, col = _csr(g)
    r, nr = _roots(roots)
    ncls = num_classes(k)
    out = np.zeros(ncls, dtype=np.uint64)
    arrs = [np.zeros(max(nr, 1), dtype=np.uint64) for _ in range(3)]
    done = np.zeros(max(nr, 1), dtype=np.uint8)
    per = np.zeros((max(nr, 1), ncls), dtype=np.uint64)
    rc = _load().or_motif_roots(g.n, rp.ctypes.data, col.ctypes.data, k, _ptr(r), nr, threads,
                                out.ctypes.data, *[_ptr(a) for a in arrs], float(root_budget), done.ctypes.data,
                                per.ctypes.data)
    if rc != 0:
        raise ValueError("bad arguments or overflow")
    return (done[:nr].astype(bool), per[:nr]) + tuple(a[:nr] for a in arrs)


# ------------------------------------------------------------------ time-bounded runs

def _timed(fn, g, k, roots, threads, seconds):
    rp, col = _csr(g)
    r = np.ascontiguousarray(roots, dtype=np.int32)
    started = ctypes.c_int64(0)
    elapsed = ctypes.c_double(0.0)
    found = fn(g.n, rp.ctypes.data, col.ctypes.data, k, r.ctypes.data, r.size, threads, seconds,
               ctypes.byref(started), ctypes.byref(elapsed))
    return int(found), int(started.value), float(elapsed.value)


def clique_timed(g, k: int, roots, threads: int, seconds: float):
    """k-cliques found from `roots` (in order) within `seconds` of wall-clock time.

    Returns (subgraphs found, roots begun, seconds used); roots still running at
    the deadline are abandoned after counting what they had found."""
    return _timed(_load().or_clique_timed, g, k, roots, threads, seconds)


def motif_timed(g, k: int, roots, threads: int, seconds: float):
    """Connected induced k-sets found from `roots` within `seconds` (see clique_timed)."""
    return _timed(_load().or_motif_timed, g, k, roots, threads, seconds)


# ------------------------------------------------------------------ features

def features(g) -> np.ndarray:
    """[n, 4] float64: degree, 2-hop degree sum, core number, triangle count."""
    rp, col = _csr(g)
    L = _load()
    two = np.zeros(max(g.n, 1), dtype=np.int64)
    tri = np.zeros(max(g.n, 1), dtype=np.int64)
    core = np.zeros(max(g.n, 1), dtype=np.int32)
    L.or_twohop(g.n, rp.ctypes.data, col.ctypes.data, two.ctypes.data)
    L.or_triangles(g.n, rp.ctypes.data, col.ctypes.data, tri.ctypes.data)
    L.or_core(g.n, rp.ctypes.data, col.ctypes.data, core.ctypes.data)
    deg = np.diff(rp)
    return np.stack([deg, two[:g.n], core[:g.n], tri[:g.n]], axis=1).astype(np.float64)


# ------------------------------------------------------------------ directed graphs

def dcanon(k: int, code: int) -> int:
    """Minimum directed code over all k! vertex orders (two bits per pair
    t < i: bit 2p = arc t->i, bit 2p+1 = arc i->t, p = i(i-1)/2 + t)."""
    return int(_load().or_dcanon(k, code))


def dnum_classes(k: int) -> int:
    """Weakly connected digraphs on k vertices up to isomorphism."""
    return int(_load().or_dnum_classes(k))


def dclass_canon(k: int) -> np.ndarray:
    """Minimum codes of the weakly connected classes, in class-id order."""
    L = _load()
    ncls = L.or_dnum_classes(k)
    out = np.zeros(max(ncls, 1), dtype=np.uint32)
    L.or_dclass_canon(k, out.ctypes.data, ncls)
    return out[:ncls]


def dclass_of_code(k: int, code: int) -> int:
    """Class id of a directed code, or -1 if the digraph is not weakly connected."""
    return int(_load().or_dclass_of_code(k, code))


def dclass_table(k: int) -> np.ndarray:
    """dclass_of_code for every code on k vertices (int32, -1 if not weakly connected)."""
    out = np.zeros(1 << (k * (k - 1)), dtype=np.int32)
    if _load().or_dclass_table(k, out.ctypes.data, out.size) != 0:
        raise ValueError("k out of range")
    return out


def dnum_connected_labelled(k: int) -> int:
    return int(_load().or_dnum_connected_labelled(k))


def undirected_of(dg):
    """The underlying undirected graph of a digraph (arcs in sorted out-lists
    row_ptr / col): every arc u->w gives the edge {u, w}; sorted, no repeats."""
    n = int(dg.n)
    rp = np.asarray(dg.row_ptr, dtype=np.int64)
    dst = np.asarray(dg.col, dtype=np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    key = np.unique(np.concatenate([src * n + dst, dst * n + src])) if dst.size else np.zeros(0, np.int64)
    a = key // max(n, 1)
    b = (key % max(n, 1)).astype(np.int32)
    urp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(a, minlength=n), out=urp[1:])
    return urp, b


def dmotif_brute(dg, k: int) -> np.ndarray:
    """Per-class counts of the weakly connected induced k-vertex subdigraphs,
    by the definition: every k-subset of the vertices."""
    rp, col = _csr(dg)
    out = np.zeros(max(dnum_classes(k), 1), dtype=np.uint64)
    if _load().or_dmotif_brute(dg.n, rp.ctypes.data, col.ctypes.data, k, out.ctypes.data) != 0:
        raise ValueError("bad arguments")
    return out[:dnum_classes(k)]


def dmotif_count(dg, k: int, threads: int = 1) -> np.ndarray:
    """The same by ESU enumeration of connected k-subsets of the underlying
    undirected graph, each classified by its arcs."""
    rp, col = _csr(dg)
    urp, ucol = undirected_of(dg)
    ucol = np.ascontiguousarray(ucol if ucol.size else np.zeros(1, np.int32))
    out = np.zeros(max(dnum_classes(k), 1), dtype=np.uint64)
    rc = _load().or_dmotif_esu(dg.n, rp.ctypes.data, col.ctypes.data, urp.ctypes.data, ucol.ctypes.data, k,
                               threads, out.ctypes.data)
    if rc != 0:
        raise ValueError("bad arguments")
    return out[:dnum_classes(k)]


# ------------------------------------------------------------------ subgraph matching

def _pattern_arcs(k: int, code: int, directed: bool):
    """Adjacency (k x k booleans) of a pattern code: undirected, bit
    i(i-1)/2 + t = edge t-i; directed, bit 2p = arc t->i and bit 2p+1 =
    arc i->t (p = i(i-1)/2 + t)."""
    A = np.zeros((k, k), dtype=bool)
    for i in range(1, k):
        for t in range(i):
            p = i * (i - 1) // 2 + t
            if directed:
                A[t, i] = bool(code >> (2 * p) & 1)
                A[i, t] = bool(code >> (2 * p + 1) & 1)
            else:
                A[t, i] = A[i, t] = bool(code >> p & 1)
    return A


def _embeddings(A, n, has, induced):
    """Injective maps phi of the pattern's vertices into 0..n-1 with
    has(phi(a), phi(b)) whenever A[a, b] (and only then, if induced)."""
    k = A.shape[0]
    und = A | A.T
    order = [0]  # a connected order: each next vertex adjacent to an earlier one
    while len(order) < k:
        order.append(next(v for v in range(k) if v not in order and any(und[v, u] for u in order)))
    phi = [-1] * k
    used = set()
    count = 0

    def ok(a, x):
        for b in range(k):
            if phi[b] < 0:
                continue
            y = phi[b]
            if A[a, b] and not has(x, y):
                return False
            if A[b, a] and not has(y, x):
                return False
            if induced and (not A[a, b] and has(x, y) or not A[b, a] and has(y, x)):
                return False
        return True

    def rec(j):
        nonlocal count
        if j == k:
            count += 1
            return
        a = order[j]
        for x in range(n):
            if x not in used and ok(a, x):
                phi[a] = x
                used.add(x)
                rec(j + 1)
                used.discard(x)
                phi[a] = -1

    rec(0)
    return count


def pattern_count_brute(g, k: int, code: int, induced: bool = False, directed: bool = False) -> int:
    """Copies of the connected pattern P (a code on k vertices) in g, by the
    definition: edge-preserving injective maps of P into g (also non-edge
    preserving when induced), divided by the maps of P onto itself.  g: an
    undirected Graph, or a Digraph with directed=True.  Pure Python: small
    graphs only."""
    A = _pattern_arcs(k, code, directed)
    adj = [set(int(x) for x in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]) for v in range(g.n)]
    emb = _embeddings(A, g.n, lambda x, y: y in adj[x], induced)
    aut = _embeddings(A, k, lambda x, y: bool(A[x, y]), True)
    assert emb % aut == 0
    return emb // aut
