"""GPU parity on the benchmark's own graphs, at full scale.

The full clique counts of the 10^6-vertex Chung-Lu graph for k >= 6 and the
full motif counts of the 10^5-vertex Chung-Lu graphs are beyond the oracle,
so they are pinned three ways:
  - per-root records {leaves, tree nodes, adjacency entries read} of seeded
    root samples equal the oracle's exactly (every count is a sum over roots:
    each subgraph belongs to its lowest (degree, id) vertex, Section IV-E's
    canonical traversals rooted at their smallest vertex);
  - the heaviest roots the oracle can finish (records written offline by
    tests/golden/make_sampled_roots.py, which calls only the oracle);
  - identities that hold for the full counts: the star identity
    sum_v C(d_v, k-1) = sum_H c_H sigma_H (sigma_H = vertices of H adjacent to
    all others) and the clique class of the motif counts = the k-clique count.
All GPU calls go through the C ABI.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2212_04551_amd import dm
from paper_2212_04551_amd import graphgen as gg

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
THREADS = min(16, os.cpu_count() or 1)


def read_golden(name):
    """(graphs {name: (n, nnz, fnv)}, roots {k: [(v, leaves, nodes, reads)]}, classes {k: array})"""
    graphs, roots, classes = {}, {}, {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            if p[0] == "graph":
                graphs[p[1]] = tuple(int(x) for x in p[2:5])
            elif p[0] == "root":
                roots.setdefault(int(p[1]), []).append(tuple(int(x) for x in p[2:6]))
            elif p[0] == "classes":
                classes[int(p[1])] = np.array([int(x) for x in p[2:]], dtype=np.uint64)
    return graphs, roots, classes


def check_graph(g, graphs, name):
    n, nnz, fnv = graphs[name]
    assert (g.n, g.nnz, gg.fnv1a64(g)) == (n, nnz, fnv), f"{name}: generator output changed"


def gpu_records(h, op, k, roots):
    import torch
    stats = torch.zeros((len(roots), 3), dtype=torch.int64, device="cuda")
    if op == "clique":
        tot = dm.count_cliques(h, k, roots=roots, root_stats=stats)
    else:
        tot = dm.count_motifs(h, k, roots=roots, root_stats=stats)
    return tot, stats.cpu().numpy().astype(np.uint64)


def sigma(k):
    """Vertices adjacent to every other vertex, per class (oracle's class order)."""
    out = []
    for code in O.class_canon(k):
        deg = [0] * k
        for i in range(1, k):
            for t in range(i):
                if int(code) >> (i * (i - 1) // 2 + t) & 1:
                    deg[i] += 1
                    deg[t] += 1
        out.append(sum(1 for d in deg if d == k - 1))
    return out


# ------------------------------------------------------------------ cl1m cliques

@pytest.fixture(scope="module")
def cl1m():
    g = gg.chung_lu(1_000_000, 20_000_000, 2.1, 1.0e4, 0)[0]
    h = dm.load_graph(g)
    return g, h


def test_cl1m_uniform_root_sample(cl1m):
    """1000 seeded uniform roots of the benchmark graph, k = 3..8: per-root
    records equal the oracle's (recording launch), and the counting launch
    (pruning, dense solver, row cache) over the same roots gives their sum."""
    g, h = cl1m
    roots = np.sort(np.random.default_rng(0).choice(g.n, 1000, replace=False)).astype(np.int32)
    for k in range(3, 9):
        tot, leaves, nodes, reads = O.clique_count(g, k, roots=roots, per_root=True, threads=THREADS)
        got, st = gpu_records(h, "clique", k, roots)
        assert got == tot, k
        assert np.array_equal(st[:, 1], leaves), k
        assert np.array_equal(st[:, 0], nodes), k
        assert np.array_equal(st[:, 2], reads), k
        assert dm.count_cliques(h, k, roots=roots) == tot, k


def test_cl1m_heaviest_finishable_roots(cl1m):
    """Per k = 3..8, the roots of most tree nodes among wide-root candidates
    that the oracle finishes within its per-root budget (records written by
    tests/golden/make_sampled_roots.py): records and counting-launch sums."""
    g, h = cl1m
    graphs, per_k, _ = read_golden("cl1m_heavy_roots.txt")
    check_graph(g, graphs, "cl1m")
    assert sorted(per_k) == [3, 4, 5, 6, 7, 8]
    for k, rows in sorted(per_k.items()):
        roots = np.array([r[0] for r in rows], dtype=np.int32)
        exp = np.array([r[1:] for r in rows], dtype=np.uint64)
        got, st = gpu_records(h, "clique", k, roots)
        assert np.array_equal(st[:, 1], exp[:, 0]), k
        assert np.array_equal(st[:, 0], exp[:, 1]), k
        assert np.array_equal(st[:, 2], exp[:, 2]), k
        assert got == int(exp[:, 0].sum()) == dm.count_cliques(h, k, roots=roots), k


# ------------------------------------------------------------------ cl100k motifs

@pytest.fixture(scope="module")
def cl100k():
    out = {}
    for k, cap in ((5, 1414.0), (6, 120.0)):
        g = gg.chung_lu(100_000, 1_000_000, 2.3, cap, 0)[0]
        out[k] = (g, dm.load_graph(g), cap)
    return out


@pytest.mark.parametrize("k", [5, 6])
def test_cl100k_full_counts_identities(cl100k, k):
    """Full motif counts of the benchmark graph (k=5 at weight cap 1414, k=6 at
    cap 120): the star identity and the clique class = the k-clique count."""
    g, h, _ = cl100k[k]
    c = dm.count_motifs(h, k)
    deg = g.degrees()
    lhs = sum(math.comb(int(d), k - 1) for d in deg)
    rhs = sum(int(x) * s for x, s in zip(c, sigma(k)))
    assert lhs == rhs, (k, lhs, rhs)
    kcls = int(np.nonzero(O.motif_brute(gg.complete(k), k))[0][0])
    assert int(c[kcls]) == dm.count_cliques(h, k)


@pytest.mark.parametrize("k", [5, 6])
def test_cl100k_sampled_roots(cl100k, k):
    """Seeded uniform root sample (the roots the oracle finishes within its
    per-root budget, written by tests/golden/make_sampled_roots.py): per-root
    records and the per-class counts over the finished roots."""
    g, h, cap = cl100k[k]
    graphs, per_k, classes = read_golden("cl100k_roots.txt")
    check_graph(g, graphs, f"cl100k_cap{int(cap)}")
    rows = per_k[k]
    assert len(rows) >= 64, "too few finished roots in the fixture"
    roots = np.array([r[0] for r in rows], dtype=np.int32)
    exp = np.array([r[1:] for r in rows], dtype=np.uint64)
    got, st = gpu_records(h, "motif", k, roots)
    assert np.array_equal(got, classes[k])
    assert np.array_equal(st[:, 1], exp[:, 0])
    assert np.array_equal(st[:, 0], exp[:, 1])
    assert np.array_equal(st[:, 2], exp[:, 2])
    assert np.array_equal(dm.count_motifs(h, k, roots=roots), classes[k])


# ------------------------------------------------------------------ motif lists kept in global memory

def test_hub_graph_long_leaf_lists_k5():
    """Three hubs of degree about 480 and 8 degree-3 roots adjacent to all of
    them: at k=5 every traversal of a root and two hubs has a leaf-level list
    of 844-877 entries, above the 800 that fit the LDS copy, so the lookups go
    through the global list's filters, fences and windows.  Oracle live."""
    g = gg.hub_graph(8, 3000, 480, 1)
    h = dm.load_graph(g)
    roots = np.arange(8, dtype=np.int32)
    c, leaves, nodes, reads = O.motif_count(g, 5, roots=roots, per_root=True, threads=THREADS)
    got, st = gpu_records(h, "motif", 5, roots)
    assert np.array_equal(got, c)
    assert np.array_equal(st[:, 1], leaves) and np.array_equal(st[:, 0], nodes) and np.array_equal(st[:, 2], reads)
    assert np.array_equal(dm.count_motifs(h, 5, roots=roots), c)
    assert np.array_equal(dm.count_motifs(h, 5, roots=roots, chunk=1, rebalance=0.01), c)


def test_hub_graph_long_leaf_lists_k6():
    """k=6: a root and three hubs of degree about 340 leave a leaf-level list
    of about 860 entries (records written by make_sampled_roots.py)."""
    g = gg.hub_graph(4, 3000, 340, 2)
    graphs, per_k, classes = read_golden("hub_roots_k6.txt")
    check_graph(g, graphs, "hub4_3000_340_s2")
    h = dm.load_graph(g)
    rows = per_k[6]
    roots = np.array([r[0] for r in rows], dtype=np.int32)
    exp = np.array([r[1:] for r in rows], dtype=np.uint64)
    got, st = gpu_records(h, "motif", 6, roots)
    assert np.array_equal(got, classes[6])
    assert np.array_equal(st[:, 1], exp[:, 0]) and np.array_equal(st[:, 0], exp[:, 1])
    assert np.array_equal(st[:, 2], exp[:, 2])
    assert np.array_equal(dm.count_motifs(h, 6, roots=roots), classes[6])
