"""Pins of the oracle's directed-motif functions (CPU only).  Directed codes:
two bits per vertex pair t < i (bit 2p = arc t->i, bit 2p+1 = arc i->t,
p = i(i-1)/2 + t); a class is the minimum code over all vertex orders; the
classes are the weakly connected digraphs.  Pinned by the published numbers
of classes and of labelled weakly connected digraphs (OEIS A003085, A003027),
by networkx's digraph isomorphism, by brute force over every k-subset, and by
closed forms (tournaments, cycles, symmetric digraphs = undirected counts)."""
import itertools
import math
import os

import networkx as nx
import numpy as np
import pytest

import oracle as O
from paper_2212_04551_amd import graphgen as gg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _published():
    rows = {}
    with open(os.path.join(GOLDEN, "digraph_counts.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, c, l = map(int, line.split())
            rows[k] = (c, l)
    return rows


def pbit(t, i):
    return i * (i - 1) // 2 + t


def digraph_of_code(k, code):
    D = nx.DiGraph()
    D.add_nodes_from(range(k))
    for i in range(1, k):
        for t in range(i):
            if code >> (2 * pbit(t, i)) & 1:
                D.add_edge(t, i)
            if code >> (2 * pbit(t, i) + 1) & 1:
                D.add_edge(i, t)
    return D


def code_of_digraph(k, D, order):
    pos = {v: j for j, v in enumerate(order)}
    c = 0
    for a, b in D.edges():
        x, y = pos[a], pos[b]
        c |= 1 << (2 * pbit(x, y)) if x < y else 1 << (2 * pbit(y, x) + 1)
    return c


def reverse_code(k, code):
    r = 0
    for i in range(1, k):
        for t in range(i):
            p = pbit(t, i)
            if code >> (2 * p) & 1:
                r |= 1 << (2 * p + 1)
            if code >> (2 * p + 1) & 1:
                r |= 1 << (2 * p)
    return r


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_class_counts_match_published(k):
    ncls, labelled = _published()[k]
    assert O.dnum_classes(k) == ncls
    assert O.dnum_connected_labelled(k) == labelled


@pytest.mark.parametrize("k", [3, 4, 5])
def test_class_representatives_pairwise_nonisomorphic(k):
    canon = O.dclass_canon(k)
    assert np.all(np.diff(canon.astype(np.int64)) > 0)
    rng = np.random.default_rng(k)
    idx = np.arange(len(canon)) if len(canon) <= 300 else rng.choice(len(canon), 600, replace=False)
    graphs = [digraph_of_code(k, int(canon[i])) for i in idx]
    assert all(nx.is_weakly_connected(D) for D in graphs)
    buckets = {}
    for D in graphs:
        buckets.setdefault(nx.weisfeiler_lehman_graph_hash(D, iterations=3), []).append(D)
    for group in buckets.values():
        for a, b in itertools.combinations(group, 2):
            assert not nx.is_isomorphic(a, b)
    # every representative is its own minimum
    for i in idx[:200]:
        assert O.dcanon(k, int(canon[i])) == int(canon[i])
        assert O.dclass_of_code(k, int(canon[i])) == int(i)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_random_codes_classified_like_networkx(k):
    rng = np.random.default_rng(100 + k)
    bits = k * (k - 1)
    codes = [int(x) for x in rng.integers(0, 1 << bits, 400)]
    cls = [O.dclass_of_code(k, c) for c in codes]
    for c, q in zip(codes, cls):
        D = digraph_of_code(k, c)
        assert (q >= 0) == nx.is_weakly_connected(D)
        if q >= 0:
            assert nx.is_isomorphic(D, digraph_of_code(k, int(O.dclass_canon(k)[q])))
            perm = list(rng.permutation(k))
            assert O.dclass_of_code(k, code_of_digraph(k, D, perm)) == q
    for (c1, q1), (c2, q2) in itertools.islice(itertools.combinations(zip(codes, cls), 2), 3000):
        if q1 >= 0 and q2 >= 0:
            assert (q1 == q2) == nx.is_isomorphic(digraph_of_code(k, c1), digraph_of_code(k, c2))


DIGRAPHS = {
    "er14": lambda: gg.random_digraph(14, 30, 1, both=0.3),
    "er18": lambda: gg.random_digraph(18, 40, 2, both=0.1),
    "ba16": lambda: gg.orient(gg.barabasi_albert(16, 2, 3), 4, both=0.25),
    "tour6": lambda: gg.orient(gg.complete(9), 5, both=0.0),
}


@pytest.mark.parametrize("name", sorted(DIGRAPHS))
@pytest.mark.parametrize("k", [3, 4, 5])
def test_esu_equals_brute_force(name, k):
    d = DIGRAPHS[name]()
    b = O.dmotif_brute(d, k)
    assert np.array_equal(O.dmotif_count(d, k, threads=4), b)
    assert b.sum() > 0


@pytest.mark.parametrize("k", [3, 4, 5])
def test_closed_forms(k):
    # transitive tournament: every k-subset is the transitive tournament on k
    n = 9
    c = O.dmotif_count(gg.transitive_tournament(n), k)
    q = O.dclass_of_code(k, code_of_digraph(k, nx.DiGraph(gg_edges(gg.transitive_tournament(k))), range(k)))
    exp = np.zeros_like(c)
    exp[q] = math.comb(n, k)
    assert np.array_equal(c, exp)
    # directed cycle on n > k vertices: n directed paths
    c = O.dmotif_count(gg.directed_cycle(11), k)
    path = nx.DiGraph([(i, i + 1) for i in range(k - 1)])
    exp = np.zeros_like(c)
    exp[O.dclass_of_code(k, code_of_digraph(k, path, range(k)))] = 11
    assert np.array_equal(c, exp)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_mixed_star_closed_form(k):
    """A hub with out-, in- and two-way spokes (every third leaf of each kind):
    each weakly connected k-set is the hub plus k-1 leaves, in the class of the
    star with that many spokes of each kind, so class counts are sums of
    binomial products (the class read by networkx isomorphism, not the oracle)."""
    leaves = 14
    kinds = [j % 3 for j in range(leaves)]
    arcs = [(0, j + 1) for j, t in enumerate(kinds) if t in (0, 2)]
    arcs += [(j + 1, 0) for j, t in enumerate(kinds) if t in (1, 2)]
    c = O.dmotif_count(gg.digraph_from_arcs(leaves + 1, arcs), k)
    nk = [kinds.count(t) for t in range(3)]
    canon = O.dclass_canon(k)
    exp = np.zeros_like(c)
    for a in range(k):
        for b in range(k - a):
            star = nx.DiGraph()
            star.add_nodes_from(range(k))
            for i in range(1, k):
                t = 0 if i <= a else (1 if i <= a + b else 2)
                if t in (0, 2):
                    star.add_edge(0, i)
                if t in (1, 2):
                    star.add_edge(i, 0)
            q = [c_ for c_ in range(len(canon))
                 if nx.is_isomorphic(digraph_of_code(k, int(canon[c_])), star)]
            assert len(q) == 1
            exp[q[0]] += math.comb(nk[0], a) * math.comb(nk[1], b) * math.comb(nk[2], k - 1 - a - b)
    assert np.array_equal(c, exp)
    assert int(c.sum()) == math.comb(leaves, k - 1)


def gg_edges(d):
    return [(v, int(u)) for v in range(d.n) for u in d.col[d.row_ptr[v]:d.row_ptr[v + 1]]]


@pytest.mark.parametrize("k", [3, 4, 5])
def test_symmetric_digraph_equals_undirected_counts(k):
    """Both arcs on every edge: each undirected class maps to the directed
    class with both bits set on each of its edges, with the same count."""
    g = gg.barabasi_albert(40, 3, 7)
    dc = O.dmotif_count(gg.symmetric(g), k, threads=4)
    uc = O.motif_count(g, k)
    exp = np.zeros_like(dc)
    for cls, ucode in enumerate(O.class_canon(k)):
        dcode = 0
        for p in range(k * (k - 1) // 2):
            if int(ucode) >> p & 1:
                dcode |= 3 << (2 * p)
        exp[O.dclass_of_code(k, dcode)] += uc[cls]
    assert np.array_equal(dc, exp)
    assert exp.sum() > 0


@pytest.mark.parametrize("k", [3, 4])
def test_reversal_permutes_classes(k):
    d = gg.random_digraph(20, 50, 9, both=0.2)
    c = O.dmotif_count(d, k)
    r = O.dmotif_count(gg.reverse(d), k)
    canon = O.dclass_canon(k)
    exp = np.zeros_like(c)
    for q in range(len(canon)):
        exp[O.dclass_of_code(k, reverse_code(k, int(canon[q])))] += c[q]
    assert np.array_equal(r, exp)
