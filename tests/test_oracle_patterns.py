"""Pins of the oracle's pattern counting (subgraph matching, CPU only): the
definition (edge-preserving injective maps / automorphisms) against
networkx's VF2 monomorphism and isomorphism matchers, undirected and
directed, and against closed forms (wedges, stars, triangles, induced counts
= motif class counts)."""
import math

import networkx as nx
import numpy as np
import pytest
from networkx.algorithms import isomorphism as iso

import oracle as O
from paper_2212_04551_amd import graphgen as gg


def pbit(t, i):
    return i * (i - 1) // 2 + t


def nx_of(g, directed=False):
    G = nx.DiGraph() if directed else nx.Graph()
    G.add_nodes_from(range(g.n))
    G.add_edges_from((v, int(u)) for v in range(g.n) for u in g.col[g.row_ptr[v]:g.row_ptr[v + 1]])
    return G


def nx_pattern(k, code, directed=False):
    P = nx.DiGraph() if directed else nx.Graph()
    P.add_nodes_from(range(k))
    for i in range(1, k):
        for t in range(i):
            p = pbit(t, i)
            if directed:
                if code >> (2 * p) & 1:
                    P.add_edge(t, i)
                if code >> (2 * p + 1) & 1:
                    P.add_edge(i, t)
            elif code >> p & 1:
                P.add_edge(t, i)
    return P


def nx_count(G, P, induced, directed):
    M = iso.DiGraphMatcher if directed else iso.GraphMatcher
    it = M(G, P).subgraph_isomorphisms_iter() if induced else M(G, P).subgraph_monomorphisms_iter()
    emb = sum(1 for _ in it)
    aut = sum(1 for _ in M(P, P).isomorphisms_iter())
    assert emb % aut == 0
    return emb // aut


def random_connected_codes(k, directed, count, seed):
    rng = np.random.default_rng(seed)
    bits = k * (k - 1) if directed else k * (k - 1) // 2
    out = []
    while len(out) < count:
        c = int(rng.integers(1, 1 << bits))
        P = nx_pattern(k, c, directed)
        if (nx.is_weakly_connected(P) if directed else nx.is_connected(P)):
            out.append(c)
    return out


@pytest.mark.parametrize("k", [3, 4, 5])
@pytest.mark.parametrize("induced", [False, True])
def test_undirected_against_networkx(k, induced):
    g = gg.erdos_renyi(13, 32, 40 + k)
    G = nx_of(g)
    for c in random_connected_codes(k, False, 6, k):
        assert O.pattern_count_brute(g, k, c, induced=induced) == nx_count(G, nx_pattern(k, c), induced, False), c


@pytest.mark.parametrize("k", [3, 4])
@pytest.mark.parametrize("induced", [False, True])
def test_directed_against_networkx(k, induced):
    d = gg.random_digraph(11, 26, 50 + k, both=0.3)
    G = nx_of(d, directed=True)
    for c in random_connected_codes(k, True, 6, 10 + k):
        assert O.pattern_count_brute(d, k, c, induced=induced, directed=True) == \
            nx_count(G, nx_pattern(k, c, True), induced, True), c


def test_closed_forms():
    g = gg.erdos_renyi(16, 40, 7)
    deg = g.degrees()
    G = nx_of(g)
    for k in (3, 4, 5):
        star = sum(1 << pbit(0, i) for i in range(1, k))
        assert O.pattern_count_brute(g, k, star) == sum(math.comb(int(d), k - 1) for d in deg)
    assert O.pattern_count_brute(g, 3, 0b111) == sum(nx.triangles(G).values()) // 3
    # induced copies of a pattern = the motif count of its class
    for k in (3, 4):
        mc = O.motif_brute(g, k)
        for c in random_connected_codes(k, False, 4, 3):
            assert O.pattern_count_brute(g, k, c, induced=True) == int(mc[O.class_of_code(k, c)])
