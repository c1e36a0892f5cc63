"""Subgraph matching on the GPU (dm_count_pattern: induced and non-induced
copies of a connected pattern, from the motif kernels' class counts) against
the oracle's definition-level count and closed forms.  All calls go through
the C ABI."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2212_04551_amd import dm
from paper_2212_04551_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def pbit(t, i):
    return i * (i - 1) // 2 + t


def code_of(k, edges, directed=False):
    c = 0
    for a, b in edges:
        if directed:
            c |= 1 << (2 * pbit(a, b)) if a < b else 1 << (2 * pbit(b, a) + 1)
        else:
            c |= 1 << pbit(min(a, b), max(a, b))
    return c


UNDIRECTED = {
    3: [[(0, 1), (1, 2)], [(0, 1), (1, 2), (0, 2)]],
    4: [[(0, 1), (1, 2), (2, 3)], [(0, 1), (0, 2), (0, 3)], [(0, 1), (1, 2), (2, 3), (3, 0)],
        [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)]],
    5: [[(0, 1), (1, 2), (2, 3), (3, 4)], [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4)],
        [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)]],
}


@pytest.mark.parametrize("k", [3, 4, 5])
def test_patterns_match_oracle(k):
    for g in (gg.erdos_renyi(18, 48, 3), gg.barabasi_albert(20, 2, 4)):
        h = dm.load_graph(g)
        for edges in UNDIRECTED[k]:
            c = code_of(k, edges)
            for induced in (False, True):
                assert dm.count_pattern(h, k, c, induced=induced) == \
                    O.pattern_count_brute(g, k, c, induced=induced), (k, edges, induced)


def test_pattern_closed_forms_up_to_k8():
    # k <= 5 on a power-law graph; k = 6..8 on a sparse graph plus a K_10 (the
    # power-law graph's hubs would make the 8-vertex enumeration run for minutes)
    big = gg.chung_lu(1500, 6000, 2.3, 60.0, 11)[0]
    small, _ = gg.disjoint_union([gg.erdos_renyi(200, 500, 12), gg.complete(10)])
    for k in range(3, 9):
        g = big if k <= 5 else small
        h = dm.load_graph(g)
        deg = g.degrees()
        star = code_of(k, [(0, i) for i in range(1, k)])
        assert dm.count_pattern(h, k, star) == sum(math.comb(int(d), k - 1) for d in deg), k
        full = code_of(k, [(a, b) for b in range(k) for a in range(b)])
        assert dm.count_pattern(h, k, full) == dm.count_cliques(h, k) == dm.count_pattern(h, k, full, induced=True)
        if k > 5:
            assert dm.count_cliques(h, k) == math.comb(10, k)
    g = big
    h = dm.load_graph(g)
    # induced copies are the motif count of the pattern's class
    for k in (4, 5):
        mc = dm.count_motifs(h, k)
        for edges in UNDIRECTED[k]:
            c = code_of(k, edges)
            assert dm.count_pattern(h, k, c, induced=True) == int(mc[O.class_of_code(k, c)])


def test_directed_patterns():
    for d in (gg.random_digraph(14, 40, 5, both=0.3), gg.orient(gg.barabasi_albert(16, 2, 6), 7, both=0.2)):
        h = dm.load_digraph(d)
        for k, arcs in ((3, [(0, 1), (1, 2)]), (3, [(0, 1), (1, 2), (2, 0)]), (3, [(0, 1), (1, 0), (1, 2)]),
                        (4, [(0, 1), (1, 2), (2, 3)]), (4, [(0, 1), (0, 2), (0, 3), (1, 2)])):
            c = code_of(k, arcs, directed=True)
            for induced in (False, True):
                assert dm.count_pattern(h, k, c, induced=induced, directed=True) == \
                    O.pattern_count_brute(d, k, c, induced=induced, directed=True), (k, arcs, induced)
    # a directed path of k vertices in a directed n-cycle: n copies; transitive tournaments: C(n, k)
    for k in (3, 4, 5):
        path = code_of(k, [(i, i + 1) for i in range(k - 1)], directed=True)
        assert dm.count_pattern(dm.load_digraph(gg.directed_cycle(40)), k, path, directed=True) == 40
        tt = code_of(k, [(a, b) for b in range(k) for a in range(b)], directed=True)
        assert dm.count_pattern(dm.load_digraph(gg.transitive_tournament(20)), k, tt, directed=True) == \
            math.comb(20, k)


def test_pattern_errors():
    h = dm.load_graph(gg.erdos_renyi(20, 40, 1))
    for k, code, flags, status in ((4, code_of(4, [(0, 1), (2, 3)]), {}, dm.DM_E_ARG),
                                   (9, 1, {}, dm.DM_E_K),
                                   (3, 1 << 5, {}, dm.DM_E_ARG),
                                   (6, 1, {"directed": True}, dm.DM_E_K)):
        with pytest.raises(dm.DMError) as e:
            dm.count_pattern(h, k, code, **flags)
        assert e.value.status == status, (k, code, flags)
