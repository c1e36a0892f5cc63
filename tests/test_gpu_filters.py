"""Property filters (Section II's property P): a vertex predicate through
dm_induced_subgraph (e.g. vertex labels in an allowed set), and the
quasi-clique density threshold through dm_count_quasi_cliques, against the
oracle on the same inputs.  All calls go through the C ABI."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2212_04551_amd import dm
from paper_2212_04551_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def test_vertex_label_filter_matches_oracle():
    """Vertex labels 0..3 (seeded); only subgraphs whose vertices all carry
    label 1 or 2 are counted and listed."""
    g = gg.chung_lu(3000, 15000, 2.2, 120.0, 12)[0]
    labels = np.random.default_rng(5).integers(0, 4, g.n)
    keep = (labels == 1) | (labels == 2)
    h = dm.load_graph(g)
    hs = dm.induced_subgraph(h, keep)
    sub = O.induced(g, keep)
    n, nnz = dm.graph_info(hs)
    assert (n, nnz) == (sub.n, sub.nnz)
    for k in (3, 4, 5):
        assert dm.count_cliques(hs, k) == O.clique_count(sub, k, threads=8), k
        assert np.array_equal(dm.count_motifs(hs, k), O.motif_count(sub, k, threads=8)), k
    rows = dm.list_subgraphs(hs, dm.DM_OP_CLIQUE, 3, wait_limit_us=20_000_000)
    assert len(rows) == O.clique_count(sub, 3)
    # all kept / none kept
    assert dm.count_cliques(dm.induced_subgraph(h, np.ones(g.n, bool)), 4) == O.clique_count(g, 4, threads=8)
    assert dm.graph_info(dm.induced_subgraph(h, np.zeros(g.n, bool))) == (0, 0)


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_quasi_cliques_match_oracle(k):
    # the oracle's class counts take about 4 s at k = 5 on BA(1500, 5) and
    # 3 s at k = 6 on BA(400, 3)
    g = gg.barabasi_albert(1500, 5, 20 + k) if k <= 5 else gg.barabasi_albert(400, 3, 20 + k)
    h = dm.load_graph(g)
    full = k * (k - 1) // 2
    cls = O.motif_count(g, k, threads=8)
    for m in sorted({0, k - 1, (full + k - 1) // 2, full - 1, full}):
        assert dm.count_quasi_cliques(h, k, m) == O.quasi_clique_count(g, k, m, class_counts=cls), (k, m)
    assert dm.count_quasi_cliques(h, k, full) == dm.count_cliques(h, k)
    assert dm.count_quasi_cliques(dm.load_graph(gg.complete(12)), k, full // 2) == math.comb(12, k)
    with pytest.raises(dm.DMError) as e:
        dm.count_quasi_cliques(h, k, full + 1)
    assert e.value.status == dm.DM_E_ARG
