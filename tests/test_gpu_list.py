"""aggregate_store (Section IV-C; Table II): dm_list hands every k-clique and
every connected induced k-subgraph to a host sink exactly once.  Checked
against the oracle's listings (as sets of vertex sets, with class ids for
motifs), and on outputs larger than the host ring (wrap-around) against
closed forms and the counting kernels.  Every call bounds the kernel's wait
for the host to 20 s."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2212_04551_amd import dm
from paper_2212_04551_amd import graphgen as gg

pytestmark = pytest.mark.gpu

WAIT = dict(wait_limit_us=20_000_000)


def as_sets(rows, k, with_class=False):
    v = np.sort(rows[:, :k].astype(np.int64), axis=1)
    if with_class:
        v = np.concatenate([v, rows[:, k:k + 1].astype(np.int64)], axis=1)
    return v[np.lexsort(v.T[::-1])]


@pytest.mark.parametrize("make", [lambda: gg.erdos_renyi(40, 260, 1), lambda: gg.erdos_renyi(300, 4000, 2),
                                  lambda: gg.barabasi_albert(200, 6, 3)], ids=["er40", "er300", "ba200"])
def test_clique_listing_matches_oracle(make):
    g = make()
    h = dm.load_graph(g)
    for k in (1, 2, 3, 4, 5):
        rows = dm.list_subgraphs(h, dm.DM_OP_CLIQUE, k, **WAIT)
        exp = O.clique_list(g, k)
        assert rows.shape == exp.shape, k
        assert np.array_equal(as_sets(rows, k), exp), k
        assert len(rows) == dm.count_cliques(h, k), k


def test_clique_listing_wraps_the_ring():
    """K_40, k = 5: C(40,5) = 658,008 rows, more than the ring's 524,288
    slots; every row a distinct 5-subset; a streaming sink sees the same."""
    h = dm.load_graph(gg.complete(40))
    rows = dm.list_subgraphs(h, dm.DM_OP_CLIQUE, 5, **WAIT)
    assert len(rows) == math.comb(40, 5)
    s = as_sets(rows, 5)
    assert (np.diff(s, axis=1) > 0).all()
    assert len(np.unique(s, axis=0)) == len(s)
    seen = [0]

    def sink(batch):
        assert batch.shape[1] == 5 and batch.min() >= 0 and batch.max() < 40
        seen[0] += len(batch)

    assert dm.list_subgraphs(h, dm.DM_OP_CLIQUE, 5, sink=sink, **WAIT) == math.comb(40, 5) == seen[0]


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_motif_listing_matches_oracle(k):
    g = gg.barabasi_albert(30 if k < 6 else 22, 2, k)
    h = dm.load_graph(g)
    rows = dm.list_subgraphs(h, dm.DM_OP_MOTIF, k, **WAIT)
    exp = O.motif_list(g, k)
    assert rows.shape == exp.shape
    assert np.array_equal(as_sets(rows, k, with_class=True), exp)


@pytest.mark.parametrize("k,n,m", [(5, 400, 1400), (7, 200, 420)])
def test_motif_listing_large_against_counts(k, n, m):
    """Sparse graphs with more rows than the ring (883,604 5-subgraphs;
    2,188,931 7-subgraphs): the class histogram of the listing equals
    dm_count_motifs, no vertex set repeats, and each row's first vertex is its
    lowest-(degree, id) vertex."""
    g = gg.erdos_renyi(n, m, 5)
    h = dm.load_graph(g)
    deg = g.degrees()
    rows = dm.list_subgraphs(h, dm.DM_OP_MOTIF, k, **WAIT)
    cnt = dm.count_motifs(h, k)
    assert np.array_equal(np.bincount(rows[:, k], minlength=len(cnt)).astype(np.uint64), cnt)
    s = as_sets(rows, k)
    assert len(np.unique(s, axis=0)) == len(s)
    key = deg[rows[:, :k]].astype(np.int64) * g.n + rows[:, :k]
    assert (key[:, 0] == key.min(axis=1)).all()
    assert len(rows) > 8 * 65536


def test_listing_argument_errors():
    h = dm.load_graph(gg.complete(5))
    with pytest.raises(dm.DMError) as e:
        dm.list_subgraphs(h, dm.DM_OP_MOTIF, 9)
    assert e.value.status == dm.DM_E_K
    with pytest.raises(dm.DMError) as e:
        dm.list_subgraphs(h, dm.DM_OP_CLIQUE, 3, sched=dm.DM_SCHED_LEARNED)
    assert e.value.status == dm.DM_E_ARG
