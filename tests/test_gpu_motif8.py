"""GPU parity of induced 8-vertex motif counting (11,117 classes, the
2^27-entry dictionary, per-wave class counters in global memory) against the
oracle, exactly (uint64).  The oracle's 8-vertex class table takes about a
minute to build, so the expected counts were written by
tests/golden/make_motif8.py (oracle only) and are read here.  All calls go
through the C ABI."""
import math
import os

import numpy as np
import pytest

from paper_2212_04551_amd import dm
from paper_2212_04551_amd import graphgen as gg

pytestmark = pytest.mark.gpu

K = 8
NCLS = 11117
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "motif8_expected.txt")


def read_fixture():
    canon, patterns, graphs = None, {}, {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            if p[0] == "canon":
                canon = [int(x) for x in p[1:]]
            elif p[0] == "pattern":
                patterns[p[1]] = int(p[2])
            elif p[0] == "graph":
                c = np.zeros(NCLS, np.uint64)
                for kv in p[5:]:
                    i, v = kv.split(":")
                    c[int(i)] = int(v)
                graphs[p[1]] = (int(p[2]), int(p[3]), int(p[4]), c)
    return canon, patterns, graphs


FIX = read_fixture()
RANDOM8 = {
    "er60": lambda: gg.erdos_renyi(60, 130, 1),
    "ba50": lambda: gg.barabasi_albert(50, 2, 2),
    "cl400": lambda: gg.chung_lu(400, 700, 2.3, 15.0, 3)[0],
    "sbm": lambda: gg.sbm(6, 10, 0.4, 0.05, 4),
}


def expected(name, g):
    n, nnz, fnv, c = FIX[2][name]
    assert (g.n, g.nnz, gg.fnv1a64(g)) == (n, nnz, fnv), f"{name}: generator output changed"
    return c


def test_classes_match_oracle_numbering():
    canon = FIX[0]
    assert dm.motif_num_classes(K) == NCLS == len(canon)
    for c in range(0, NCLS, 97):
        assert dm.motif_class_mask(K, c) == canon[c]


def test_closed_forms_k8():
    pat = FIX[1]
    for G, cls, count in [
        (gg.path(40), pat["path"], 40 - K + 1),
        (gg.cycle(31), pat["path"], 31),
        (gg.cycle(8), pat["cycle"], 1),
        (gg.star(20), pat["star"], math.comb(20, K - 1)),
        (gg.complete(12), pat["complete"], math.comb(12, K)),
    ]:
        exp = np.zeros(NCLS, np.uint64)
        exp[cls] = count
        assert np.array_equal(dm.count_motifs(dm.load_graph(G), K), exp), G.n
    assert not dm.count_motifs(dm.load_graph(gg.empty(30)), K).any()


@pytest.mark.parametrize("name", sorted(RANDOM8))
def test_random_graphs_k8(name):
    g = RANDOM8[name]()
    exp = expected(name, g)
    assert exp.sum() > 0
    h = dm.load_graph(g)
    assert np.array_equal(dm.count_motifs(h, K), exp), name
    assert np.array_equal(dm.count_motifs(h, K, chunk=1, rebalance=0.01), exp), name
    assert np.array_equal(dm.count_motifs(h, K, sched=dm.DM_NO_DONATION, waves_per_cu=1), exp), name


def test_sampled_eight_vertex_graphs_batched():
    """302 of the 2^28 labelled 8-vertex graphs (fixed stride) in one dm_batch
    launch, against the oracle's brute-force classification."""
    pairs = [(i, j) for i in range(K) for j in range(i + 1, K)]
    names = sorted((n for n in FIX[2] if n.startswith("mask")), key=lambda s: int(s[4:]))
    graphs = [gg.from_edges(K, [p for b, p in enumerate(pairs) if int(n[4:]) >> b & 1]) for n in names]
    exp = np.stack([expected(n, g) for n, g in zip(names, graphs)])
    got = dm.batch([dm.load_graph(g) for g in graphs], dm.DM_OP_MOTIF, K)
    assert np.array_equal(got, exp)
    # one class per connected graph, none for a disconnected one; 133 of the
    # 302 sampled graphs are connected
    assert exp.sum(axis=1).max() == 1 and exp.sum() == 133


def test_listing_k8_histogram():
    """dm_list at k = 8: the class histogram of the listed subgraphs equals
    the oracle's counts."""
    g = RANDOM8["er60"]()
    rows = dm.list_subgraphs(dm.load_graph(g), dm.DM_OP_MOTIF, K, wait_limit_us=20_000_000)
    assert np.array_equal(np.bincount(rows[:, K], minlength=NCLS).astype(np.uint64), expected("er60", g))


def test_k8_limits():
    h = dm.load_graph(gg.complete(10), rank=True)
    with pytest.raises(dm.DMError) as e:
        dm.count_motifs(h, K, sched=dm.DM_IMPL_DFS)
    assert e.value.status == dm.DM_E_K
    with pytest.raises(dm.DMError) as e:
        dm.count_motifs_static(h, K)
    assert e.value.status == dm.DM_E_K
