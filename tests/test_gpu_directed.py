"""GPU parity of directed motif counting (k = 3..5) against the oracle:
digraphs loaded with dm_load_digraph (the underlying undirected graph plus
two arc bits per adjacency entry), counts exact (uint64) per class.  All calls
go through the C ABI."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2212_04551_amd import dm
from paper_2212_04551_amd import graphgen as gg

pytestmark = pytest.mark.gpu

GRAPHS = {
    "er300": lambda: gg.random_digraph(300, 900, 1, both=0.2),
    "ba400": lambda: gg.orient(gg.barabasi_albert(400, 3, 2), 3, both=0.3),
    "cl1500": lambda: gg.orient(gg.chung_lu(1500, 5000, 2.2, 40.0, 4)[0], 5, both=0.15),
    "sbm": lambda: gg.orient(gg.sbm(6, 12, 0.5, 0.03, 6), 7, both=0.5),
    "dag": lambda: gg.orient(gg.erdos_renyi(200, 800, 8), 9, both=0.0),
}


def pbit(t, i):
    return i * (i - 1) // 2 + t


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("k", [3, 4, 5])
def test_directed_motifs_match_oracle(name, k):
    d = GRAPHS[name]()
    h = dm.load_digraph(d)
    exp = O.dmotif_count(d, k, threads=8)
    got = dm.count_motifs_directed(h, k)
    assert np.array_equal(got, exp), (name, k)
    assert exp.sum() > 0
    # the same traversals, classified without directions, are the undirected counts
    urp, ucol = O.undirected_of(d)
    ug = gg.Graph(d.n, urp, ucol)
    assert np.array_equal(dm.count_motifs(h, k), O.motif_count(ug, k, threads=8))
    assert int(got.sum()) == int(dm.count_motifs(h, k).sum())


@pytest.mark.parametrize("k", [3, 4, 5])
def test_directed_closed_forms(k):
    # transitive tournament: C(n, k) in the transitive class
    n = 30
    got = dm.count_motifs_directed(dm.load_digraph(gg.transitive_tournament(n)), k)
    code = 0
    for i in range(1, k):
        for t in range(i):
            code |= 1 << (2 * pbit(t, i))
    exp = np.zeros_like(got)
    exp[O.dclass_of_code(k, code)] = math.comb(n, k)
    assert np.array_equal(got, exp)
    # directed cycle: n directed paths
    got = dm.count_motifs_directed(dm.load_digraph(gg.directed_cycle(50)), k)
    code = 0
    for i in range(1, k):
        code |= 1 << (2 * pbit(i - 1, i))
    exp = np.zeros_like(got)
    exp[O.dclass_of_code(k, code)] = 50
    assert np.array_equal(got, exp)
    # both arcs on every edge: the undirected class counts, mapped
    g = gg.chung_lu(1500, 6000, 2.3, 60.0, 11)[0]
    got = dm.count_motifs_directed(dm.load_digraph(gg.symmetric(g)), k)
    uc = dm.count_motifs(dm.load_graph(g), k)
    exp = np.zeros_like(got)
    for cls in range(dm.motif_num_classes(k)):
        ucode = O.class_canon(k)[cls]
        dcode = 0
        for p in range(k * (k - 1) // 2):
            if int(ucode) >> p & 1:
                dcode |= 3 << (2 * p)
        exp[O.dclass_of_code(k, dcode)] += uc[cls]
    assert np.array_equal(got, exp)


def test_directed_options_and_errors():
    d = GRAPHS["er300"]()
    h = dm.load_digraph(d)
    exp = O.dmotif_count(d, 4, threads=8)
    for kw in (dict(chunk=1), dict(chunk=64), dict(waves_per_cu=1), dict(sched=dm.DM_NO_DONATION)):
        assert np.array_equal(dm.count_motifs_directed(h, 4, **kw), exp), kw
    assert dm.digraph_info(h) == (1, d.arcs)
    assert dm.digraph_info(dm.load_graph(gg.erdos_renyi(20, 40, 1))) == (0, 0)
    for k in (2, 6):
        with pytest.raises(dm.DMError) as e:
            dm.count_motifs_directed(h, k)
        assert e.value.status == dm.DM_E_K
    with pytest.raises(dm.DMError) as e:
        dm.count_motifs_directed(dm.load_graph(gg.erdos_renyi(20, 40, 1)), 3)
    assert e.value.status == dm.DM_E_ARG
    with pytest.raises(dm.DMError) as e:
        dm.count_motifs_directed(h, 3, sched=dm.DM_SCHED_AUTOTUNE)
    assert e.value.status == dm.DM_E_ARG
    # empty and arc-free digraphs
    assert not dm.count_motifs_directed(dm.load_digraph(gg.digraph_from_arcs(10, [])), 3).any()
    assert not dm.count_motifs_directed(dm.load_digraph(gg.digraph_from_arcs(0, [])), 3).any()


@pytest.mark.parametrize("k,leaves", [(4, 1500), (5, 700)])
def test_directed_star_launch_shapes(k, leaves):
    """A hub with out-, in- and two-way spokes: every weakly connected k-set
    is the hub plus k-1 leaves, its class fixed by how many spokes of each
    kind it holds (a closed form).  The leaf roots' level k-2 lists run from
    about `leaves` entries down to none, so launches planned for different
    resident-wave caps keep some of them in LDS and some in HBM."""
    kinds = [j % 3 for j in range(leaves)]  # 0: hub -> leaf, 1: leaf -> hub, 2: both
    arcs = []
    for j, t in enumerate(kinds):
        if t in (0, 2):
            arcs.append((0, j + 1))
        if t in (1, 2):
            arcs.append((j + 1, 0))
    h = dm.load_digraph(gg.digraph_from_arcs(leaves + 1, arcs))
    nk = [kinds.count(t) for t in range(3)]
    exp = np.zeros(dm.motif_directed_num_classes(k), dtype=np.uint64)
    for a in range(k):
        for b in range(k - a):
            c = k - 1 - a - b
            code = 0
            for i in range(1, k):  # the hub at position 0, leaves 1..k-1
                t = 0 if i <= a else (1 if i <= a + b else 2)
                if t in (0, 2):
                    code |= 1 << (2 * pbit(0, i))
                if t in (1, 2):
                    code |= 1 << (2 * pbit(0, i) + 1)
            exp[O.dclass_of_code(k, code)] += math.comb(nk[0], a) * math.comb(nk[1], b) * math.comb(nk[2], c)
    for cap in (0, 4, 1) if k == 4 else (0, 4):
        assert np.array_equal(dm.count_motifs_directed(h, k, waves_per_cu=cap), exp), (k, cap)


def test_directed_counts_ignore_vertex_ids():
    """The kernel renames vertices by (degree, id) rank and roots each
    subgraph at its lowest rank; the class counts depend on the digraph only,
    so any renaming of the input ids gives the same counts (hubs at the lowest
    ids, at the highest, or shuffled)."""
    d = GRAPHS["cl1500"]()
    src = np.repeat(np.arange(d.n), np.diff(d.row_ptr))
    arcs = np.stack([src, d.col.astype(np.int64)], axis=1)
    deg = np.bincount(arcs.ravel(), minlength=d.n)
    orders = {
        "hubs_first": np.argsort(-deg, kind="stable"),
        "hubs_last": np.argsort(deg, kind="stable"),
        "shuffled": np.random.default_rng(21).permutation(d.n),
    }
    base = {k: dm.count_motifs_directed(dm.load_digraph(d), k) for k in (3, 4, 5)}
    for name, order in orders.items():
        new_id = np.empty(d.n, dtype=np.int64)
        new_id[order] = np.arange(d.n)
        h = dm.load_digraph(gg.digraph_from_arcs(d.n, new_id[arcs].tolist()))
        for k in (3, 4, 5):
            assert np.array_equal(dm.count_motifs_directed(h, k), base[k]), (name, k)


def test_directed_device_input_and_validation():
    import torch
    d = GRAPHS["ba400"]()
    rp = torch.from_numpy(d.row_ptr).cuda()
    col = torch.from_numpy(d.col).cuda()
    h = dm.load_digraph_device(d.n, rp, col)
    assert np.array_equal(dm.count_motifs_directed(h, 3), O.dmotif_count(d, 3))
    bad = [
        gg.Digraph(3, np.array([0, 1, 1, 1], np.int64), np.array([0], np.int32)),           # self-arc
        gg.Digraph(3, np.array([0, 2, 2, 2], np.int64), np.array([2, 1], np.int32)),        # unsorted
        gg.Digraph(3, np.array([0, 1, 1, 1], np.int64), np.array([7], np.int32)),           # out of range
    ]
    for b in bad:
        with pytest.raises(dm.DMError) as e:
            dm.load_digraph(b)
        assert e.value.status == dm.DM_E_CSR
        with pytest.raises(dm.DMError) as e:
            dm.load_digraph_device(b.n, torch.from_numpy(b.row_ptr).cuda(), torch.from_numpy(b.col).cuda())
        assert e.value.status == dm.DM_E_CSR


def _reverse_code(k, code):
    r = 0
    for p in range(k * (k - 1) // 2):
        if code >> (2 * p) & 1:
            r |= 1 << (2 * p + 1)
        if code >> (2 * p + 1) & 1:
            r |= 1 << (2 * p)
    return r


def test_directed_invariants_at_scale():
    """A 10^5-vertex power-law graph (m = 5*10^5, cap 100): with both arcs on
    every edge the directed counts are the oracle's undirected class counts
    mapped to two-arc codes (k = 3, 4) and the GPU's (k = 5); on a random
    orientation the counts sum to the oracle's connected-set count (k = 3, 4),
    and reversing every arc permutes the classes by the reversed codes."""
    g = gg.chung_lu(100_000, 500_000, 2.3, 100.0, 0)[0]
    hs = dm.load_digraph(gg.symmetric(g))
    oc = {k: O.motif_count(g, k, threads=8) for k in (3, 4)}
    for k in (3, 4, 5):
        uc = oc[k] if k <= 4 else dm.count_motifs(hs, k)
        exp = np.zeros(dm.motif_directed_num_classes(k), np.uint64)
        for cls in range(dm.motif_num_classes(k)):
            ucode = int(O.class_canon(k)[cls])
            dcode = 0
            for p in range(k * (k - 1) // 2):
                if ucode >> p & 1:
                    dcode |= 3 << (2 * p)
            exp[O.dclass_of_code(k, dcode)] += uc[cls]
        assert np.array_equal(dm.count_motifs_directed(hs, k), exp), k
    d = gg.orient(g, 1, both=0.2)
    h = dm.load_digraph(d)
    hr = dm.load_digraph(gg.reverse(d))
    for k in (3, 4, 5):
        c = dm.count_motifs_directed(h, k)
        if k <= 4:
            assert int(c.sum()) == int(oc[k].sum()), k
        canon = O.dclass_canon(k)
        exp = np.zeros_like(c)
        for q in range(len(canon)):
            exp[O.dclass_of_code(k, _reverse_code(k, int(canon[q])))] += c[q]
        assert np.array_equal(dm.count_motifs_directed(hr, k), exp), k
