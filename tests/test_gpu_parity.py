"""GPU parity: every count from the HIP library equals the CPU oracle exactly
(uint64), on closed-form families, exhaustive tiny graphs, seeded random
graphs with ragged sizes (several 64-bit tiles plus a tail), per-root records,
and under every scheduling knob.  All calls go through the C ABI."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2212_04551_amd import dm
from paper_2212_04551_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def _esym(parts, k):
    poly = np.array([1], dtype=object)
    for a in parts:
        poly = np.convolve(poly, np.array([1, a], dtype=object))
    return int(poly[k]) if k < len(poly) else 0


def cliques(g, k, **kw):
    h = dm.load_graph(g)
    return dm.count_cliques(h, k, **kw)


def motifs(g, k, **kw):
    h = dm.load_graph(g)
    return dm.count_motifs(h, k, **kw)


def test_native_library_is_loaded():
    dm.lib()
    maps = open("/proc/self/maps").read()
    assert "libdumato_mi.so" in maps


# ------------------------------------------------------------------ closed forms

@pytest.mark.parametrize("n", [1, 2, 5, 30, 65, 130])
def test_clique_complete(n):
    """K_n: C(n, k); k is kept where the (k-2)-clique level stays below ~1e7 nodes."""
    h = dm.load_graph(gg.complete(n))
    for k in range(1, n + 2):
        if k > 2 and math.comb(n, k - 2) > 10_000_000:
            break
        assert dm.count_cliques(h, k) == math.comb(n, k), (n, k)


def test_clique_large_k_complete():
    """K_40 at k = 10..12 (non-zero large-k counts, C(40, 12) = 5,586,853,480),
    with the default schedule and with small chunks on one wave per CU."""
    h = dm.load_graph(gg.complete(40))
    for k in (10, 11, 12):
        assert dm.count_cliques(h, k) == math.comb(40, k), k
        assert dm.count_cliques(h, k, chunk=3, waves_per_cu=1) == math.comb(40, k), k


def test_clique_dense_wide_roots():
    """Cocktail party on 80 pairs (160 vertices, degree 158): roots wider than
    128 keep their rows in global memory and hand dense re-indexed sets with
    5 or more levels to the solver, which splits them among idle waves.
    Closed form C(80, k) 2^k."""
    h = dm.load_graph(gg.cocktail_party(80))
    for k in (5, 6, 7):
        assert dm.count_cliques(h, k) == math.comb(80, k) * 2 ** k, k


@pytest.mark.parametrize("parts", [[3] * 12, [1, 2, 3, 4, 5, 6, 7], [2] * 9, [40, 1, 1, 25]])
def test_clique_multipartite(parts):
    h = dm.load_graph(gg.complete_multipartite(parts))
    for k in range(1, len(parts) + 2):
        assert dm.count_cliques(h, k) == _esym(parts, k), (parts, k)


def test_clique_global_rows_path():
    """Out-degrees up to 897: bitmap rows exceed LDS and live in global scratch."""
    parts = [3] * 300
    h = dm.load_graph(gg.complete_multipartite(parts))
    for k in (3, 4):
        assert dm.count_cliques(h, k) == _esym(parts, k), k


@pytest.mark.parametrize("g", [gg.complete_bipartite(70, 90), gg.hypercube(7), gg.cycle(200), gg.star(300),
                               gg.empty(50), gg.path(129)], ids=["K70,90", "Q7", "C200", "S300", "E50", "P129"])
def test_clique_bipartite_zero(g):
    h = dm.load_graph(g)
    assert dm.count_cliques(h, 1) == g.n
    assert dm.count_cliques(h, 2) == g.m
    for k in range(3, 7):
        assert dm.count_cliques(h, k) == 0


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_motif_closed_forms(k):
    ncls = dm.motif_num_classes(k)
    for G, n_expected_class_pattern, count in [
        (gg.path(150), gg.path(k), 150 - k + 1),
        (gg.cycle(131), gg.path(k), 131),
        (gg.star(200), gg.star(k - 1), math.comb(200, k - 1)),
        (gg.complete(20), gg.complete(k), math.comb(20, k)),
    ]:
        cls = int(np.nonzero(O.motif_brute(n_expected_class_pattern, k))[0][0])
        exp = np.zeros(ncls, np.uint64)
        exp[cls] = count
        assert np.array_equal(motifs(G, k), exp), (k, G.n)
    assert not motifs(gg.empty(40), k).any()


def test_motif_complete_bipartite():
    a, b = 70, 65
    g = gg.complete_bipartite(a, b)
    c4 = int(np.nonzero(O.motif_brute(gg.cycle(4), 4))[0][0])
    s3 = int(np.nonzero(O.motif_brute(gg.star(3), 4))[0][0])
    exp = np.zeros(6, np.uint64)
    exp[c4] = math.comb(a, 2) * math.comb(b, 2)
    exp[s3] = a * math.comb(b, 3) + b * math.comb(a, 3)
    assert np.array_equal(motifs(g, 4), exp)


def test_motif_long_leaf_lists():
    """Leaf-level lists longer than the LDS copy (800 entries) stay in global
    memory behind two LDS membership filters.  K_{820,860}: at k=3 every list
    is one side (820 entries, all neighbours of an entry are non-members); at
    k=4 a list holds both sides (about 1680 entries, the neighbours of an
    entry are members).  Closed forms: paths of 3 = a C(b,2) + b C(a,2);
    4-cycles C(a,2) C(b,2), 3-stars a C(b,3) + b C(a,3)."""
    a, b = 820, 860
    g = gg.complete_bipartite(a, b)
    p3 = int(np.nonzero(O.motif_brute(gg.path(3), 3))[0][0])
    exp3 = np.zeros(2, np.uint64)
    exp3[p3] = a * math.comb(b, 2) + b * math.comb(a, 2)
    assert np.array_equal(motifs(g, 3), exp3)
    c4 = int(np.nonzero(O.motif_brute(gg.cycle(4), 4))[0][0])
    s3 = int(np.nonzero(O.motif_brute(gg.star(3), 4))[0][0])
    exp4 = np.zeros(6, np.uint64)
    exp4[c4] = math.comb(a, 2) * math.comb(b, 2)
    exp4[s3] = a * math.comb(b, 3) + b * math.comb(a, 3)
    assert np.array_equal(motifs(g, 4), exp4)


def test_motif_hub_lists_match_oracle():
    """A sparse graph with two adjacent hubs of degree 850: the lists of
    traversals through a hub exceed the LDS copy, and most neighbours looked
    up in them are absent (filter rejections and false positives)."""
    rng = np.random.default_rng(11)
    base = gg.erdos_renyi(3000, 9000, 3)
    src = np.repeat(np.arange(base.n), np.diff(base.row_ptr))
    edges = set((int(x), int(y)) for x, y in zip(src, base.col) if x < y)
    for hub in (3000, 3001):
        for v in rng.choice(3000, 850, replace=False):
            edges.add((int(v), hub))
    edges.add((3000, 3001))
    g = gg.from_edges(3002, sorted(edges))
    for k in (3, 4):
        assert np.array_equal(motifs(g, k), O.motif_count(g, k, threads=8)), k


# ------------------------------------------------------------------ exhaustive tiny graphs

def _all_graphs(n):
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    for mask in range(1 << len(pairs)):
        yield gg.from_edges(n, [p for b, p in enumerate(pairs) if mask >> b & 1])


def test_exhaustive_five_vertices_batched():
    graphs = list(_all_graphs(5))
    hs = [dm.load_graph(g) for g in graphs]
    for k in (3, 4, 5):
        got = dm.batch(hs, dm.DM_OP_MOTIF, k)
        exp = np.stack([O.motif_brute(g, k) for g in graphs])
        assert np.array_equal(got, exp), k
        got = dm.batch(hs, dm.DM_OP_CLIQUE, k)[:, 0]
        exp = np.array([O.clique_brute(g, k) for g in graphs], np.uint64)
        assert np.array_equal(got, exp), k


def test_exhaustive_six_vertices_sampled():
    pairs = [(i, j) for i in range(6) for j in range(i + 1, 6)]
    graphs = [gg.from_edges(6, [p for b, p in enumerate(pairs) if m >> b & 1]) for m in range(0, 1 << 15, 37)]
    hs = [dm.load_graph(g) for g in graphs]
    for k in (4, 5, 6):
        got = dm.batch(hs, dm.DM_OP_MOTIF, k)
        exp = np.stack([O.motif_brute(g, k) for g in graphs])
        assert np.array_equal(got, exp), k


# ------------------------------------------------------------------ seeded random graphs

def test_er516_motifs_and_cliques():
    g = gg.workload_graph("er516", 0)
    h = dm.load_graph(g)
    for k in (3, 4, 5, 6):
        assert np.array_equal(dm.count_motifs(h, k), O.motif_count(g, k, threads=8)), k
    for k in range(1, 9):
        assert dm.count_cliques(h, k) == O.clique_count(g, k), k


RANDOM = [
    ("er", lambda s: gg.erdos_renyi(300, 9000, s)),       # dense: out-degrees span 2-3 tiles
    ("er_sparse", lambda s: gg.erdos_renyi(2000, 6000, s)),
    ("ba", lambda s: gg.barabasi_albert(1500, 5, s)),     # hubs: long neighbour scans
    ("cl", lambda s: gg.chung_lu(3000, 12000, 2.2, 80.0, s)[0]),
    ("sbm", lambda s: gg.sbm(12, 40, 0.5, 0.01, s)),
]


@pytest.mark.parametrize("name,make", RANDOM, ids=[r[0] for r in RANDOM])
@pytest.mark.parametrize("seed", [1, 2])
def test_random_graphs_cliques(name, make, seed):
    g = make(seed)
    h = dm.load_graph(g)
    for k in range(3, 8):
        assert dm.count_cliques(h, k) == O.clique_count(g, k, threads=8), (name, seed, k)


@pytest.mark.parametrize("name,make", RANDOM, ids=[r[0] for r in RANDOM])
@pytest.mark.parametrize("seed", [1])
def test_random_graphs_motifs(name, make, seed):
    g = make(seed)
    h = dm.load_graph(g)
    kmax = {"er": 4, "sbm": 5}.get(name, 5 if name in ("ba", "cl") else 6)
    for k in range(3, kmax + 1):
        assert np.array_equal(dm.count_motifs(h, k), O.motif_count(g, k, threads=8)), (name, seed, k)


# ------------------------------------------------------------------ per-root records

def test_clique_record_mode():
    import torch
    g = gg.chung_lu(2000, 12000, 2.2, 300.0, 5)[0]
    h = dm.load_graph(g)
    for k in (3, 4, 5):
        stats = torch.zeros((g.n, 3), dtype=torch.int64, device="cuda")
        tot = dm.count_cliques(h, k, root_stats=stats)
        st = stats.cpu().numpy().astype(np.uint64)
        t2, leaves, nodes, reads = O.clique_count(g, k, per_root=True, threads=8)
        assert tot == t2
        assert np.array_equal(st[:, 1], leaves)
        assert np.array_equal(st[:, 0], nodes)
        assert np.array_equal(st[:, 2], reads)


def test_motif_record_mode():
    """Per-root leaves, tree nodes and adjacency entries read (the degree of
    the last vertex of each expanded set's canonical order) equal the
    oracle's, on a preferential-attachment graph and on a Chung-Lu graph."""
    import torch
    for g in (gg.barabasi_albert(800, 3, 4), gg.chung_lu(3000, 12000, 2.2, 80.0, 6)[0]):
        h = dm.load_graph(g)
        for k in (3, 4, 5, 6):
            if k == 6 and g.n == 800:
                continue
            stats = torch.zeros((g.n, 3), dtype=torch.int64, device="cuda")
            c = dm.count_motifs(h, k, root_stats=stats)
            st = stats.cpu().numpy().astype(np.uint64)
            c2, leaves, nodes, reads = O.motif_count(g, k, per_root=True, threads=8)
            assert np.array_equal(c, c2), k
            assert np.array_equal(st[:, 1], leaves), k
            assert np.array_equal(st[:, 0], nodes), k
            assert np.array_equal(st[:, 2], reads), k


# ------------------------------------------------------------------ schedule invariance

SCHED = [
    dict(),
    dict(chunk=1),
    dict(chunk=37),
    dict(chunk=512),
    dict(sched=dm.DM_NO_DONATION),
    dict(waves_per_cu=1),
    dict(waves_per_cu=2, chunk=3),
    dict(rebalance=0.5),
    dict(rebalance=0.01, chunk=2),
]


def test_queue_heads_small_and_ragged_queues():
    """The root queue is dealt in blocks of `chunk` entries to 8 heads: queues
    shorter than the head count, block counts that do not divide evenly, a
    last block shorter than `chunk`, and one block larger than the queue all
    run every root exactly once (root subsets against the oracle's per-root
    sums, and full launches)."""
    g = gg.chung_lu(3000, 30000, 2.1, 400.0, 9)[0]  # 80% of roots have a triangle
    h = dm.load_graph(g)
    k = 3
    tot, leaves, _, _ = O.clique_count(g, k, per_root=True, threads=8)
    rng = np.random.default_rng(5)
    for nroots in (1, 3, 8, 9, 17, 1001):
        roots = np.sort(rng.choice(g.n, nroots, replace=False)).astype(np.int32)
        want = int(leaves[roots].astype(np.uint64).sum())
        for chunk in (1, 2, 3, 7, 64, 4096):
            assert dm.count_cliques(h, k, roots=roots, chunk=chunk) == want, (nroots, chunk)
    for chunk in (1, 5, 375, 376, 377, 4096):
        assert dm.count_cliques(h, k, chunk=chunk) == tot, chunk


def test_schedule_invariance_cliques():
    g = gg.chung_lu(20000, 200000, 2.1, 1500.0, 3)[0]
    h = dm.load_graph(g)
    for k in (4, 6):
        ref = O.clique_count(g, k, threads=8)
        for s in SCHED:
            assert dm.count_cliques(h, k, **s) == ref, (k, s)
        for _ in range(5):
            assert dm.count_cliques(h, k) == ref


def test_schedule_invariance_motifs():
    for k, g in ((4, gg.chung_lu(5000, 20000, 2.2, 300.0, 9)[0]), (5, gg.chung_lu(2000, 6000, 2.2, 60.0, 9)[0])):
        h = dm.load_graph(g)
        ref = O.motif_count(g, k, threads=8)
        for s in SCHED:
            assert np.array_equal(dm.count_motifs(h, k, **s), ref), (k, s)


def test_range_donation_runs_every_root_once():
    """Chunks far larger than n / waves: a few waves take the whole queue and
    hand untried entry ranges to idle waves.  Counts and per-root records equal
    the oracle's, so every root ran exactly once."""
    import torch
    g = gg.chung_lu(6000, 36000, 2.2, 300.0, 13)[0]
    h = dm.load_graph(g)
    for k in (3, 5):
        tot, leaves, nodes, reads = O.clique_count(g, k, per_root=True, threads=8)
        for chunk in (1500, 6000):
            ws = torch.zeros(256 * 32 * 4, dtype=torch.int64, device="cuda")
            stats = torch.zeros((g.n, 3), dtype=torch.int64, device="cuda")
            assert dm.count_cliques(h, k, chunk=chunk, root_stats=stats, wave_stats=ws) == tot, (k, chunk)
            st = stats.cpu().numpy().astype(np.uint64)
            assert np.array_equal(st[:, 0], nodes) and np.array_equal(st[:, 1], leaves) and np.array_equal(st[:, 2], reads)
            w = ws.view(-1, 4).cpu().numpy()
            assert (w[:, 3] > 0).sum() > 4, "no entry range was handed over"
    ref, ml, mn, _ = O.motif_count(g, 4, per_root=True, threads=8)
    for chunk in (1500, 6000):
        stats = torch.zeros((g.n, 3), dtype=torch.int64, device="cuda")
        assert np.array_equal(dm.count_motifs(h, 4, chunk=chunk, root_stats=stats), ref), chunk
        st = stats.cpu().numpy().astype(np.uint64)
        assert np.array_equal(st[:, 0], mn) and np.array_equal(st[:, 1], ml)


def test_row_cache_any_call_order():
    """The per-graph row cache is filled by the first counting launch over all
    roots and read by later ones: a first call at large k (whose pruned roots
    still fill their rows), root subsets before and after the cache exists, and
    recording calls all give the oracle's counts."""
    import torch
    g = gg.chung_lu(4000, 24000, 2.2, 250.0, 17)[0]
    ref = {k: O.clique_count(g, k, threads=8) for k in (3, 4, 5, 6, 7)}
    sub = np.random.default_rng(3).permutation(g.n)[:1000].astype(np.int32)
    h = dm.load_graph(g)
    part = dm.count_cliques(h, 4, roots=sub)          # no cache yet: subsets do not fill it
    assert part == O.clique_count(g, 4, roots=sub, threads=8)
    assert dm.count_cliques(h, 7) == ref[7]           # fills the cache
    for k in (3, 4, 5, 6):
        assert dm.count_cliques(h, k) == ref[k], k    # reads it
    assert dm.count_cliques(h, 4, roots=sub) == part
    stats = torch.zeros((g.n, 3), dtype=torch.int64, device="cuda")
    tot, leaves, nodes, reads = O.clique_count(g, 5, per_root=True, threads=8)
    assert dm.count_cliques(h, 5, root_stats=stats) == tot
    st = stats.cpu().numpy().astype(np.uint64)
    assert np.array_equal(st[:, 0], nodes) and np.array_equal(st[:, 2], reads)


def test_root_lists_partition_the_count():
    g = gg.chung_lu(4000, 16000, 2.2, 80.0, 11)[0]
    h = dm.load_graph(g)
    rng = np.random.default_rng(0)
    perm = rng.permutation(g.n).astype(np.int32)
    a, b = perm[:1500], perm[1500:]
    for k in (3, 5):
        tot = dm.count_cliques(h, k)
        ca, cb = dm.count_cliques(h, k, roots=a), dm.count_cliques(h, k, roots=b)
        assert ca + cb == tot
        assert ca == O.clique_count(g, k, roots=a, threads=8)
        ma, mb = dm.count_motifs(h, k, roots=a), dm.count_motifs(h, k, roots=b)
        assert np.array_equal(ma + mb, dm.count_motifs(h, k))
        assert np.array_equal(mb, O.motif_count(g, k, roots=b, threads=8))
        assert dm.count_cliques(h, k, roots=perm) == tot


# ------------------------------------------------------------------ batching

def test_batch_matches_single_calls():
    graphs = [gg.batch_graph(i, nhi=300) for i in range(24)]
    hs = [dm.load_graph(g) for g in graphs]
    for k in (3, 4, 5):
        got = dm.batch(hs, dm.DM_OP_MOTIF, k)
        for i, g in enumerate(graphs):
            assert np.array_equal(got[i], O.motif_count(g, k)), (k, i)
    got = dm.batch(hs, dm.DM_OP_CLIQUE, 4)[:, 0]
    assert list(got) == [O.clique_count(g, 4) for g in graphs]
    # the cached union is reused on a second call
    assert np.array_equal(dm.batch(hs, dm.DM_OP_MOTIF, 4), dm.batch(hs, dm.DM_OP_MOTIF, 4))


# ------------------------------------------------------------------ errors

def test_error_paths():
    import torch
    g = gg.erdos_renyi(100, 400, 1)
    h = dm.load_graph(g)
    for bad_k in (0, 33):
        with pytest.raises(dm.DMError) as e:
            dm.count_cliques(h, bad_k)
        assert e.value.status == dm.DM_E_K
    for bad_k in (2, 9):
        with pytest.raises(dm.DMError) as e:
            dm.count_motifs(h, bad_k)
        assert e.value.status == dm.DM_E_K
    with pytest.raises(dm.DMError) as e:
        dm.count_cliques(h, 3, sched=dm.DM_SCHED_LEARNED)
    assert e.value.status == dm.DM_E_MODEL
    # device-side validation
    rp = torch.tensor([0, 1, 1], dtype=torch.int64, device="cuda")
    col = torch.tensor([1], dtype=torch.int32, device="cuda")
    with pytest.raises(dm.DMError) as e:
        dm.load_csr(2, rp, col, device=True)
    assert e.value.status == dm.DM_E_CSR
    rpd = torch.from_numpy(g.row_ptr).cuda()
    cold = torch.from_numpy(g.col).cuda()
    hd = dm.load_csr(g.n, rpd, cold, device=True)
    assert dm.count_cliques(hd, 3) == O.clique_count(g, 3)


def test_overflow_detected():
    g = gg.complete(30)
    h = dm.load_graph(g)
    c = math.comb(30, 4)
    assert dm.count_cliques(h, 4, counter_bias=2**64 - c - 1) == 2**64 - 1
    with pytest.raises(dm.DMError) as e:
        dm.count_cliques(h, 4, counter_bias=2**64 - c)
    assert e.value.status == dm.DM_E_OVERFLOW
    m = O.motif_count(g, 4).max()
    with pytest.raises(dm.DMError) as e:
        dm.count_motifs(h, 4, counter_bias=2**64 - int(m))
    assert e.value.status == dm.DM_E_OVERFLOW


def test_wait_limit_gives_up_with_an_error():
    """The idle wait of the persistent grid is bounded.  With a host-set limit
    of 1 microsecond, waves left without work while K_40's 12-clique roots
    still run stop waiting; every wave exits, the call fails with DM_E_HIP,
    and the next call with the default limit is exact."""
    h = dm.load_graph(gg.complete(40))
    with pytest.raises(dm.DMError) as e:
        dm.count_cliques(h, 12, wait_limit_us=1)
    assert e.value.status == dm.DM_E_HIP
    assert "wait limit" in str(e.value)
    assert dm.count_cliques(h, 12) == math.comb(40, 12)
    hs = dm.load_graph(gg.star(600))
    with pytest.raises(dm.DMError) as e:
        dm.count_motifs(hs, 5, wait_limit_us=1)
    assert e.value.status == dm.DM_E_HIP
    exp = np.zeros(21, np.uint64)
    exp[int(np.nonzero(O.motif_brute(gg.star(4), 5))[0][0])] = math.comb(600, 4)
    assert np.array_equal(dm.count_motifs(hs, 5), exp)


# ------------------------------------------------------------------ graph replay and autotuning

def test_batch_graph_replays_match_eager():
    """The batch launch is captured once and replayed; eager single-graph calls
    run between replays, and every replay equals the eager per-graph counts."""
    graphs = [gg.batch_graph(i, nhi=400) for i in range(40)]
    hs = [dm.load_graph(g) for g in graphs]
    eager5 = np.stack([dm.count_motifs(h, 5) for h in hs])
    eager4c = np.array([dm.count_cliques(h, 4) for h in hs], np.uint64)
    for rep in range(4):
        assert np.array_equal(dm.batch(hs, dm.DM_OP_MOTIF, 5), eager5), rep
        assert np.array_equal(dm.batch(hs, dm.DM_OP_CLIQUE, 4)[:, 0], eager4c), rep
        # eager work between replays
        assert dm.count_cliques(hs[rep], 3) == O.clique_count(graphs[rep], 3)
    assert np.array_equal(eager5[7], O.motif_count(graphs[7], 5))


def test_autotune_picks_valid_knobs_and_keeps_counts():
    graphs = [gg.batch_graph(i, nhi=300) for i in range(16)]
    hs = [dm.load_graph(g) for g in graphs]
    ref = dm.batch(hs, dm.DM_OP_MOTIF, 4)
    t = dm.autotune(hs, dm.DM_OP_MOTIF, 4)
    assert t["chunk"] in (1, 2, 4, 8, 16, 32, 64, 128)
    assert 0.0 <= t["rebalance"] <= 0.4 + 1e-6 and t["waves_per_cu"] in (0, 1, 2, 4, 8) and t["ms"] > 0
    assert np.array_equal(dm.batch(hs, dm.DM_OP_MOTIF, 4, sched=dm.DM_SCHED_AUTOTUNE), ref)
    g = gg.chung_lu(3000, 15000, 2.2, 200.0, 4)[0]
    h = dm.load_graph(g)
    t1 = dm.autotune([h], dm.DM_OP_CLIQUE, 5)
    assert t1["ms"] > 0
    assert dm.count_cliques(h, 5, sched=dm.DM_SCHED_AUTOTUNE) == O.clique_count(g, 5, threads=8)


# ------------------------------------------------------------------ one lane per traversal (ablation)

@pytest.mark.parametrize("name,make", RANDOM, ids=[r[0] for r in RANDOM])
def test_dfs_ablation_matches_oracle(name, make):
    """DM_IMPL_DFS (each lane enumerates one root's tree alone) gives the
    oracle's clique and motif counts."""
    g = make(1)
    h = dm.load_graph(g)
    for k in range(3, 8):
        assert dm.count_cliques(h, k, sched=dm.DM_IMPL_DFS) == O.clique_count(g, k, threads=8), (name, k)
    kmax = {"er": 4, "sbm": 5}.get(name, 5)
    for k in range(3, kmax + 1):
        assert np.array_equal(dm.count_motifs(h, k, sched=dm.DM_IMPL_DFS), O.motif_count(g, k, threads=8)), (name, k)


def test_dfs_ablation_closed_forms_and_options():
    h = dm.load_graph(gg.complete(24))
    for k in (1, 2, 3, 9, 12, 16):
        assert dm.count_cliques(h, k, sched=dm.DM_IMPL_DFS) == math.comb(24, k), k
    parts = [3] * 300  # out-degrees up to 897
    assert dm.count_cliques(dm.load_graph(gg.complete_multipartite(parts)), 4, sched=dm.DM_IMPL_DFS) == _esym(parts, 4)
    hs = dm.load_graph(gg.star(300))
    exp = np.zeros(6, np.uint64)
    exp[int(np.nonzero(O.motif_brute(gg.star(3), 4))[0][0])] = math.comb(300, 3)
    assert np.array_equal(dm.count_motifs(hs, 4, sched=dm.DM_IMPL_DFS | dm.DM_NO_DONATION), exp)
    with pytest.raises(dm.DMError) as e:
        dm.count_cliques(h, 17, sched=dm.DM_IMPL_DFS)
    assert e.value.status == dm.DM_E_K
    for kw in (dict(roots=np.arange(5)), dict(chunk=0, sched=dm.DM_IMPL_DFS | dm.DM_SCHED_AUTOTUNE)):
        with pytest.raises(dm.DMError) as e:
            dm.count_cliques(h, 4, **dict(dict(sched=dm.DM_IMPL_DFS), **kw))
        assert e.value.status == dm.DM_E_ARG


# ------------------------------------------------------------------ host-driven balancing (Section IV-D)

def _k300_plus_background():
    bg = gg.erdos_renyi(6000, 30000, 9)
    g, _ = gg.disjoint_union([bg, gg.complete(300)])
    return g, bg


def test_host_balanced_relaunch_is_exact():
    """DM_SCHED_HOST_BALANCE: the launch stops once the queue is drained and
    most waves are idle, busy waves spill their untried extensions, the host
    splits them and relaunches.  K_300 sits last in the rank order (degree
    299), so its heavy roots are still running when the stop comes: the call
    relaunches, and the counts stay exact (closed form for K_300 plus the
    oracle on the background), with per-root records equal to the plain
    launch's."""
    import torch
    g, bg = _k300_plus_background()
    h = dm.load_graph(g)
    for k in (4, 5):
        exp = math.comb(300, k) + O.clique_count(bg, k, threads=8)
        assert dm.count_cliques(h, k) == exp
        assert dm.count_cliques(h, k, sched=dm.DM_SCHED_HOST_BALANCE) == exp, k
        assert dm.last_launch_count() > 1, k
        assert dm.count_cliques(h, k, sched=dm.DM_SCHED_HOST_BALANCE, rebalance=0.9) == exp, k
    s1 = torch.zeros((g.n, 3), dtype=torch.int64, device="cuda")
    s2 = torch.zeros((g.n, 3), dtype=torch.int64, device="cuda")
    assert dm.count_cliques(h, 5, root_stats=s1) == dm.count_cliques(h, 5, root_stats=s2,
                                                                      sched=dm.DM_SCHED_HOST_BALANCE)
    assert torch.equal(s1, s2)
    for k in (4, 5):
        ck = O.motif_count(bg, k, threads=8)
        kcls = int(np.nonzero(O.motif_brute(gg.complete(k), k))[0][0])
        ck[kcls] += math.comb(300, k)
        assert np.array_equal(dm.count_motifs(h, k, sched=dm.DM_SCHED_HOST_BALANCE), ck), k
        # the motif default stops only below 10% busy waves (more than the
        # 300 K_300 roots' waves); at 50% the K_300 roots are still running
        # when the background's waves have finished
        assert np.array_equal(dm.count_motifs(h, k, sched=dm.DM_SCHED_HOST_BALANCE, rebalance=0.5), ck), k
        assert dm.last_launch_count() > 1, k
    for bad in (dict(sched=dm.DM_SCHED_HOST_BALANCE | dm.DM_NO_DONATION),):
        with pytest.raises(dm.DMError) as e:
            dm.count_cliques(h, 4, **bad)
        assert e.value.status == dm.DM_E_ARG
    with pytest.raises(dm.DMError) as e:
        dm.batch([h, h], dm.DM_OP_CLIQUE, 3, sched=dm.DM_SCHED_HOST_BALANCE)
    assert e.value.status == dm.DM_E_ARG
