"""dm_count_motifs_static (the motif count that allocates no device memory:
its buffers live in one static device array per GPU) against dm_count_motifs,
exactly, through the C ABI: two calls in a row with the second on a smaller
input, a change of k in between (the array keeps the last call's dictionary),
records and knobs, and the size and option limits."""
import numpy as np
import pytest

from paper_2212_04551_amd import dm
from paper_2212_04551_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def test_static_matches_allocating_entry_point():
    import torch
    big = gg.chung_lu(20000, 80000, 2.3, 300.0, 3)[0]
    small = gg.erdos_renyi(300, 900, 4)
    hb = dm.load_graph(big, rank=True)
    hs = dm.load_graph(small, rank=True)
    for k in (5, 4):
        ref_b = dm.count_motifs(dm.load_graph(big), k)
        ref_s = dm.count_motifs(dm.load_graph(small), k)
        got_b = dm.count_motifs_static(hb, k)
        got_s = dm.count_motifs_static(hs, k)  # second call, smaller input
        assert np.array_equal(got_b, ref_b), k
        assert np.array_equal(got_s, ref_s), k
        assert ref_b.sum() > 0 and ref_s.sum() > 0
    # k = 7 (the largest dictionary) and back to k = 3
    assert np.array_equal(dm.count_motifs_static(hs, 7), dm.count_motifs(dm.load_graph(small), 7))
    assert np.array_equal(dm.count_motifs_static(hs, 3), dm.count_motifs(dm.load_graph(small), 3))
    # per-root records and scheduling knobs
    st1 = torch.zeros((small.n, 3), dtype=torch.int64, device="cuda")
    st2 = torch.zeros((small.n, 3), dtype=torch.int64, device="cuda")
    a = dm.count_motifs(dm.load_graph(small), 5, root_stats=st1)
    b = dm.count_motifs_static(hs, 5, root_stats=st2, chunk=3, rebalance=0.01)
    assert np.array_equal(a, b)
    assert torch.equal(st1, st2)
    assert np.array_equal(dm.count_motifs_static(hb, 5, sched=dm.DM_NO_DONATION, waves_per_cu=1),
                          dm.count_motifs(hb, 5))


def test_static_limits():
    small = gg.erdos_renyi(300, 900, 4)
    h = dm.load_graph(small)  # not loaded with DM_CSR_RANK, never counted
    with pytest.raises(dm.DMError) as e:
        dm.count_motifs_static(h, 4)
    assert e.value.status == dm.DM_E_ARG
    dm.count_motifs(h, 4)  # builds the rank-renamed copy
    dm.count_motifs_static(h, 4)
    with pytest.raises(dm.DMError) as e:
        dm.count_motifs_static(h, 4, roots=np.arange(5, dtype=np.int32))
    assert e.value.status == dm.DM_E_ARG
    with pytest.raises(dm.DMError) as e:
        dm.count_motifs_static(h, 8)
    assert e.value.status == dm.DM_E_K
    # a star with 2.5 million leaves: one wave's k=6 stack (10 x 2.5e6 entries
    # of 5 bytes) exceeds the 64 MiB array, so the call is refused
    hub = dm.load_graph(gg.star(2_500_000), rank=True)
    with pytest.raises(dm.DMError) as e:
        dm.count_motifs_static(hub, 6)
    assert e.value.status == dm.DM_E_NOMEM
    # after the refusal the array still serves a normal call
    assert np.array_equal(dm.count_motifs_static(h, 4), dm.count_motifs(h, 4))
