"""Input generators: reproducible fingerprints and CSR well-formedness."""
import os

import numpy as np
import pytest

from paper_2212_04551_amd import graphgen as gg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _check_csr(g, m=None):
    rp, col = g.row_ptr, g.col
    assert rp.dtype == np.int64 and col.dtype == np.int32
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == col.size
    src = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(col >= 0) and np.all(col < g.n)
    assert np.all(src != col)
    # strictly ascending inside each row
    same_row = src[1:] == src[:-1]
    assert np.all(col[1:][same_row] > col[:-1][same_row])
    # symmetric
    fwd = set(zip(src.tolist(), col.tolist()))
    assert all((b, a) in fwd for a, b in fwd)
    if m is not None:
        assert col.size == 2 * m


def test_fingerprints_reproduce():
    import sys
    sys.path.insert(0, GOLDEN)
    from make_generator_hashes import CASES
    with open(os.path.join(GOLDEN, "generator_hashes.txt")) as f:
        for line in f:
            if line.startswith("#"):
                continue
            name, n, nnz, h = line.split()
            g = CASES[name]()
            assert (g.n, g.nnz, gg.fnv1a64(g)) == (int(n), int(nnz), int(h)), name


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_well_formed(seed):
    _check_csr(gg.erdos_renyi(300, 1000, seed), 1000)
    _check_csr(gg.chung_lu(3000, 12000, 2.2, 300.0, seed)[0], 12000)
    _check_csr(gg.barabasi_albert(400, 3, seed), 3 * 4 // 2 + (400 - 4) * 3)
    _check_csr(gg.sbm(10, 20, 0.5, 0.01, seed))
    _check_csr(gg.batch_graph(seed))


def test_chung_lu_mean_weight_and_cap():
    g, i0 = gg.chung_lu(20000, 100000, 2.3, 400.0, 0)
    d = g.degrees()
    assert i0 > 0 and d.mean() == pytest.approx(10.0)
    assert d.max() <= 500


def test_sbm_block_density():
    g = gg.sbm(20, 50, 0.4, 0.001, 3)
    # ids are shuffled, so only global density is checked: E[m] = 20*C(50,2)*0.4 + C(20,2)*2500*0.001
    exp = 20 * 1225 * 0.4 + 190 * 2500 * 0.001
    assert abs(g.m - exp) < 5 * np.sqrt(exp)


def test_batch_params_ranges():
    for i in range(200):
        kind, n, x = gg.batch_params(i)
        assert 20 <= n <= 2000
        if kind == "er":
            assert 2 * n <= x <= 8 * n + 1
        else:
            assert 2 <= x <= 6


def test_structured_families():
    assert gg.complete(6).m == 15
    assert gg.hypercube(3).m == 12
    assert gg.cocktail_party(4).m == 24
    assert gg.complete_multipartite([2, 3, 4]).m == 2 * 3 + 2 * 4 + 3 * 4
    u, offs = gg.disjoint_union([gg.path(4), gg.cycle(5)])
    assert u.n == 9 and u.m == 3 + 5 and list(offs) == [0, 4, 9]
    _check_csr(u)
