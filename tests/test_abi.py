"""C-ABI library: loads, exports every declared symbol, host-only entry points
agree with the oracle, and argument / CSR errors are reported before any GPU
work (so these run without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2212_04551_amd import dm
from paper_2212_04551_amd import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "dm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dm_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = dm.lib()
    names = _declared_symbols()
    assert "dm_load_csr" in names and "dm_batch" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(dm.EXPORTS)


def test_options_struct_layout(tmp_path):
    """The ctypes mirror of dm_options has the C struct's size and field
    offsets, as the host C compiler lays them out from include/dm.h."""
    fields = [f[0] for f in dm.dm_options._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "dm.h"\nint main(void){\n'
                   '  printf("%zu\\n", sizeof(dm_options));\n'
                   + "".join(f'  printf("%zu\\n", offsetof(dm_options, {f}));\n' for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    vals = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert vals[0] == ctypes.sizeof(dm.dm_options)
    for f, off in zip(fields, vals[1:]):
        assert getattr(dm.dm_options, f).offset == off, f


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_class_ids_and_masks_match_oracle(k):
    assert dm.motif_num_classes(k) == O.num_classes(k)
    canon = O.class_canon(k)
    for c in range(len(canon)):
        assert dm.motif_class_mask(k, c) == int(canon[c])


@pytest.mark.parametrize("k,reachable", [(3, 3), (4, 21), (5, 315), (6, 9765)])
def test_dictionary_matches_oracle_on_every_code(k, reachable):
    """Section IV-C dictionary: traversal code t is the full bitmap (t<<1)|1."""
    T = dm.motif_class_table(k)
    assert T.size == 1 << (k * (k - 1) // 2 - 1)
    hit = 0
    for t in range(T.size):
        fields_ok = all((t >> (i * (i - 1) // 2 - 1)) & ((1 << i) - 1) for i in range(2, k))
        if fields_ok:
            hit += 1
            assert T[t] == O.class_of_code(k, (t << 1) | 1), t
        else:
            assert T[t] == 0xFF
    assert hit == reachable


@pytest.mark.parametrize("k", [3, 4, 5, 6, 7])
def test_16bit_dictionary_matches_oracle_on_every_code(k):
    """The 16-bit dictionary the kernels read (k = 7: 2^20 codes, 853
    classes) against the oracle's class of every full bitmap (t<<1)|1;
    for k <= 6 it equals the 8-bit table (0xFF -> 0xFFFF)."""
    T = dm.motif_class_table16(k)
    assert T.dtype == np.uint16 and T.size == 1 << (k * (k - 1) // 2 - 1)
    assert dm.motif_num_classes(k) == O.num_classes(k)
    canon = O.class_canon(k)
    for c in range(0, len(canon), max(1, len(canon) // 64)):
        assert dm.motif_class_mask(k, c) == int(canon[c])
    t = np.arange(T.size, dtype=np.int64)
    reach = np.ones(T.size, dtype=bool)
    for i in range(2, k):
        reach &= ((t >> (i * (i - 1) // 2 - 1)) & ((1 << i) - 1)) != 0
    assert (T[~reach] == 0xFFFF).all()
    exp = O.class_of_codes(k, (t[reach] << 1) | 1)
    assert np.array_equal(T[reach].astype(np.int64), exp)
    if k <= 6:
        T8 = dm.motif_class_table(k)
        assert np.array_equal(np.where(T8 == 0xFF, 0xFFFF, T8.astype(np.uint16)), T)


def test_16bit_dictionary_k8_against_oracle():
    """k = 8 (2^27 codes, 11,117 classes): every class's canonical code, and
    the class of 2^20 seeded random reachable traversal codes, against the
    oracle's orbit labelling (an independent implementation)."""
    k = 8
    assert dm.motif_num_classes(k) == O.num_classes(k) == 11117
    canon = O.class_canon(k)
    for c in range(len(canon)):
        assert dm.motif_class_mask(k, c) == int(canon[c])
    T = dm.motif_class_table16(k)
    assert T.size == 1 << 27
    rng = np.random.default_rng(8)
    t = rng.integers(0, 1 << 27, size=1 << 20, dtype=np.int64)
    reach = np.ones(t.size, dtype=bool)
    for i in range(2, k):
        reach &= ((t >> (i * (i - 1) // 2 - 1)) & ((1 << i) - 1)) != 0
    assert (T[t[~reach]] == 0xFFFF).all()
    assert np.array_equal(T[t[reach]].astype(np.int64), O.class_of_codes(k, (t[reach] << 1) | 1))


def test_unsupported_k():
    assert dm.motif_num_classes(2) == -1 and dm.motif_num_classes(9) == -1
    assert dm.motif_num_classes(7) == 853
    with pytest.raises(dm.DMError) as e:
        dm.motif_class_table(7)
    assert e.value.status == dm.DM_E_K
    with pytest.raises(dm.DMError) as e:
        dm.motif_class_table16(9)
    assert e.value.status == dm.DM_E_K
    with pytest.raises(dm.DMError) as e:
        dm.motif_class_mask(4, 6)
    assert e.value.status == dm.DM_E_ARG


def _bad_csrs():
    ok = gg.cycle(5)
    yield "self-loop", ok.n, ok.row_ptr, np.array([0, 1, 4, 0, 2, 1, 3, 2, 4, 0, 3], np.int32)[: ok.nnz]
    rp = ok.row_ptr.copy()
    col = ok.col.copy()
    col[0], col[1] = col[1], col[0]
    yield "unsorted", ok.n, rp, col
    col = ok.col.copy()
    col[0] = 9
    yield "out of range", ok.n, rp, col
    g = gg.from_edges(3, [(0, 1)])
    yield "asymmetric", 3, np.array([0, 1, 1, 1], np.int64), np.array([1], np.int32)
    yield "repeat", 2, np.array([0, 2, 4], np.int64), np.array([1, 1, 0, 0], np.int32)
    yield "bad offsets", 2, np.array([1, 1, 2], np.int64), np.array([1, 0], np.int32)


@pytest.mark.parametrize("case", list(_bad_csrs()), ids=lambda c: c[0])
def test_host_csr_validation_rejects(case):
    _, n, rp, col = case
    with pytest.raises(dm.DMError) as e:
        dm.load_csr(n, rp, col)
    assert e.value.status == dm.DM_E_CSR


def test_argument_errors_without_gpu():
    L = dm.lib()
    out = ctypes.c_uint64(0)
    assert L.dm_count_cliques(None, 3, ctypes.byref(out), None) == dm.DM_E_ARG
    assert L.dm_count_motifs(None, 4, None, 0, None) == dm.DM_E_ARG
    assert L.dm_batch(None, 0, 0, 3, None, 0, None) == dm.DM_E_ARG
    h = ctypes.c_void_p(None)
    assert L.dm_load_csr(-1, None, None, 0, None, ctypes.byref(h)) == dm.DM_E_ARG
    assert L.dm_load_csr(3, None, None, 0, None, None) == dm.DM_E_ARG
    assert L.dm_strerror(dm.DM_E_OVERFLOW) == b"uint64 count overflow"


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with status 2 and a
    message, before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_directed_dictionary_matches_oracle_on_every_code(k):
    """The directed dictionary the kernel reads: the class of every one of the
    2^(k(k-1)) codes equals the oracle's (brute force over all k! orders), and
    each class's smallest code is the oracle's."""
    T = dm.motif_directed_class_table(k)
    assert T.dtype == np.uint16 and T.size == 1 << (k * (k - 1))
    assert dm.motif_directed_num_classes(k) == O.dnum_classes(k)
    exp = O.dclass_table(k)
    assert np.array_equal(np.where(T == 0xFFFF, -1, T.astype(np.int64)), exp.astype(np.int64))
    canon = O.dclass_canon(k)
    for c in range(0, len(canon), max(1, len(canon) // 97)):
        assert dm.motif_directed_class_code(k, c) == int(canon[c])


def test_directed_host_errors():
    assert dm.motif_directed_num_classes(6) == -1 and dm.motif_directed_num_classes(0) == -1
    with pytest.raises(dm.DMError) as e:
        dm.motif_directed_class_code(3, 13)
    assert e.value.status == dm.DM_E_ARG
    with pytest.raises(dm.DMError) as e:
        dm.motif_directed_class_table(6)
    assert e.value.status == dm.DM_E_K
    # arc conventions are checked on the host before any GPU work
    for rp, col in (([0, 1, 1, 1], [0]), ([0, 2, 2, 2], [2, 1]), ([0, 1, 1, 1], [7]), ([1, 1, 1, 1], [])):
        with pytest.raises(dm.DMError) as e:
            dm.load_digraph_csr(3, np.array(rp, np.int64), np.array(col, np.int32))
        assert e.value.status == dm.DM_E_CSR
