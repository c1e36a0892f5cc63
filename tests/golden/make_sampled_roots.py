"""Write the per-root expected records of the benchmark graphs (oracle only).

The full counts of the 10^6-vertex clique workload (k >= 6) and of the
10^5-vertex motif workloads are out of the oracle's reach, so their GPU totals
are checked root by root: every count is a sum over roots (each subgraph is
credited to its lowest (degree, id) vertex), and the oracle computes a root's
records exactly when it can finish that root.  This script runs only the
oracle (and the seeded input generators) and writes:

  cl1m_heavy_roots.txt  Chung-Lu n=1e6 m=2e7 gamma=2.1 wmax=1e4 seed 0,
                        cliques k=3..8: the heaviest roots the oracle finishes
                        within ROOT_BUDGET seconds each.  Candidates: the 64
                        roots of largest out-degree in the (degree, id) DAG and
                        192 seeded roots of out-degree >= 128; a candidate goes
                        on to k+1 only if it finished k; per k the HEAVY roots
                        with the most tree nodes are kept.
  cl100k_roots.txt      Chung-Lu n=1e5 m=1e6 gamma=2.3 seed 0, motifs k=5
                        (weight cap 1414) and k=6 (weight cap 120): a seeded
                        uniform sample of SAMPLE roots, each given ROOT_BUDGET
                        seconds; the roots that finish, their records and the
                        class counts summed over them.
  hub_roots_k6.txt      hub_graph(roots=4, base=3000, hub_degree=340, seed 2),
                        motifs k=6 over its 4 roots (leaf-level lists of about
                        860 entries).

Line formats (all integers):
  graph <name> <n> <nnz> <fnv1a64>
  root <k> <vertex> <leaves> <nodes> <reads>
  classes <k> <count of class 0> <count of class 1> ...   (motif files)

Run: python tests/golden/make_sampled_roots.py [cl1m|cl100k|hub ...]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402
from paper_2212_04551_amd import graphgen as gg  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
THREADS = int(os.environ.get("ORACLE_THREADS", "8"))
ROOT_BUDGET = 15.0
HEAVY = 48
SAMPLE = 384


def dag_outdegree(g):
    deg = g.degrees()
    rank = np.empty(g.n, np.int64)
    rank[np.lexsort((np.arange(g.n), deg))] = np.arange(g.n)
    src = np.repeat(np.arange(g.n), deg)
    return np.bincount(src[rank[g.col] > rank[src]], minlength=g.n)


def log(*a):
    print(*a, flush=True)


def cl1m():
    g = gg.chung_lu(1_000_000, 20_000_000, 2.1, 1.0e4, 0)[0]
    od = dag_outdegree(g)
    top = np.argsort(-od, kind="stable")[:64]
    wide = np.setdiff1d(np.nonzero(od >= 128)[0], top)
    cand = np.unique(np.concatenate([top, np.random.default_rng(2024).choice(wide, 192, replace=False)]))
    cand = cand.astype(np.int32)
    lines = [f"graph cl1m {g.n} {g.nnz} {gg.fnv1a64(g)}"]
    for k in range(3, 9):
        t = time.time()
        done, leaves, nodes, reads = O.clique_budgeted(g, k, cand, THREADS, ROOT_BUDGET)
        keep = np.nonzero(done)[0]
        heavy = keep[np.argsort(-nodes[keep].astype(np.float64), kind="stable")[:HEAVY]]
        for i in sorted(heavy, key=lambda i: cand[i]):
            lines.append(f"root {k} {cand[i]} {leaves[i]} {nodes[i]} {reads[i]}")
        log(f"cl1m k={k}: {len(cand)} candidates, {len(keep)} finished, kept {len(heavy)} "
            f"(nodes {int(nodes[heavy].min()) if len(heavy) else 0}..{int(nodes[heavy].max()) if len(heavy) else 0}) "
            f"in {time.time() - t:.0f}s")
        cand = cand[keep]
    return lines


def cl100k():
    lines = []
    for k, cap in ((5, 1414.0), (6, 120.0)):
        g = gg.chung_lu(100_000, 1_000_000, 2.3, cap, 0)[0]
        lines.append(f"graph cl100k_cap{int(cap)} {g.n} {g.nnz} {gg.fnv1a64(g)}")
        roots = np.sort(np.random.default_rng(77).choice(g.n, SAMPLE, replace=False)).astype(np.int32)
        t = time.time()
        done, per, leaves, nodes, reads = O.motif_budgeted(g, k, roots, THREADS, ROOT_BUDGET)
        keep = np.nonzero(done)[0]
        for i in keep:
            lines.append(f"root {k} {roots[i]} {leaves[i]} {nodes[i]} {reads[i]}")
        cls = per[keep].sum(axis=0)
        lines.append(f"classes {k} " + " ".join(str(int(c)) for c in cls))
        log(f"cl100k k={k} cap {cap}: {len(keep)} of {len(roots)} roots finished, "
            f"{int(leaves[keep].sum())} subgraphs, in {time.time() - t:.0f}s")
    return lines


def hub():
    g = gg.hub_graph(4, 3000, 340, 2)
    k = 6
    roots = np.arange(4, dtype=np.int32)
    t = time.time()
    done, per, leaves, nodes, reads = O.motif_budgeted(g, k, roots, THREADS, 3600.0)
    assert done.all()
    lines = [f"graph hub4_3000_340_s2 {g.n} {g.nnz} {gg.fnv1a64(g)}"]
    for i in range(len(roots)):
        lines.append(f"root {k} {roots[i]} {leaves[i]} {nodes[i]} {reads[i]}")
    lines.append(f"classes {k} " + " ".join(str(int(c)) for c in per.sum(axis=0)))
    log(f"hub k=6: {int(leaves.sum())} subgraphs in {time.time() - t:.0f}s")
    return lines


JOBS = {"cl1m": ("cl1m_heavy_roots.txt", cl1m), "cl100k": ("cl100k_roots.txt", cl100k),
        "hub": ("hub_roots_k6.txt", hub)}

if __name__ == "__main__":
    for name in sys.argv[1:] or list(JOBS):
        fname, fn = JOBS[name]
        body = fn()
        with open(os.path.join(HERE, fname), "w") as f:
            f.write(f"# written by make_sampled_roots.py ({name}); oracle only; root budget {ROOT_BUDGET}s\n")
            f.write("\n".join(body) + "\n")
        log(f"wrote {fname}: {len(body)} lines")
