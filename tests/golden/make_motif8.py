"""Write the expected 8-motif counts of the k = 8 GPU tests (oracle only).

Building the oracle's 8-vertex class table takes about a minute on one core,
so the GPU tests read these counts instead of calling the oracle.  This script
runs only the oracle and the seeded input generators and writes
motif8_expected.txt:

  canon <code of class 0> <code of class 1> ...      (11,117 canonical codes)
  pattern <name> <class id>                           (path, star, cycle, K_8)
  graph <name> <n> <nnz> <fnv1a64> <cls>:<count> ...  (non-zero classes only)

Run: python tests/golden/make_motif8.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402
from paper_2212_04551_amd import graphgen as gg  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
K = 8

# seeded inputs of the k = 8 tests: name -> generator call
GRAPHS = {
    "er60": lambda: gg.erdos_renyi(60, 130, 1),
    "ba50": lambda: gg.barabasi_albert(50, 2, 2),
    "cl400": lambda: gg.chung_lu(400, 700, 2.3, 15.0, 3)[0],
    "sbm": lambda: gg.sbm(6, 10, 0.4, 0.05, 4),
}


def sampled_eight_vertex_graphs():
    """300 of the 2^28 labelled graphs on 8 vertices (a fixed stride) plus K_8."""
    pairs = [(i, j) for i in range(K) for j in range(i + 1, K)]
    masks = list(range(0, 1 << 28, (1 << 28) // 300)) + [(1 << 28) - 1]
    return masks, [gg.from_edges(K, [p for b, p in enumerate(pairs) if m >> b & 1]) for m in masks]


def main():
    lines = ["canon " + " ".join(str(int(c)) for c in O.class_canon(K))]
    for name, pat in (("path", gg.path(K)), ("star", gg.star(K - 1)), ("cycle", gg.cycle(K)),
                      ("complete", gg.complete(K))):
        lines.append(f"pattern {name} {int(np.nonzero(O.motif_brute(pat, K))[0][0])}")
    for name, make in GRAPHS.items():
        g = make()
        c = O.motif_count(g, K, threads=8)
        nz = " ".join(f"{i}:{int(c[i])}" for i in np.nonzero(c)[0])
        lines.append(f"graph {name} {g.n} {g.nnz} {gg.fnv1a64(g)} {nz}")
        print(name, int(c.sum()), flush=True)
    masks, graphs = sampled_eight_vertex_graphs()
    for m, g in zip(masks, graphs):
        c = O.motif_brute(g, K)
        nz = " ".join(f"{i}:{int(c[i])}" for i in np.nonzero(c)[0])
        lines.append(f"graph mask{m} {g.n} {g.nnz} {gg.fnv1a64(g)} {nz}")
    with open(os.path.join(HERE, "motif8_expected.txt"), "w") as f:
        f.write("# written by make_motif8.py; oracle only\n" + "\n".join(lines) + "\n")
    print("wrote motif8_expected.txt", len(lines), "lines")


if __name__ == "__main__":
    main()
