"""Write tests/golden/generator_hashes.txt: FNV-1a-64 fingerprints of seeded graphs.

These pin the input generators (not any count): a change to a generator or its
random stream changes the fingerprint.  Run: python tests/golden/make_generator_hashes.py
"""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from paper_2212_04551_amd import graphgen as gg  # noqa: E402

CASES = {
    "er516_s0": lambda: gg.workload_graph("er516", 0),
    "er516_s1": lambda: gg.workload_graph("er516", 1),
    "cl100k_s0": lambda: gg.workload_graph("cl100k", 0),
    "sbm200x60_s0": lambda: gg.workload_graph("sbm200x60", 0),
    "batch_0": lambda: gg.batch_graph(0),
    "batch_1": lambda: gg.batch_graph(1),
    "batch_4095": lambda: gg.batch_graph(4095),
}

if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "generator_hashes.txt")
    with open(out, "w") as f:
        f.write("# name n nnz fnv1a64  (written by make_generator_hashes.py)\n")
        for name, fn in CASES.items():
            g = fn()
            f.write(f"{name} {g.n} {g.nnz} {gg.fnv1a64(g)}\n")
    print(open(out).read())
