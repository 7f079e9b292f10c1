"""Writes the stored expected values under tests/golden/ (calls only the CPU oracle).

er1000_m10000_p0.1_seed42.txt: the Erdos-Renyi workload (n = 1,000,
m = 10,000 edges, graph seed 42, uniform p = 0.1 in fp32), 64 RRR sets for
sample ids 0..63 with Philox seed 42.  Each line: sample id, then the set's
members in ascending order.  The header records the input digest, so a change
in the generator is noticed separately from a change in the oracle.

Run:  python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen  # noqa: E402
import oracle  # noqa: E402


def er_case():
    n, m = 1000, 10_000
    src, dst = graphgen.er_graph(n, m, seed=42)
    prob = graphgen.uniform_prob(m, 0.1)
    return n, src, dst, prob


def main():
    n, src, dst, prob = er_case()
    g = oracle.Graph(n, src, dst, prob)
    res = g.sample(42, 64)
    path = os.path.join(HERE, "er1000_m10000_p0.1_seed42.txt")
    with open(path, "w") as f:
        f.write(f"# graph sha256 {graphgen.edges_sha256(n, src, dst, prob)}\n")
        f.write("# n 1000 m 10000 p 0.1 samples 0..63 seed 42\n")
        for i in range(len(res)):
            f.write(" ".join([str(i)] + [str(v) for v in res.set_of(i).tolist()]) + "\n")
    print("wrote", path, "members", int(res.offsets[-1]))


if __name__ == "__main__":
    main()
