"""The oracle reproduces its stored expected sets for the Erdos-Renyi workload
(n = 1,000, m = 10,000, p = 0.1, 64 samples, seed 42), written by
tests/golden/make_golden.py.  A change here means the oracle's arithmetic or
the input generator changed and must be justified against the paper."""
import os

import numpy as np

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "er1000_m10000_p0.1_seed42.txt")


def load_golden():
    sha, sets = None, []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("# graph sha256"):
                sha = line.split()[-1]
            elif not line.startswith("#"):
                parts = [int(x) for x in line.split()]
                assert parts[0] == len(sets)
                sets.append(parts[1:])
    return sha, sets


def test_er_golden():
    n, m = 1000, 10_000
    src, dst = graphgen.er_graph(n, m, seed=42)
    prob = graphgen.uniform_prob(m, 0.1)
    sha, sets = load_golden()
    assert graphgen.edges_sha256(n, src, dst, prob) == sha
    assert len(set(zip(src.tolist(), dst.tolist()))) == m and not np.any(src == dst)
    res = oracle.Graph(n, src, dst, prob).sample(42, 64)
    assert len(sets) == 64
    for i in range(64):
        assert res.set_of(i).tolist() == sets[i]
        assert oracle.start_vertex(42, i, n) in sets[i]
