"""Sorted starts (paper Section 5): with BPT_FLAG_SORTED_STARTS the fused
batches take samples in order of their start vertex, or of its rank in a
vertex order such as reverse Cuthill-McKee; the sets (and their order) stay
the oracle's, and the edge-access counters equal the oracle's accounting for
the same batch composition."""

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee

import graphgen
import oracle
import paper_2311_10201_amd as bpt
from gpu_util import announce, assert_same_sets, sample_device

pytestmark = pytest.mark.gpu


def rcm_rank(n, src, dst):
    a = sp.csr_matrix((np.ones(len(src)), (src, dst)), shape=(n, n))
    perm = reverse_cuthill_mckee((a + a.T).tocsr(), symmetric_mode=True)
    rank = np.empty(n, dtype=np.uint32)
    rank[perm] = np.arange(n, dtype=np.uint32)
    return rank


@pytest.mark.parametrize("case", ["er", "rmat-wc", "lfr-dense"])
def test_sorted_starts_match_oracle(case):
    if case == "er":
        n = 1000
        src, dst = graphgen.er_graph(n, 10_000, seed=42)
        prob = graphgen.uniform_prob(len(src), 0.1)
    elif case == "rmat-wc":
        n = 1 << 14
        src, dst = graphgen.rmat_graph(14, 16, 0.57, 0.19, 0.19, seed=14)
        prob = graphgen.wc_prob(n, dst)
    else:
        n = 10_000
        src, dst = graphgen.lfr_graph(n, 11, 2)
        prob = graphgen.uniform_prob(len(src), 0.2)
    S, seed, first = 3000, 17, 250
    og = oracle.Graph(n, src, dst, prob)
    ref = og.sample(seed, S, first_sample=first, nthreads=8)
    g = bpt.bpt_create_graph(n, src, dst, prob)
    rank = rcm_rank(n, src, dst)
    for label, rk in (("start ids", None), ("RCM ranks", rank)):
        bpt.bpt_graph_set_vertex_order(g, rk)
        order = oracle.sorted_start_order(ref, rk)
        for c in (16, 64, 256):
            announce(f"sorted starts {case} by {label} C={c}")
            off, ver, cnt = sample_device(g, first, S, c, seed, flags=bpt.BPT_FLAG_SORTED_STARTS)
            assert_same_sets(off, ver, ref, f"sorted {label} C={c}")
            assert cnt.edge_accesses == oracle.fused_edge_accesses(og, ref, c, order)
            assert cnt.frontier_entries == oracle.fused_frontier_entries(ref, c, order)
            assert cnt.sample_edges == int(ref.te.sum())


def test_sorted_starts_invalid():
    n = 1000
    src, dst = graphgen.er_graph(n, 10_000, seed=42)
    g = bpt.bpt_create_graph(n, src, dst, graphgen.uniform_prob(len(src), 0.1))
    with pytest.raises(bpt.BptError):
        bpt.bpt_graph_set_vertex_order(g, np.zeros(n, dtype=np.uint32))   # not a permutation
    with pytest.raises(bpt.BptError):
        sample_device(g, 0, 100, 64, 1, flags=bpt.BPT_FLAG_SORTED_STARTS | bpt.BPT_FLAG_UNFUSED)
