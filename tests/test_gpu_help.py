"""GPU parity with tail helping forced on and off (BPT_HELP=1 / 0).  When a
launch runs out of batches, workgroups without one join the heavy levels of
batches still running: the owner publishes a chunk's staging and helpers
claim units of its work items.  The sets must equal the oracle's either way;
the graphs are chosen so that levels are heavy (thousands of frontier
entries) and batches are fewer than the resident workgroups."""

import numpy as np
import pytest

import graphgen
import oracle
import paper_2311_10201_amd as bpt
from gpu_util import announce, assert_same_sets, sample_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def heavy():
    n = 1 << 14
    src, dst = graphgen.rmat_graph(14, 32, 0.57, 0.19, 0.19, seed=14)
    prob = graphgen.uniform_prob(len(src), 0.1)
    return bpt.bpt_create_graph(n, src, dst, prob), oracle.Graph(n, src, dst, prob)


@pytest.mark.parametrize("force", ["1", "0"])
@pytest.mark.parametrize("colors", [64, 32])
def test_helping_matches_oracle(heavy, monkeypatch, force, colors):
    g, og = heavy
    S, first, seed = 4096, 11, 77
    monkeypatch.setenv("BPT_HELP", force)
    announce(f"helping forced {force}: R-MAT 14 p=0.1, {S} samples, colours {colors}")
    ref = og.sample(seed, S, first_sample=first, nthreads=8)
    assert ref.offsets[-1] / S > 1000  # heavy sets: the regime helping is for
    off, ver, cnt = sample_device(g, first, S, colors, seed, capacity=int(ref.offsets[-1]))
    assert_same_sets(off, ver, ref, f"BPT_HELP={force} colours {colors}")
    assert cnt.sample_edges == int(ref.te.sum())
    assert cnt.edge_accesses == oracle.fused_edge_accesses(og, ref, colors)
