"""GPU parity at the workloads' full sizes.

* R-MAT scale 20, edge factor 16, weighted cascade, 100,000 samples (the
  benchmark's workload and launch configuration): every set of fused C=64,
  fused C=256 and unfused equals the oracle's, and the edge-access counters
  equal the oracle's level-synchronous accounting.
* R-MAT scale 22, edge factor 16, uniform p = 0.01, 1,000,000 samples (the
  largest single-GPU workload): the oracle computes the sets of every sample
  id that is a multiple of 97 (10,310 sets; all 1,000,000 would be ~2e12
  sample-edges), and the unfused traversal's sets are compared with them
  element by element.  Then the fused traversal at every colour count 64 ..
  1024 returns all 1,000,000 sets identical to the unfused ones (9.9e9 ids
  compared on the device) and the oracle's on the subset; its work counters
  equal the unfused ones where the method fixes them (members, sample-edges,
  Philox blocks) and obey Theorem 1 (edge accesses <= sample-edges).
"""

import os

import numpy as np
import pytest

import graphgen
import oracle
import paper_2311_10201_amd as bpt
from gpu_util import announce, assert_same_sets, sample_device

pytestmark = pytest.mark.gpu

# the GPU machine's CPU share is 16 cores per GPU
THREADS = min(16, len(os.sched_getaffinity(0)))


@pytest.fixture(scope="module")
def rmat20():
    src, dst = graphgen.rmat_graph(20, 16, 0.57, 0.19, 0.19, seed=20)
    n = 1 << 20
    prob = graphgen.wc_prob(n, dst)
    return n, src, dst, prob


@pytest.mark.timeout(300)
def test_rmat20_wc_full(rmat20):
    n, src, dst, prob = rmat20
    S, seed = 100_000, 42
    announce("R-MAT 20 WC: oracle")
    og = oracle.Graph(n, src, dst, prob)
    ref = og.sample(seed, S, nthreads=THREADS)
    g = bpt.bpt_create_graph(n, src, dst, prob)
    assert bpt.bpt_graph_info(g)[2] == bpt.BPT_PROB_ROW
    te = int(ref.te.sum())
    blocks = oracle.philox_blocks(og, ref)
    for c in (64, 256):
        announce(f"R-MAT 20 WC S={S} C={c}")
        off, ver, cnt = sample_device(g, 0, S, c, seed)
        assert_same_sets(off, ver, ref, f"C={c}")
        assert cnt.sample_edges == te
        assert cnt.edge_accesses == oracle.fused_edge_accesses(og, ref, c)
        assert cnt.philox_blocks == blocks
    announce(f"R-MAT 20 WC S={S} unfused")
    off, ver, cnt = sample_device(g, 0, S, 0, seed, flags=bpt.BPT_FLAG_UNFUSED)
    assert_same_sets(off, ver, ref, "unfused")
    assert cnt.edge_accesses == te
    assert cnt.philox_blocks == blocks


def _subset_on_device(off, vert, ids):
    """The sets of sample ids `ids` from a device CSR, as (sizes, members) numpy arrays."""
    import torch
    idx = torch.as_tensor(ids.astype(np.int64), device=off.device)
    lo, hi = off[idx], off[idx + 1]
    lens = hi - lo
    before = torch.cumsum(lens, 0) - lens
    pos = torch.repeat_interleave(lo - before, lens) + torch.arange(int(lens.sum().item()), device=off.device)
    return lens.cpu().numpy().astype(np.uint64), vert[pos].cpu().numpy().view(np.uint32)


@pytest.fixture(scope="module")
def rmat22():
    """R-MAT 22 p = 0.01: the graph on the device, the oracle's sets of ids
    = 0 mod 97, and the unfused traversal's 1,000,000 sets kept on the device
    as the reference of the fused runs."""
    import torch
    announce("R-MAT 22 p=0.01: generating")
    src, dst = graphgen.rmat_graph(22, 16, 0.57, 0.19, 0.19, seed=22)
    n = 1 << 22
    prob = graphgen.uniform_prob(len(src), 0.01)
    S, seed = 1_000_000, 42
    ids = np.arange(0, S, 97, dtype=np.uint64)
    announce(f"R-MAT 22 oracle on {len(ids)} ids (multiples of 97), {THREADS} threads")
    og = oracle.Graph(n, src, dst, prob)
    ref = og.sample_ids(seed, ids, nthreads=THREADS)
    g = bpt.bpt_create_graph(n, src, dst, prob)
    assert bpt.bpt_graph_info(g)[2] == bpt.BPT_PROB_UNIFORM
    announce(f"R-MAT 22 S={S} unfused, all sets")
    off = torch.empty(S + 1, dtype=torch.int64, device="cuda")
    probe = torch.empty(1, dtype=torch.int32, device="cuda")
    st, total, _ = bpt.bpt_sample_rrr_device(g, 0, S, 0, seed, bpt.BPT_FLAG_UNFUSED, None, off, probe, 1)
    assert st == bpt.BPT_ERANGE and total > S
    vert = torch.empty(total, dtype=torch.int32, device="cuda")
    st, total2, cnt = bpt.bpt_sample_rrr_device(g, 0, S, 0, seed, bpt.BPT_FLAG_UNFUSED, None, off, vert, total)
    assert st == bpt.BPT_OK and total2 == total
    torch.cuda.synchronize()
    bpt.bpt_graph_release_cache(g)
    yield dict(n=n, S=S, seed=seed, ids=ids, ref=ref, og=og, g=g, off=off, vert=vert, total=total, unfused=cnt)
    bpt.bpt_free(g)
    del off, vert
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
def test_rmat22_unfused_matches_oracle_subset(rmat22):
    r = rmat22
    ref, ids = r["ref"], r["ids"]
    sizes, members = _subset_on_device(r["off"], r["vert"], ids)
    assert np.array_equal(sizes, np.diff(ref.offsets)), "set sizes differ from the oracle"
    assert np.array_equal(members, ref.members), "members differ from the oracle"
    off_h = r["off"].cpu().numpy().view(np.uint64)
    assert int(off_h[-1]) == r["total"] == r["unfused"].members
    assert np.all(np.diff(off_h) >= 1)  # every set holds its start
    assert r["unfused"].sample_edges >= int(ref.te.sum())


@pytest.mark.timeout(600)
@pytest.mark.parametrize("colors", [64, 128, 256, 512, 1024])
def test_rmat22_fused_all_sets(rmat22, colors):
    import torch
    r = rmat22
    S, total = r["S"], r["total"]
    announce(f"R-MAT 22 S={S} fused C={colors}")
    off = torch.empty(S + 1, dtype=torch.int64, device="cuda")
    vert = torch.empty(total, dtype=torch.int32, device="cuda")
    st, total_f, cnt = bpt.bpt_sample_rrr_device(r["g"], 0, S, colors, r["seed"], 0, None, off, vert, total)
    assert st == bpt.BPT_OK and total_f == total
    bpt.bpt_graph_release_cache(r["g"])
    assert torch.equal(off, r["off"]), f"C={colors}: offsets differ from the unfused traversal"
    step = 1 << 30
    for a in range(0, total, step):
        e = min(a + step, total)
        assert torch.equal(vert[a:e], r["vert"][a:e]), f"C={colors}: ids {a}..{e} differ from the unfused traversal"
    sizes, members = _subset_on_device(off, vert, r["ids"])
    assert np.array_equal(sizes, np.diff(r["ref"].offsets)) and np.array_equal(members, r["ref"].members)
    u = r["unfused"]
    assert cnt.members == u.members and cnt.sample_edges == u.sample_edges
    assert cnt.philox_blocks == u.philox_blocks
    assert cnt.edge_accesses <= cnt.sample_edges
    assert cnt.batches == (S + colors - 1) // colors
    announce(f"R-MAT 22 C={colors}: traversal {cnt.traversal_ns / 1e9:.2f} s, TE/EA "
             f"{cnt.sample_edges / cnt.edge_accesses:.2f}, workgroups {cnt.workgroups}")
    del off, vert
