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
    assert cnt.philox_blocks == oracle.philox_blocks(og, ref)  # helpers' blocks included


def test_helping_in_a_multi_job_launch(heavy, monkeypatch):
    """Helpers join batches of any job of the launch (the job table tells them
    which graph and sample range a batch belongs to)."""
    import torch
    g, og = heavy
    src, dst = graphgen.er_graph(1000, 10_000, seed=42)
    prob = graphgen.uniform_prob(len(src), 0.1)
    g2, og2 = bpt.bpt_create_graph(1000, src, dst, prob), oracle.Graph(1000, src, dst, prob)
    monkeypatch.setenv("BPT_HELP", "1")
    specs = [(g, og, 5, 3000, 21), (g2, og2, 0, 2000, 8), (g, og, 90_000, 1500, 4)]
    announce("helping forced 1: three jobs on two graphs in one launch")
    jobs, refs = [], []
    for gg, oo, first, S, seed in specs:
        ref = oo.sample(seed, S, first_sample=first, nthreads=8)
        cap = int(ref.offsets[-1])
        jobs.append(bpt.Job(gg, first, S, seed, torch.empty(S + 1, dtype=torch.int64, device="cuda"),
                            torch.empty(max(cap, 1), dtype=torch.int32, device="cuda"), cap, 64))
        refs.append(ref)
    st, cnt = bpt.bpt_sample_rrr_jobs(jobs)
    torch.cuda.synchronize()
    assert st == bpt.BPT_OK
    for j, ref, spec in zip(jobs, refs, specs):
        assert j.status == bpt.BPT_OK and j.total == int(ref.offsets[-1])
        assert_same_sets(j.d_offsets.cpu().numpy().view(np.uint64),
                         j.d_vertices[:j.total].cpu().numpy().view(np.uint32), ref, f"job {spec[2:]}")


def test_helping_in_a_plan_and_its_graph(heavy, monkeypatch):
    """A plan enqueued with helping on, eagerly and replayed from a captured graph."""
    import torch
    g, og = heavy
    monkeypatch.setenv("BPT_HELP", "1")
    S, seed = 2048, 13
    ref = og.sample(seed, S, nthreads=8)
    need = int(ref.offsets[-1])
    plan = bpt.bpt_plan_create(g, S, 64, need)
    off = torch.empty(S + 1, dtype=torch.int64, device="cuda")
    vert = torch.empty(need, dtype=torch.int32, device="cuda")
    res = torch.zeros(2, dtype=torch.int64, device="cuda")
    stream = torch.cuda.Stream()
    announce("helping forced 1: plan, eager then graph replays")
    with torch.cuda.stream(stream):
        bpt.bpt_plan_enqueue(plan, 0, S, seed, None, stream, off, vert, need, res)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream, capture_error_mode="thread_local"):
        bpt.bpt_plan_enqueue(plan, 0, S, seed, None, stream, off, vert, need, res)
    torch.cuda.synchronize()
    for rep in range(3):
        res.fill_(99)
        vert.fill_(-1)
        graph.replay()
        torch.cuda.synchronize()
        assert res.cpu().tolist() == [bpt.BPT_OK, need], rep
        assert_same_sets(off.cpu().numpy().view(np.uint64), vert.cpu().numpy().view(np.uint32), ref, f"replay {rep}")
    del graph
    plan.close()
