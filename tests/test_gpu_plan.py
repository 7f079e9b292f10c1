"""GPU parity of sampling plans (bpt_plan_create / bpt_plan_enqueue): the fused
path as kernels only, run eagerly and captured into a hipGraph (through
torch.cuda.CUDAGraph) and replayed with sample ranges and seeds written into
device memory between replays.  Every call's sets equal the oracle's."""

import numpy as np
import pytest

import graphgen
import oracle
import paper_2311_10201_amd as bpt
from gpu_util import announce, assert_same_sets

pytestmark = pytest.mark.gpu


def _graphs():
    out = []
    src, dst = graphgen.er_graph(1000, 10_000, seed=42)
    out.append((1000, src, dst, graphgen.uniform_prob(len(src), 0.1)))
    src, dst = graphgen.rmat_graph(12, 8, 0.57, 0.19, 0.19, seed=12)
    out.append((1 << 12, src, dst, graphgen.wc_prob(1 << 12, dst)))
    src, dst = graphgen.rmat_graph(10, 16, 0.57, 0.19, 0.19, seed=10)
    rng = np.random.Generator(np.random.PCG64(10))
    out.append((1 << 10, src, dst, (rng.random(len(src), dtype=np.float32) * np.float32(0.2)).astype(np.float32)))
    return out


@pytest.fixture(scope="module")
def graphs():
    return [(bpt.bpt_create_graph(n, s, d, p), oracle.Graph(n, s, d, p)) for n, s, d, p in _graphs()]


def _buffers(S, cap):
    import torch
    return (torch.empty(S + 1, dtype=torch.int64, device="cuda"),
            torch.empty(max(cap, 1), dtype=torch.int32, device="cuda"),
            torch.full((2,), 99, dtype=torch.int64, device="cuda"))


def _check(off, vert, res, ref, what):
    status, members = (int(x) for x in res.cpu().tolist())
    assert status == bpt.BPT_OK, (what, status)
    assert members == int(ref.offsets[-1]), what
    assert_same_sets(off.cpu().numpy().view(np.uint64), vert[:members].cpu().numpy().view(np.uint32), ref, what)


@pytest.mark.parametrize("gi,colors", [(0, 64), (1, 16), (2, 256), (1, 0)])
def test_plan_eager_matches_oracle(graphs, gi, colors):
    import torch
    g, og = graphs[gi]
    S, first, seed = 1500, 77, 5 + gi
    announce(f"plan eager: graph {gi}, colours {colors}, {S} samples from {first}")
    ref = og.sample(seed, S, first_sample=first, nthreads=8)
    need = int(ref.offsets[-1])
    # pool: the library's estimate (32 members per set before any history) where it
    # suffices, else sized from the oracle (graph 2's sets average ~150 members)
    plan = bpt.bpt_plan_create(g, 2000, colors, need if gi == 2 else 0)
    off, vert, res = _buffers(S, need)
    for rep in range(2):  # the workspace comes back clean
        bpt.bpt_plan_enqueue(plan, first, S, seed, None, torch.cuda.current_stream(), off, vert, need, res)
        torch.cuda.synchronize()
        _check(off, vert, res, ref, f"graph {gi} colours {colors} call {rep}")
    plan.close()


def test_plan_graph_replays_follow_device_params(graphs):
    """Capture once with the range and seed in device memory, replay with
    new values written there, with eager library and torch work between."""
    import torch
    g, og = graphs[1]
    S = 1200
    plan = bpt.bpt_plan_create(g, S, 64, 0)
    cases = [(0, 3), (4096, 11), ((1 << 33) + 5, (1 << 40) + 9), (100, 3)]
    refs = [og.sample(seed, S, first_sample=first, nthreads=8) for first, seed in cases]
    cap = max(int(r.offsets[-1]) for r in refs)
    off, vert, res = _buffers(S, cap)
    params = torch.zeros(2, dtype=torch.int64, device="cuda")
    stream = torch.cuda.Stream()
    announce("plan graph: eager warm-up on the capture stream")
    params.copy_(torch.tensor([cases[0][0], cases[0][1]], dtype=torch.int64))
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        bpt.bpt_plan_enqueue(plan, 0, S, 0, params, stream, off, vert, cap, res)
    torch.cuda.synchronize()
    _check(off, vert, res, refs[0], "eager with device params")
    announce("plan graph: capture")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream, capture_error_mode="thread_local"):
        bpt.bpt_plan_enqueue(plan, 0, S, 0, params, stream, off, vert, cap, res)
    torch.cuda.synchronize()
    for i, ((first, seed), ref) in enumerate(zip(cases, refs)):
        announce(f"plan graph: replay {i} first {first} seed {seed}")
        params.copy_(torch.tensor([first, seed], dtype=torch.int64))
        res.fill_(99)
        graph.replay()
        torch.cuda.synchronize()
        _check(off, vert, res, ref, f"replay {i}")
        # eager work between replays: another library call and a torch reduction
        o2 = torch.empty(65, dtype=torch.int64, device="cuda")
        v2 = torch.empty(64 * 64, dtype=torch.int32, device="cuda")
        st, _, _ = bpt.bpt_sample_rrr_device(g, i, 64, 64, 1, 0, None, o2, v2, 64 * 64)
        assert st in (bpt.BPT_OK, bpt.BPT_ERANGE)
        assert int(vert[:8].to(torch.int64).sum().item()) >= 0
        torch.cuda.synchronize()
    del graph
    plan.close()


def test_plan_reports_small_buffers(graphs):
    import torch
    g, og = graphs[0]
    S, seed = 900, 21
    ref = og.sample(seed, S, nthreads=8)
    need = int(ref.offsets[-1])
    announce("plan: capacity one short, then a pool too small")
    plan = bpt.bpt_plan_create(g, S, 64, 0)
    off, vert, res = _buffers(S, need)
    bpt.bpt_plan_enqueue(plan, 0, S, seed, None, None, off, vert, need - 1, res)
    torch.cuda.synchronize()
    assert res.cpu().tolist() == [bpt.BPT_ERANGE, need]
    assert np.array_equal(off.cpu().numpy().view(np.uint64), ref.offsets)
    plan.close()
    part = og.sample(seed, 3, nthreads=1)
    room = int(part.offsets[-1])  # a pool that holds the first three sets only
    assert room < need
    small = bpt.bpt_plan_create(g, S, 64, room)
    bpt.bpt_plan_enqueue(small, 0, S, seed, None, None, off, vert, need, res)
    torch.cuda.synchronize()
    status, pool_need = res.cpu().tolist()
    assert status == bpt.BPT_ERANGE and pool_need == need
    # the workspace is clean afterwards: a call that fits in the pool is exact
    off2, vert2, res2 = _buffers(3, room)
    bpt.bpt_plan_enqueue(small, 0, 3, seed, None, None, off2, vert2, room, res2)
    torch.cuda.synchronize()
    _check(off2, vert2, res2, part, "small plan after an overflow")
    small.close()


def test_plan_edges(graphs):
    import torch
    g, og = graphs[0]
    plan = bpt.bpt_plan_create(g, 100, 64, 0)
    announce("plan: zero samples, a device range past 2^34, too many samples")
    off, vert, res = _buffers(0, 1)
    bpt.bpt_plan_enqueue(plan, 5, 0, 1, None, None, off, vert, 0, res)
    torch.cuda.synchronize()
    assert res.cpu().tolist() == [bpt.BPT_OK, 0] and int(off[0].item()) == 0
    params = torch.tensor([(1 << 34) - 10, 3], dtype=torch.int64, device="cuda")
    off, vert, res = _buffers(100, 100 * 64)
    bpt.bpt_plan_enqueue(plan, 0, 100, 0, params, None, off, vert, 100 * 64, res)
    torch.cuda.synchronize()
    assert int(res[0].item()) == bpt.BPT_EINVAL
    with pytest.raises(bpt.BptError) as ei:
        bpt.bpt_plan_enqueue(plan, 0, 101, 0, None, None, off, vert, 100 * 64, res)
    assert ei.value.status == bpt.BPT_EINVAL
    with pytest.raises(bpt.BptError):
        bpt.bpt_plan_enqueue(plan, (1 << 34) - 10, 100, 0, None, None, off, vert, 100 * 64, res)
    plan.close()
