"""GPU parity of multi-job plans (bpt_jobs_plan_create / bpt_jobs_plan_enqueue):
many jobs on graphs of different sizes, probability layouts and colour
counts, sampled by a fixed sequence of kernels, eagerly and from one captured
hipGraph replayed with new sample ranges and seeds written to device memory
between replays.  Every job's sets equal the oracle's for that job alone."""

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
    src, dst = graphgen.rmat_graph(14, 8, 0.57, 0.19, 0.19, seed=14)
    out.append((1 << 14, src, dst, graphgen.uniform_prob(len(src), 0.03)))
    src, dst = graphgen.rmat_graph(10, 16, 0.57, 0.19, 0.19, seed=10)
    rng = np.random.Generator(np.random.PCG64(10))
    out.append((1 << 10, src, dst, (rng.random(len(src), dtype=np.float32) * np.float32(0.2)).astype(np.float32)))
    return out


@pytest.fixture(scope="module")
def graphs():
    return [(n, bpt.bpt_create_graph(n, s, d, p), oracle.Graph(n, s, d, p)) for n, s, d, p in _graphs()]


def _jobs(graphs, specs, refs_cap):
    import torch
    jobs = []
    for (gi, first, S, seed, colors), cap in zip(specs, refs_cap):
        jobs.append(bpt.Job(graphs[gi][1], first, S, seed, torch.empty(S + 1, dtype=torch.int64, device="cuda"),
                            torch.empty(max(cap, 1), dtype=torch.int32, device="cuda"), cap, colors))
    return jobs


def _check(jobs, res, refs, what):
    r = res.cpu().numpy().reshape(-1, 2)
    for i, (j, ref) in enumerate(zip(jobs, refs)):
        assert int(r[i, 0]) == bpt.BPT_OK, (what, i, int(r[i, 0]))
        assert int(r[i, 1]) == int(ref.offsets[-1]), (what, i)
        total = int(r[i, 1])
        assert_same_sets(j.d_offsets.cpu().numpy().view(np.uint64),
                         j.d_vertices[:total].cpu().numpy().view(np.uint32), ref, f"{what} job {i}")


def test_jobs_plan_eager(graphs):
    import torch
    # mask widths 1 (8..64 colours), 2, 4 and 16 words; an empty job; a range past 2^32
    specs = [(0, 0, 700, 3, 64), (1, 1000, 2000, 9, 16), (2, 5, 1500, 23, 256), (3, 0, 500, 7, 8),
             (0, 0, 0, 1, 64), (1, (1 << 32) - 100, 300, (1 << 40) + 7, 1024), (2, 0, 900, 4, 128)]
    refs = [graphs[gi][2].sample(seed, S, first_sample=first, nthreads=8) for gi, first, S, seed, _ in specs]
    caps = [int(r.offsets[-1]) for r in refs]
    jobs = _jobs(graphs, specs, caps)
    announce(f"jobs plan eager: {len(jobs)} jobs")
    plan = bpt.bpt_jobs_plan_create(jobs, 2 * sum(caps))
    res = torch.full((2 * len(jobs),), 99, dtype=torch.int64, device="cuda")
    for rep in range(2):  # the workspaces come back clean
        bpt.bpt_jobs_plan_enqueue(plan, None, torch.cuda.current_stream(), res)
        torch.cuda.synchronize()
        _check(jobs, res, refs, f"eager call {rep}")
    plan.close()


def test_jobs_plan_graph_replays(graphs):
    """One captured graph samples every job; new ranges and seeds are written
    to device memory before each replay, with eager work in between."""
    import torch
    base = [(0, 0, 1200, 0, 0), (1, 0, 3000, 0, 32), (2, 0, 2500, 0, 64), (3, 0, 800, 0, 16), (1, 0, 1000, 0, 0)]
    rounds = [[(0, 3), (7, 11), (1 << 33, 5), (64, 2), (9, 9)],
              [(500, 4), (0, 1), (3, 3), (1 << 20, (1 << 40) + 1), (77, 12)],
              [(0, 3), (7, 11), (1 << 33, 5), (64, 2), (9, 9)]]
    refs = [[graphs[gi][2].sample(seed, S, first_sample=first, nthreads=8)
             for (gi, _, S, _, _), (first, seed) in zip(base, rnd)] for rnd in rounds]
    caps = [max(int(refs[r][i].offsets[-1]) for r in range(len(rounds))) for i in range(len(base))]
    jobs = _jobs(graphs, base, caps)
    # a pool large enough for every round (the default estimate comes from earlier calls)
    plan = bpt.bpt_jobs_plan_create(jobs, 2 * sum(caps))
    params = torch.zeros(2 * len(jobs), dtype=torch.int64, device="cuda")
    res = torch.full((2 * len(jobs),), 99, dtype=torch.int64, device="cuda")
    stream = torch.cuda.Stream()

    def write(rnd):
        params.copy_(torch.tensor([x for fs in rnd for x in fs], dtype=torch.int64))

    announce("jobs plan graph: eager on the capture stream")
    write(rounds[0])
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        bpt.bpt_jobs_plan_enqueue(plan, params, stream, res)
    torch.cuda.synchronize()
    _check(jobs, res, refs[0], "eager with device params")
    announce("jobs plan graph: capture")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream, capture_error_mode="thread_local"):
        bpt.bpt_jobs_plan_enqueue(plan, params, stream, res)
    torch.cuda.synchronize()
    for r, rnd in enumerate(rounds):
        announce(f"jobs plan graph: replay {r}")
        write(rnd)
        res.fill_(99)
        graph.replay()
        torch.cuda.synchronize()
        _check(jobs, res, refs[r], f"replay {r}")
        g = graphs[0][1]
        o2 = torch.empty(65, dtype=torch.int64, device="cuda")
        v2 = torch.empty(64 * 64, dtype=torch.int32, device="cuda")
        st, _, _ = bpt.bpt_sample_rrr_device(g, r, 64, 64, 1, 0, None, o2, v2, 64 * 64)
        assert st in (bpt.BPT_OK, bpt.BPT_ERANGE)
        torch.cuda.synchronize()
    del graph
    plan.close()


def test_jobs_plan_reports(graphs):
    """A job whose buffer is too small reports BPT_ERANGE with its total; a
    range from device memory past 2^34 reports BPT_EINVAL."""
    import torch
    specs = [(0, 0, 600, 3, 64), (1, 0, 900, 4, 64)]
    refs = [graphs[gi][2].sample(seed, S, first_sample=first, nthreads=8) for gi, first, S, seed, _ in specs]
    caps = [int(refs[0].offsets[-1]), int(refs[1].offsets[-1]) - 1]
    jobs = _jobs(graphs, specs, caps)
    plan = bpt.bpt_jobs_plan_create(jobs, 0)
    res = torch.full((4,), 99, dtype=torch.int64, device="cuda")
    bpt.bpt_jobs_plan_enqueue(plan, None, None, res)
    torch.cuda.synchronize()
    r = res.cpu().tolist()
    assert r[0] == bpt.BPT_OK and r[1] == caps[0]
    assert r[2] == bpt.BPT_ERANGE and r[3] == caps[1] + 1
    params = torch.tensor([0, 3, (1 << 34) - 10, 4], dtype=torch.int64, device="cuda")
    bpt.bpt_jobs_plan_enqueue(plan, params, None, res)
    torch.cuda.synchronize()
    assert res.cpu().tolist()[0] == bpt.BPT_EINVAL and res.cpu().tolist()[2] == bpt.BPT_EINVAL
    plan.close()
    with pytest.raises(bpt.BptError):
        bpt.bpt_jobs_plan_create([], 0)
