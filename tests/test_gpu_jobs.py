"""GPU parity of the multi-job launch (bpt_sample_rrr_jobs): jobs on graphs of
different sizes, probability layouts, colour counts and sample ranges share
one persistent fused launch, and every job's sets equal the oracle's for that
job alone."""

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
    return [(n, s, d, p, bpt.bpt_create_graph(n, s, d, p), oracle.Graph(n, s, d, p)) for n, s, d, p in _graphs()]


def _run(graphs, specs, cap_scale=None):
    import torch
    jobs, refs = [], []
    for gi, first, S, seed, colors in specs:
        n = graphs[gi][0]
        ref = graphs[gi][5].sample(seed, S, first_sample=first, nthreads=8)
        refs.append(ref)
        need = int(ref.offsets[-1])
        cap = need if cap_scale is None else cap_scale(need)
        jobs.append(bpt.Job(graphs[gi][4], first, S, seed, torch.empty(S + 1, dtype=torch.int64, device="cuda"),
                            torch.empty(max(cap, 1), dtype=torch.int32, device="cuda"), cap, colors))
    st, cnt = bpt.bpt_sample_rrr_jobs(jobs)
    torch.cuda.synchronize()
    return st, cnt, jobs, refs


@pytest.mark.parametrize("widest", [64, 1024])
def test_jobs_match_oracle(graphs, widest):
    specs = [(0, 0, 700, 3, 64), (1, 1000, 2000, 9, 16), (2, 5, 1500, 23, 32), (3, 0, 500, 7, 8),
             (0, 0, 0, 1, 64), (1, (1 << 32) - 100, 300, (1 << 40) + 7, widest), (2, 0, 900, 4, 0)]
    announce(f"jobs: {len(specs)} jobs, widest colours {widest}")
    st, cnt, jobs, refs = _run(graphs, specs)
    assert st == bpt.BPT_OK
    for j, ref, spec in zip(jobs, refs, specs):
        assert j.status == bpt.BPT_OK
        assert j.total == int(ref.offsets[-1])
        off = j.d_offsets.cpu().numpy().view(np.uint64)
        ver = j.d_vertices[:j.total].cpu().numpy().view(np.uint32)
        assert_same_sets(off, ver, ref, f"job {spec}")
    assert cnt.samples == sum(s[2] for s in specs)
    assert cnt.members == sum(j.total for j in jobs)
    assert cnt.sample_edges == sum(int(r.te.sum()) for r in refs)


def test_jobs_erange_is_per_job(graphs):
    specs = [(0, 0, 700, 3, 64), (1, 0, 1200, 9, 32), (2, 0, 800, 5, 64)]
    announce("jobs: the middle job's buffer one entry short")
    need = [int(graphs[gi][5].sample(seed, S, first_sample=first, nthreads=8).offsets[-1])
            for gi, first, S, seed, _ in specs]
    caps = iter([need[0], need[1] - 1, need[2]])
    st, _, jobs, refs = _run(graphs, specs, cap_scale=lambda _n: next(caps))
    assert st == bpt.BPT_ERANGE
    assert jobs[1].status == bpt.BPT_ERANGE and jobs[1].total == need[1]
    assert np.array_equal(jobs[1].d_offsets.cpu().numpy().view(np.uint64), refs[1].offsets)
    for i in (0, 2):
        assert jobs[i].status == bpt.BPT_OK
        off = jobs[i].d_offsets.cpu().numpy().view(np.uint64)
        ver = jobs[i].d_vertices[:jobs[i].total].cpu().numpy().view(np.uint32)
        assert_same_sets(off, ver, refs[i], f"job {i} next to a short one")


def test_jobs_invalid(graphs):
    import torch
    g = graphs[0][4]
    off = torch.empty(11, dtype=torch.int64, device="cuda")
    ver = torch.empty(100, dtype=torch.int32, device="cuda")
    for bad in (dict(colors_per_batch=24), dict(n_samples=1 << 35), dict(d_offsets=None)):
        kw = dict(graph=g, first_sample=0, n_samples=10, seed=1, d_offsets=off, d_vertices=ver, capacity=100)
        kw.update(bad)
        with pytest.raises(bpt.BptError) as ei:
            bpt.bpt_sample_rrr_jobs([bpt.Job(**kw)])
        assert ei.value.status == bpt.BPT_EINVAL
    assert bpt.bpt_sample_rrr_jobs([])[0] == bpt.BPT_OK
