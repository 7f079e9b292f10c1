"""The serving loop (bpt_server_*): requests for RRR sets and for
influence-maximization seeds on two graphs, submitted from two threads, are
batched by the server and each gets exactly its oracle result."""

import threading

import numpy as np
import pytest

import graphgen
import oracle
import paper_2311_10201_amd as bpt
from gpu_util import announce, assert_same_sets

pytestmark = pytest.mark.gpu


def test_server_mixed_requests_match_oracle():
    import torch
    graphs = []
    src, dst = graphgen.er_graph(1000, 10_000, seed=42)
    graphs.append((1000, src, dst, graphgen.uniform_prob(len(src), 0.1)))
    src, dst = graphgen.rmat_graph(12, 8, 0.57, 0.19, 0.19, seed=12)
    graphs.append((1 << 12, src, dst, graphgen.wc_prob(1 << 12, dst)))
    handles = [bpt.bpt_create_graph(n, s, d, p) for n, s, d, p in graphs]
    ogs = [oracle.Graph(n, s, d, p) for n, s, d, p in graphs]
    specs = []  # (graph, kind, first, S, seed, k)
    for i in range(14):
        gi = i % 2
        kind = bpt.BPT_REQ_SEEDS if i % 3 == 0 else bpt.BPT_REQ_SAMPLE
        specs.append((gi, kind, 1000 * i, 500 + 137 * i, 5 + i, 10 if kind == bpt.BPT_REQ_SEEDS else 0))
    refs = [ogs[gi].sample(seed, S, first_sample=first, nthreads=8) for gi, _, first, S, seed, _ in specs]
    reqs = []
    for t, ((gi, kind, first, S, seed, k), ref) in enumerate(zip(specs, refs)):
        if kind == bpt.BPT_REQ_SAMPLE:
            cap = int(ref.offsets[-1])
            reqs.append(bpt.Request(kind, handles[gi], first, S, seed, d_offsets=torch.empty(S + 1, dtype=torch.int64,
                                    device="cuda"), d_vertices=torch.empty(cap, dtype=torch.int32, device="cuda"),
                                    capacity=cap, tag=t))
        else:
            reqs.append(bpt.Request(kind, handles[gi], first, S, seed, k=k, tag=t))
    announce(f"server: {len(reqs)} requests from two threads")
    srv = bpt.Server()
    try:
        halves = [reqs[0::2], reqs[1::2]]
        threads = [threading.Thread(target=lambda h=h: [srv.submit(r) for r in h]) for h in halves]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        done = []
        while len(done) < len(reqs):
            r = srv.wait(60.0)
            assert r is not None, "server did not complete the requests"
            done.append(r)
        info = srv.stats()
    finally:
        srv.close()
    assert info["served"] == len(reqs) and 1 <= info["launches"] <= len(reqs)
    assert 0 < info["sample_s"] <= info["busy_s"]
    for r in done:
        gi, kind, first, S, seed, k = specs[r.tag]
        ref = refs[r.tag]
        assert r.status == bpt.BPT_OK, (r.tag, r.status)
        assert r.total == int(ref.offsets[-1])
        assert r.t_submit <= r.t_start <= r.t_done
        if kind == bpt.BPT_REQ_SAMPLE:
            torch.cuda.synchronize()
            off = r.d_offsets.cpu().numpy().view(np.uint64)
            ver = r.d_vertices[:r.total].cpu().numpy().view(np.uint32)
            assert_same_sets(off, ver, ref, f"request {r.tag}")
        else:
            want_seeds, want_gains = oracle.greedy_max_cover(ref.offsets.astype(np.int64),
                                                             ref.members.astype(np.int64), graphs[gi][0], k)
            assert r.seeds[:k].tolist() == want_seeds.tolist()
            assert r.gains[:k].astype(np.int64).tolist() == want_gains.tolist()


def test_server_rejects_bad_requests():
    src, dst = graphgen.er_graph(1000, 10_000, seed=42)
    g = bpt.bpt_create_graph(1000, src, dst, graphgen.uniform_prob(len(src), 0.1))
    srv = bpt.Server()
    try:
        with pytest.raises(bpt.BptError):
            srv.submit(bpt.Request(bpt.BPT_REQ_SEEDS, g, 0, 100, 1, k=0))
        with pytest.raises(bpt.BptError):
            srv.submit(bpt.Request(bpt.BPT_REQ_SAMPLE, g, 0, 100, 1))   # no output buffers
    finally:
        srv.close()
