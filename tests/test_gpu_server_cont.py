"""Continuous batching in the serving loop: a request submitted while another
request's launches are on the GPU joins the next launch, finishes first, and
both get exactly the oracle's sets."""

import time

import numpy as np
import pytest

import graphgen
import oracle
import paper_2311_10201_amd as bpt
from gpu_util import announce, assert_same_sets

pytestmark = pytest.mark.gpu


def test_request_joins_running_work():
    import torch
    src, dst = graphgen.rmat_graph(16, 16, 0.57, 0.19, 0.19, seed=16)
    n = 1 << 16
    prob = graphgen.wc_prob(n, dst)
    g = bpt.bpt_create_graph(n, src, dst, prob)
    og = oracle.Graph(n, src, dst, prob)
    big_S, small_S = 2_000_000, 3_000
    ids = np.arange(0, big_S, 997, dtype=np.uint64)
    ref_big = og.sample_ids(11, ids, nthreads=8)
    ref_small = og.sample(5, small_S, first_sample=123, nthreads=8)
    # warm the graph's set-size estimate so the big request's launches are sized
    warm = bpt.bpt_sample_rrr(g, 20_000, 0, 1)
    cap_big = int(warm.offsets[-1] / 20_000 * big_S * 1.5) + (1 << 20)
    del warm
    big = bpt.Request(bpt.BPT_REQ_SAMPLE, g, 0, big_S, 11,
                      d_offsets=torch.empty(big_S + 1, dtype=torch.int64, device="cuda"),
                      d_vertices=torch.empty(cap_big, dtype=torch.int32, device="cuda"), capacity=cap_big, tag=1)
    cap_small = int(ref_small.offsets[-1])
    small = bpt.Request(bpt.BPT_REQ_SAMPLE, g, 123, small_S, 5,
                        d_offsets=torch.empty(small_S + 1, dtype=torch.int64, device="cuda"),
                        d_vertices=torch.empty(cap_small, dtype=torch.int32, device="cuda"), capacity=cap_small, tag=2)
    seeds = bpt.Request(bpt.BPT_REQ_SEEDS, g, 777, 4_000, 9, k=20, tag=3)
    announce(f"server: {big_S} samples, then {small_S} samples and a seed request while it runs")
    srv = bpt.Server()
    try:
        srv.submit(big)
        time.sleep(0.005)  # the big request's first launches are on the GPU
        srv.submit(small)
        srv.submit(seeds)
        done = {}
        while len(done) < 3:
            r = srv.wait(120.0)
            assert r is not None, "server did not complete the requests"
            done[r.tag] = r
        info = srv.stats()
    finally:
        srv.close()
    assert all(r.status == bpt.BPT_OK for r in done.values()), [(r.tag, r.status) for r in done.values()]
    # the small requests were admitted while the big one ran and finished before it
    assert small.t_start < big.t_done and small.t_done < big.t_done
    assert seeds.t_done < big.t_done
    assert info["launches"] >= 3
    # a lane keeps one slot per resident 512-thread workgroup, although this
    # graph's small sets give its own calls 256-thread workgroups
    assert info["lane_slots"] == 2 * torch.cuda.get_device_properties(0).multi_processor_count
    torch.cuda.synchronize()
    off = small.d_offsets.cpu().numpy().view(np.uint64)
    ver = small.d_vertices[:small.total].cpu().numpy().view(np.uint32)
    assert_same_sets(off, ver, ref_small, "small request")
    off = big.d_offsets.cpu().numpy().view(np.uint64)
    assert int(off[-1]) == big.total
    sizes = off[ids.astype(np.int64) + 1] - off[ids.astype(np.int64)]
    assert np.array_equal(sizes, np.diff(ref_big.offsets))
    idx = torch.as_tensor(ids.astype(np.int64), device="cuda")
    lo = big.d_offsets[idx]
    lens = big.d_offsets[idx + 1] - lo
    pos = torch.repeat_interleave(lo - (torch.cumsum(lens, 0) - lens), lens) + torch.arange(int(lens.sum()), device="cuda")
    assert np.array_equal(big.d_vertices[pos].cpu().numpy().view(np.uint32), ref_big.members)
    ref_seeds = og.sample(9, 4_000, first_sample=777, nthreads=8)
    want_seeds, want_gains = oracle.greedy_max_cover(ref_seeds.offsets.astype(np.int64),
                                                     ref_seeds.members.astype(np.int64), n, 20)
    assert seeds.seeds[:20].tolist() == want_seeds.tolist()
    assert seeds.gains[:20].astype(np.int64).tolist() == want_gains.tolist()
    bpt.bpt_free(g)
