"""GPU parity of the influence-maximization query (bpt_max_cover): the greedy
seeds and per-step gains equal the oracle's greedy maximum coverage, exactly,
on RRR sets sampled by the library; malformed inputs are rejected."""

import numpy as np
import pytest

import graphgen
import oracle
import paper_2311_10201_amd as bpt
from gpu_util import announce, sample_device

pytestmark = pytest.mark.gpu


def _device_sets(g, S, seed, colors=64):
    import torch
    off, ver, _ = sample_device(g, 0, S, colors, seed)
    return (torch.from_numpy(off.view(np.int64).copy()).cuda(),
            torch.from_numpy(ver.view(np.int32).copy()).cuda(), off, ver)


@pytest.mark.parametrize("case", ["er", "rmat-wc", "rmat-dense"])
def test_max_cover_matches_oracle(case):
    if case == "er":
        n = 1000
        src, dst = graphgen.er_graph(n, 10_000, seed=42)
        prob, S, k = graphgen.uniform_prob(len(src), 0.1), 3000, 50
    elif case == "rmat-wc":
        n = 1 << 16
        src, dst = graphgen.rmat_graph(16, 16, 0.57, 0.19, 0.19, seed=16)
        prob, S, k = graphgen.wc_prob(n, dst), 20_000, 100
    else:
        n = 1 << 12
        src, dst = graphgen.rmat_graph(12, 16, 0.57, 0.19, 0.19, seed=3)
        prob, S, k = graphgen.uniform_prob(len(src), 0.2), 2000, 64
    announce(f"max cover {case} S={S} k={k}")
    g = bpt.bpt_create_graph(n, src, dst, prob)
    d_off, d_ver, off, ver = _device_sets(g, S, 7)
    seeds, gains = bpt.bpt_max_cover(d_off, d_ver, S, n, k)
    want_seeds, want_gains = oracle.greedy_max_cover(off.astype(np.int64), ver.astype(np.int64), n, k)
    assert seeds.tolist() == want_seeds.tolist()
    assert gains.astype(np.int64).tolist() == want_gains.tolist()
    # the oracle's own sets give the same answer (the sets are the oracle's)
    ref = oracle.Graph(n, src, dst, prob).sample(7, S, nthreads=8)
    assert np.array_equal(ref.members, ver)


def test_max_cover_exhausts_and_breaks_ties():
    import torch
    # sets {1,3}, {1,3}, {4}: 1 beats 3 on the tie, then 4, then the lowest unchosen ids with gain 0
    off = torch.tensor([0, 2, 4, 5], dtype=torch.int64, device="cuda")
    ver = torch.tensor([1, 3, 1, 3, 4], dtype=torch.int32, device="cuda")
    seeds, gains = bpt.bpt_max_cover(off, ver, 3, 6, 4)
    assert seeds.tolist() == [1, 4, 0, 2] and gains.tolist() == [2, 1, 0, 0]


def test_max_cover_rejects_bad_input():
    import torch
    ver = torch.tensor([1, 3, 1, 9, 4], dtype=torch.int32, device="cuda")
    off = torch.tensor([0, 2, 4, 5], dtype=torch.int64, device="cuda")
    with pytest.raises(bpt.BptError) as ei:      # member 9 >= n = 6
        bpt.bpt_max_cover(off, ver, 3, 6, 2)
    assert ei.value.status == bpt.BPT_EINVAL
    ver_ok = torch.tensor([1, 3, 1, 3, 4], dtype=torch.int32, device="cuda")
    bad_off = torch.tensor([0, 4, 2, 5], dtype=torch.int64, device="cuda")   # not non-decreasing
    with pytest.raises(bpt.BptError):
        bpt.bpt_max_cover(bad_off, ver_ok, 3, 6, 2)
    with pytest.raises(bpt.BptError):             # k > n
        bpt.bpt_max_cover(off, ver_ok, 3, 6, 7)
