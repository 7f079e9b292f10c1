"""Helpers of the GPU parity tests: run libbpt through its C ABI and compare
with the CPU oracle."""

import sys

import numpy as np

import oracle
import paper_2311_10201_amd as bpt


def announce(msg: str) -> None:
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def sample_device(g, first, n_samples, colors, seed, flags=0, capacity=None):
    """bpt_sample_rrr_device into torch buffers; returns (offsets, vertices, counters)."""
    import torch
    off = torch.empty(n_samples + 1, dtype=torch.int64, device="cuda")
    cap = capacity if capacity is not None else max(1024, 64 * n_samples)
    vert = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
    st, total, cnt = bpt.bpt_sample_rrr_device(g, first, n_samples, colors, seed, flags, None, off, vert, cap)
    if st == bpt.BPT_ERANGE:
        vert = torch.empty(max(total, 1), dtype=torch.int32, device="cuda")
        st, total2, cnt = bpt.bpt_sample_rrr_device(g, first, n_samples, colors, seed, flags, None, off, vert,
                                                    total)
        assert st == bpt.BPT_OK and total2 == total
    torch.cuda.synchronize()
    offsets = off.cpu().numpy().view(np.uint64)
    vertices = vert[:total].cpu().numpy().view(np.uint32)
    assert int(offsets[-1]) == total
    return offsets, vertices, cnt


def assert_same_sets(offsets, vertices, ref: oracle.RRRSets, what=""):
    """Element-by-element equality with the oracle's CSR."""
    assert len(offsets) == len(ref.offsets), what
    if not np.array_equal(offsets, ref.offsets):
        i = int(np.nonzero(offsets != ref.offsets)[0][0])
        raise AssertionError(f"{what}: offsets differ first at {i}: {offsets[i]} vs {ref.offsets[i]}")
    if not np.array_equal(vertices, ref.members):
        j = int(np.nonzero(vertices != ref.members)[0][0])
        s = int(np.searchsorted(ref.offsets, j, side="right") - 1)
        raise AssertionError(f"{what}: members differ first in sample index {s}")
