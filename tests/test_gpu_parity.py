"""GPU parity: the HIP path (through the C ABI) returns exactly the oracle's
RRR sets, for every colour count, the unfused path, every probability layout
and the degenerate cases; its work counters match the oracle's accounting of
Sections 3.1-3.2."""

import os

import numpy as np
import pytest

import graphgen
import oracle
import paper_2311_10201_amd as bpt
from gpu_util import announce, assert_same_sets, sample_device

pytestmark = pytest.mark.gpu

COLORS = [8, 16, 32, 64, 128, 256, 512, 1024]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "er1000_m10000_p0.1_seed42.txt")


@pytest.fixture(scope="module")
def er_case():
    n, m = 1000, 10_000
    src, dst = graphgen.er_graph(n, m, seed=42)
    prob = graphgen.uniform_prob(m, 0.1)
    return n, src, dst, prob


def test_er_host_api_matches_oracle_and_golden(er_case):
    announce("ER n=1000 m=10000 p=0.1 S=64 C=64 host API")
    n, src, dst, prob = er_case
    g = bpt.bpt_create_graph(n, src, dst, prob)
    assert bpt.bpt_graph_info(g) == (n, 10_000, bpt.BPT_PROB_UNIFORM)
    res = bpt.bpt_sample_rrr(g, 64, 64, 42)
    ref = oracle.Graph(n, src, dst, prob).sample(42, 64)
    assert_same_sets(res.offsets, res.vertices, ref, "host API")
    with open(GOLDEN) as f:
        rows = [line.split() for line in f if not line.startswith("#")]
    for i, row in enumerate(rows):
        assert res.set_of(i).tolist() == [int(x) for x in row[1:]]


def test_er_all_colors_and_unfused(er_case):
    n, src, dst, prob = er_case
    g = bpt.bpt_create_graph(n, src, dst, prob)
    og = oracle.Graph(n, src, dst, prob)
    S = 3000  # ragged: not a multiple of any colour count
    ref = og.sample(42, S, nthreads=8)
    te = int(ref.te.sum())
    blocks = oracle.philox_blocks(og, ref)
    for c in COLORS:
        announce(f"ER S={S} C={c}")
        off, ver, cnt = sample_device(g, 0, S, c, 42)
        assert_same_sets(off, ver, ref, f"fused C={c}")
        assert cnt.sample_edges == te
        assert cnt.members == int(ref.offsets[-1])
        assert cnt.edge_accesses == oracle.fused_edge_accesses(og, ref, c)
        assert cnt.frontier_entries == oracle.fused_frontier_entries(ref, c)
        assert cnt.philox_blocks == blocks
        assert cnt.batches == (S + c - 1) // c
    announce(f"ER S={S} unfused")
    off, ver, cnt = sample_device(g, 0, S, 0, 42, flags=bpt.BPT_FLAG_UNFUSED)
    assert_same_sets(off, ver, ref, "unfused")
    assert cnt.edge_accesses == te and cnt.sample_edges == te
    assert cnt.philox_blocks == blocks


@pytest.mark.parametrize("layout", ["uniform", "row", "edge"])
def test_probability_layouts(layout):
    n = 3000
    src, dst = graphgen.rmat_graph(12, 8, 0.57, 0.19, 0.19, seed=5)
    src = src % n
    dst = dst % n
    key = np.unique((src.astype(np.uint64) << np.uint64(32)) | dst)
    src = (key >> np.uint64(32)).astype(np.uint32)
    dst = (key & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    if layout == "uniform":
        prob = graphgen.uniform_prob(len(src), 0.07)
        want = bpt.BPT_PROB_UNIFORM
    elif layout == "row":
        prob = graphgen.wc_prob(n, dst)
        want = bpt.BPT_PROB_ROW
    else:
        prob = (np.random.Generator(np.random.PCG64(3)).random(len(src), dtype=np.float32)
                * np.float32(0.3)).astype(np.float32)
        want = bpt.BPT_PROB_EDGE
    announce(f"layout {layout} n={n} m={len(src)}")
    g = bpt.bpt_create_graph(n, src, dst, prob)
    assert bpt.bpt_graph_info(g)[2] == want
    og = oracle.Graph(n, src, dst, prob)
    S = 2500
    ref = og.sample(7, S, nthreads=8)
    blocks = oracle.philox_blocks(og, ref)
    for c in (64, 256):
        off, ver, cnt = sample_device(g, 0, S, c, 7)
        assert_same_sets(off, ver, ref, f"{layout} C={c}")
        assert cnt.edge_accesses == oracle.fused_edge_accesses(og, ref, c)
        assert cnt.philox_blocks == blocks
    off, ver, cnt = sample_device(g, 0, S, 0, 7, flags=bpt.BPT_FLAG_UNFUSED)
    assert_same_sets(off, ver, ref, f"{layout} unfused")
    assert cnt.philox_blocks == blocks


def test_degenerate_probabilities():
    src, dst = graphgen.rmat_graph(11, 8, 0.57, 0.19, 0.19, seed=9)
    n = 1 << 11
    for p in (0.0, 1.0):
        announce(f"p={p}")
        prob = graphgen.uniform_prob(len(src), p)
        g = bpt.bpt_create_graph(n, src, dst, prob)
        og = oracle.Graph(n, src, dst, prob)
        ref = og.sample(3, 700, nthreads=8)
        blocks = oracle.philox_blocks(og, ref)
        if p == 0.0:
            assert blocks == 0  # rows that can never be live draw no coins
        for c, flags in ((64, 0), (1024, 0), (0, bpt.BPT_FLAG_UNFUSED)):
            off, ver, cnt = sample_device(g, 0, 700, c, 3, flags=flags)
            assert_same_sets(off, ver, ref, f"p={p} C={c} flags={flags}")
            assert cnt.philox_blocks == blocks
        if p == 0.0:
            assert np.all(np.diff(ref.offsets) == 1)


def test_edge_cases_small():
    # no edges at all
    announce("m=0")
    g = bpt.bpt_create_graph(17, [], [], [])
    off, ver, _ = sample_device(g, 0, 100, 64, 1)
    assert np.array_equal(np.diff(off), np.ones(100, dtype=np.uint64))
    ref = oracle.Graph(17, np.array([], np.uint32), np.array([], np.uint32), np.array([], np.float32)).sample(1, 100)
    assert_same_sets(off, ver, ref, "m=0")
    # zero samples
    announce("S=0")
    off, ver, cnt = sample_device(g, 0, 0, 64, 1)
    assert off.tolist() == [0] and len(ver) == 0 and cnt.samples == 0
    res = bpt.bpt_sample_rrr(g, 0, 64, 1)
    assert res.offsets.tolist() == [0]
    # single vertex with a self-loop, one sample
    announce("n=1 self-loop")
    g1 = bpt.bpt_create_graph(1, [0], [0], [1.0])
    off, ver, _ = sample_device(g1, 0, 1, 64, 5)
    assert off.tolist() == [0, 1] and ver.tolist() == [0]


def test_self_loops_and_sample_ranges():
    n = 500
    src, dst, prob = graphgen.random_small_graph(n, 4000, 77, allow_self_loops=True)
    assert np.any(src == dst)
    g = bpt.bpt_create_graph(n, src, dst, prob)
    og = oracle.Graph(n, src, dst, prob)
    seed = (1 << 63) + 12345  # high key word in use
    first = (1 << 32) - 300   # ids cross 2^32
    ref = og.sample(seed, 1000, first_sample=first, nthreads=8)
    announce("ranges crossing 2^32")
    off, ver, _ = sample_device(g, first, 1000, 128, seed)
    assert_same_sets(off, ver, ref, "first_sample")
    # two shards concatenate to the whole
    o1, v1, _ = sample_device(g, first, 333, 64, seed)
    o2, v2, _ = sample_device(g, first + 333, 667, 512, seed)
    assert np.array_equal(np.concatenate([v1, v2]), ref.members)
    assert np.array_equal(np.concatenate([o1[:-1], o2 + o1[-1]]), ref.offsets)


def test_erange_and_repeatability(er_case):
    n, src, dst, prob = er_case
    g = bpt.bpt_create_graph(n, src, dst, prob)
    import torch
    S = 500
    off = torch.empty(S + 1, dtype=torch.int64, device="cuda")
    vert = torch.empty(8, dtype=torch.int32, device="cuda")
    announce("ERANGE")
    st, total, _ = bpt.bpt_sample_rrr_device(g, 0, S, 64, 9, 0, None, off, vert, 8)
    assert st == bpt.BPT_ERANGE and total > 8
    # the retry with a large enough buffer re-assembles the kept sets without traversing ...
    a = sample_device(g, 0, S, 64, 9)
    assert a[2].traversal_ns == 0 and int(a[0][-1]) == total
    # ... while every later call traverses again and returns the same sets
    for _ in range(3):
        b = sample_device(g, 0, S, 64, 9)
        assert b[2].traversal_ns > 0
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_erange_retry_after_other_launches(er_case):
    """A retry after BPT_ERANGE returns the oracle's sets even when a
    multi-job launch and a tuning run used the graph's cached workspaces in
    between (they overwrite the sets the failed call left there), and the
    tuning trial is not served from those sets either."""
    import torch
    n, src, dst, prob = er_case
    g = bpt.bpt_create_graph(n, src, dst, prob)
    og = oracle.Graph(n, src, dst, prob)
    S, seed = 500, 9
    ref = og.sample(seed, S, nthreads=8)
    off = torch.empty(S + 1, dtype=torch.int64, device="cuda")
    vert = torch.empty(8, dtype=torch.int32, device="cuda")
    announce("ERANGE, then a jobs call on the same graph")
    st, total, _ = bpt.bpt_sample_rrr_device(g, 0, S, 64, seed, 0, None, off, vert, 8)
    assert st == bpt.BPT_ERANGE and total == int(ref.offsets[-1])
    other = og.sample(3, 700, first_sample=40, nthreads=8)
    job = bpt.Job(g, 40, 700, 3, torch.empty(701, dtype=torch.int64, device="cuda"),
                  torch.empty(int(other.offsets[-1]), dtype=torch.int32, device="cuda"), int(other.offsets[-1]), 64)
    st, _ = bpt.bpt_sample_rrr_jobs([job])
    assert st == bpt.BPT_OK
    announce("retry after the jobs call")
    a = sample_device(g, 0, S, 64, seed)
    assert_same_sets(a[0], a[1], ref, "retry after a jobs call")
    assert a[2].traversal_ns > 0
    announce("ERANGE, then a tuning run")
    st, _, _ = bpt.bpt_sample_rrr_device(g, 0, S, 64, seed, 0, None, off, vert, 8)
    assert st == bpt.BPT_ERANGE
    assert bpt.bpt_tune_colors(g, S, seed) in (8, 16, 32, 64, 128, 256, 512, 1024)
    a = sample_device(g, 0, S, 64, seed)
    assert_same_sets(a[0], a[1], ref, "retry after tuning")


def test_invalid_sampling_arguments(er_case):
    n, src, dst, prob = er_case
    g = bpt.bpt_create_graph(n, src, dst, prob)
    for c in (1, 4, 24, 96, 2048):
        with pytest.raises(bpt.BptError) as ei:
            bpt.bpt_sample_rrr(g, 10, c, 1)
        assert ei.value.status == bpt.BPT_EINVAL
    with pytest.raises(bpt.BptError):
        bpt.bpt_sample_rrr(g, 1 << 34, 64, 1)


def test_default_colors_fill_the_gpu(er_case):
    """colors_per_batch = 0: 64 colours when there are batches for every
    resident workgroup, narrower batches for small jobs; the sets equal the
    oracle's either way."""
    n, src, dst, prob = er_case
    g = bpt.bpt_create_graph(n, src, dst, prob)
    assert bpt.bpt_default_colors(g, 10_000_000) == 64
    assert bpt.bpt_default_colors(g, 100) == 8
    widths = [bpt.bpt_default_colors(g, s) for s in (100, 3_000, 10_000, 30_000, 100_000, 1_000_000)]
    assert widths == sorted(widths) and set(widths) <= {8, 16, 32, 64}
    S = 3000
    ref = oracle.Graph(n, src, dst, prob).sample(5, S, nthreads=8)
    announce(f"default colours S={S}: {bpt.bpt_default_colors(g, S)}")
    off, ver, cnt = sample_device(g, 0, S, 0, 5)
    assert_same_sets(off, ver, ref, "default colours")
    c = bpt.bpt_default_colors(g, S)
    assert cnt.batches == (S + c - 1) // c


def test_tuned_colors_are_remembered(er_case):
    """bpt_tune_colors measures the widths and the chosen one becomes the
    default for jobs of that size range on that graph only; the sets stay the
    oracle's."""
    n, src, dst, prob = er_case
    g = bpt.bpt_create_graph(n, src, dst, prob)
    other = bpt.bpt_create_graph(n, src, dst, prob)
    before = bpt.bpt_default_colors(other, 3000)
    announce("tune colours S=3000")
    c = bpt.bpt_tune_colors(g, 3000, 5)
    assert c in (8, 16, 32, 64, 128, 256, 512, 1024)
    assert bpt.bpt_default_colors(g, 3000) == c
    assert bpt.bpt_default_colors(g, 2048) == c and bpt.bpt_default_colors(g, 4095) == c
    assert bpt.bpt_default_colors(other, 3000) == before
    S = 2500
    ref = oracle.Graph(n, src, dst, prob).sample(11, S, nthreads=8)
    off, ver, cnt = sample_device(g, 0, S, 0, 11)
    assert_same_sets(off, ver, ref, "tuned colours")
    assert cnt.batches == (S + c - 1) // c
    with pytest.raises(bpt.BptError):
        bpt.bpt_tune_colors(g, 0, 5)


def hub_graph(n=20_000, hubs=12, hub_in=9_000, hub_out=1_500, m_rand=60_000, seed=17):
    """Random graph plus hub vertices with thousands of in-edges (rows that the
    fused kernel splits into many work items over a workgroup's lanes) and many
    out-edges (so samples reach them often)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    src = [rng.integers(0, n, m_rand)]
    dst = [rng.integers(0, n, m_rand)]
    for h in range(hubs):
        src.append(rng.integers(0, n, hub_in))
        dst.append(np.full(hub_in, h))
        src.append(np.full(hub_out, h))
        dst.append(rng.integers(0, n, hub_out))
    key = np.unique((np.concatenate(src).astype(np.uint64) << np.uint64(32)) | np.concatenate(dst).astype(np.uint64))
    s = (key >> np.uint64(32)).astype(np.uint32)
    d = (key & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    keep = s != d
    return n, s[keep], d[keep]


@pytest.mark.parametrize("layout", ["uniform", "row", "edge"])
def test_hub_rows_split_into_work_items(layout):
    n, src, dst = hub_graph()
    if layout == "uniform":
        prob = graphgen.uniform_prob(len(src), 0.02)
    elif layout == "row":
        prob = graphgen.wc_prob(n, dst)
    else:
        prob = (np.random.Generator(np.random.PCG64(8)).random(len(src), dtype=np.float32)
                * np.float32(0.05)).astype(np.float32)
    announce(f"hub graph layout={layout} n={n} m={len(src)}")
    g = bpt.bpt_create_graph(n, src, dst, prob)
    og = oracle.Graph(n, src, dst, prob)
    S = 3000
    ref = og.sample(23, S, nthreads=8)
    indeg = og.indegree()
    hub_expansions = int(np.sum(indeg[ref.members.astype(np.int64)] >= 4096))
    assert hub_expansions > 100  # rows of over a thousand 8-quad items are expanded
    blocks = oracle.philox_blocks(og, ref)
    for c in COLORS:
        off, ver, cnt = sample_device(g, 0, S, c, 23)
        assert_same_sets(off, ver, ref, f"hub {layout} C={c}")
        assert cnt.edge_accesses == oracle.fused_edge_accesses(og, ref, c)
        assert cnt.sample_edges == int(ref.te.sum())
        assert cnt.philox_blocks == blocks
    off, ver, _ = sample_device(g, 0, S, 0, 23, flags=bpt.BPT_FLAG_UNFUSED)
    assert_same_sets(off, ver, ref, f"hub {layout} unfused")


@pytest.mark.parametrize("block", ["128", "512", "1024"])
def test_workgroup_shapes(block, monkeypatch):
    """Every workgroup-size instantiation (128, 512 and 1024 threads besides
    the default; sizes a colour count does not have fall back to it) returns
    the oracle's sets, hub rows and every colour count included."""
    n, src, dst = hub_graph()
    prob = graphgen.wc_prob(n, dst)
    og = oracle.Graph(n, src, dst, prob)
    S = 2000
    ref = og.sample(31, S, nthreads=8)
    monkeypatch.setenv("BPT_FUSED_BLOCK", block)
    g = bpt.bpt_create_graph(n, src, dst, prob)
    for c in COLORS:
        announce(f"hub graph block={block} C={c}")
        off, ver, cnt = sample_device(g, 0, S, c, 31)
        assert_same_sets(off, ver, ref, f"block={block} C={c}")
        assert cnt.edge_accesses == oracle.fused_edge_accesses(og, ref, c)


@pytest.mark.parametrize("force", ["0", "1"])
def test_visited_read_first(force, monkeypatch):
    """Discoveries with and without the read of visited[u] before the
    fetch-or (BPT_READ_FIRST forces the per-job choice) return the oracle's
    sets and work counters, on a graph whose colours meet at hubs so that many
    live coins find their colour already there, under both colour schedules."""
    n, src, dst = hub_graph(n=6_000, hubs=6, hub_in=5_000, hub_out=800, m_rand=30_000, seed=31)
    prob = graphgen.uniform_prob(len(src), 0.05)
    og = oracle.Graph(n, src, dst, prob)
    S = 1200
    ref = og.sample(41, S, nthreads=8)
    blocks = oracle.philox_blocks(og, ref)
    monkeypatch.setenv("BPT_READ_FIRST", force)
    g = bpt.bpt_create_graph(n, src, dst, prob)
    for mode in ("never", "always"):
        monkeypatch.setenv("BPT_GATHER", mode)
        for c in (8, 64, 256):
            announce(f"BPT_READ_FIRST={force} BPT_GATHER={mode} C={c}")
            off, ver, cnt = sample_device(g, 0, S, c, 41)
            assert_same_sets(off, ver, ref, f"read first {force} {mode} C={c}")
            assert cnt.edge_accesses == oracle.fused_edge_accesses(og, ref, c)
            assert cnt.frontier_entries == oracle.fused_frontier_entries(ref, c)
            assert cnt.philox_blocks == blocks


@pytest.mark.parametrize("mode", ["never", "always"])
@pytest.mark.parametrize("layout", ["uniform", "edge"])
def test_colour_schedules(mode, layout, monkeypatch):
    """Both colour schedules of the fused expansion (one atomic per live coin,
    or live colours gathered per edge into one mask atomic) return the
    oracle's sets and edge-access counts, at a probability where entries carry
    many colours."""
    n, src, dst = hub_graph(n=6_000, hubs=6, hub_in=5_000, hub_out=800, m_rand=30_000, seed=29)
    if layout == "uniform":
        prob = graphgen.uniform_prob(len(src), 0.2)
    else:
        prob = (np.random.Generator(np.random.PCG64(4)).random(len(src), dtype=np.float32)
                * np.float32(0.4)).astype(np.float32)
    og = oracle.Graph(n, src, dst, prob)
    S = 1500
    ref = og.sample(37, S, nthreads=8)
    blocks = oracle.philox_blocks(og, ref)
    monkeypatch.setenv("BPT_GATHER", mode)
    g = bpt.bpt_create_graph(n, src, dst, prob)
    for c in COLORS:
        announce(f"colour schedule {mode} layout={layout} C={c}")
        off, ver, cnt = sample_device(g, 0, S, c, 37)
        assert_same_sets(off, ver, ref, f"{mode} {layout} C={c}")
        assert cnt.edge_accesses == oracle.fused_edge_accesses(og, ref, c)
        assert cnt.philox_blocks == blocks
        assert cnt.live_coins <= cnt.philox_blocks * 4


def test_workgroup_size_follows_set_size_history(er_case, monkeypatch):
    """A graph without set-size history runs 512-thread workgroups; once its
    sets are known to be small it runs 256-thread ones (twice the batches in
    flight), unless BPT_FUSED_BLOCK forces a size.  Every call returns the
    oracle's sets."""
    n, src, dst, prob = er_case
    og = oracle.Graph(n, src, dst, prob)
    S, seed = 3000, 13
    ref = og.sample(seed, S, nthreads=8)
    monkeypatch.delenv("BPT_FUSED_BLOCK", raising=False)
    g = bpt.bpt_create_graph(n, src, dst, prob)
    sizes = []
    for i in range(3):
        announce(f"set-size history call {i}")
        off, ver, cnt = sample_device(g, 0, S, 64, seed)
        assert_same_sets(off, ver, ref, f"call {i}")
        sizes.append(cnt.workgroup_size)
    assert sizes == [512, 256, 256]
    monkeypatch.setenv("BPT_FUSED_BLOCK", "512")
    off, ver, cnt = sample_device(g, 0, S, 64, seed)
    assert_same_sets(off, ver, ref, "forced 512")
    assert cnt.workgroup_size == 512
